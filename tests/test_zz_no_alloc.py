"""The allocation-free warm-start entry point against the allocating one.

glbm_cnn_apply_noalloc stages rho - 1 and the velocity in the library's static
per-GPU scratch instead of a buffer allocated per call; its result must be the
state glbm_cnn_apply writes, bit for bit.  Two calls in a row, the second on a
smaller instance (the scratch keeps the first call's contents), then the first
instance again; an instance larger than the scratch is rejected on the host.
"""
import numpy as np
import pytest

from helpers import random_case

pytestmark = pytest.mark.gpu


def _solver(g, store, shapes, cases):
    descs = [g.make_desc(sh, store=g.STORE_NAMES[store], g=(1e-6, 0, 0), check_every=100) for sh in shapes]
    s = g.Solver(descs, [c[0] for c in cases])
    for i, c in enumerate(cases):
        s.set_local_perm(c[1][:255], c[2][:255], inst=i)
    return s


@pytest.mark.parametrize("store", ["f32", "f32loc", "f16loc", "f64"])
def test_noalloc_apply_matches_apply(gpu, store):
    import torch
    g = gpu
    shapes = [(256, 320), (96, 128)]
    cases = [random_case(sh, seed=60 + i, wall_frac=0.05) for i, sh in enumerate(shapes)]
    rng = np.random.default_rng(17)
    ys = [torch.from_numpy(rng.standard_normal(sh[0] * sh[1] * 4).astype(np.float32)).cuda() for sh in shapes]
    rs, us = 3e-5, 1e-6
    states = {}
    for name, fn in (("apply", g.glbm_cnn_apply), ("noalloc", g.glbm_cnn_apply_noalloc)):
        print("case store=%s entry=%s" % (store, name), flush=True)
        s = _solver(g, store, shapes, cases)
        try:
            fn(s.ctx, 0, ys[0].data_ptr(), rs, us)
            p0 = s.populations(0).copy()
            fn(s.ctx, 1, ys[1].data_ptr(), rs, us)
            p1 = s.populations(1).copy()
            fn(s.ctx, 0, ys[0].data_ptr(), 2 * rs, us)
            p2 = s.populations(0).copy()
            s.step(100)
            r, _ = s.residual()
        finally:
            s.close()
        states[name] = (p0, p1, p2, r)
    a, b = states["apply"], states["noalloc"]
    for k in range(3):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a[3], b[3])
    assert not np.array_equal(a[0], a[2])


def test_noalloc_rejects_oversize_instance(gpu):
    import torch
    g = gpu
    shape = (1025, 1024)
    assert shape[0] * shape[1] > g.GLBM_NOALLOC_MAX_NODES
    cls = np.zeros(shape, np.uint8)
    s = g.Solver([g.make_desc(shape, store=g.GLBM_STORE_F32)], [cls])
    try:
        s.set_local_perm(np.ones(1), np.full(1, np.inf))
        y = torch.zeros(16, dtype=torch.float32, device="cuda")
        with pytest.raises(g.GlbmError) as ei:
            g.glbm_cnn_apply_noalloc(s.ctx, 0, y.data_ptr(), 1e-5, 1e-6)
        assert ei.value.code == g.GLBM_EINVAL and "scratch" in str(ei.value)
    finally:
        s.close()
