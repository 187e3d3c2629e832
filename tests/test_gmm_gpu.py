"""Batched EM fit of pore-size mixtures on the GPU (glbm_gmm_fit) against the oracle's
EM (Sec. 2.2, Eq. 20-24), and the pipeline that feeds the class table from a
measured pore-size distribution."""
import math

import numpy as np
import pytest

import shale_inputs as si
from oracle import gmm

pytestmark = pytest.mark.gpu


def _fit_gpu(g, sets, starts, iters, tol=0.0):
    import torch
    offs = np.concatenate([[0], np.cumsum([len(x) for x in sets])]).astype(np.int64)
    xd = torch.from_numpy(np.concatenate(sets)).cuda()
    phi, mu, var = (np.array([s[i] for s in starts]) for i in range(3))
    out = g.glbm_gmm_fit(offs, xd.data_ptr(), phi, mu, var, iters, tol)
    torch.cuda.synchronize()
    return out


def test_gmm_batch_matches_oracle(gpu):
    """Uneven batch of sets (Tab. 3 mixture, lognormal pore radii in ln r, three
    components, a single Gaussian; sizes from 3 to 300k samples, chunk tails), fixed
    iteration counts: parameters within 1e-11 relative of the oracle, log-likelihood
    within 1e-11 (FP64 with a different summation order)."""
    g = gpu
    sets, starts, ks = [], [], []
    sets.append(si.mixture_samples(11, 300000))
    starts.append(([0.5, 0.5], [8.0, 25.0], [4.0, 25.0]))
    sets.append(np.log(si.pore_radius_samples(12, 50001)))
    starts.append(([0.5, 0.5], [math.log(3e-9), math.log(30e-9)], [0.5, 0.5]))
    sets.append(si.mixture_samples(13, 4097, ((0.0, 1.0, 0.2), (5.0, 1.5, 0.5), (12.0, 0.7, 0.3))))
    starts.append(([0.3, 0.3, 0.4], [1.0, 4.0, 10.0], [2.0, 2.0, 2.0]))
    sets.append(si.mixture_samples(14, 3, ((2.0, 1.0, 1.0),)))
    starts.append(([1.0], [0.0], [1.0]))
    for k in (1, 2, 3):
        idx = [i for i, s in enumerate(starts) if len(s[0]) == k]
        if not idx:
            continue
        print("case k=%d sets %s" % (k, [len(sets[i]) for i in idx]), flush=True)
        iters = 40
        phi, mu, var, ll, it = _fit_gpu(g, [sets[i] for i in idx], [starts[i] for i in idx], iters)
        for r, i in enumerate(idx):
            p0, m0, v0, hist = gmm.fit(sets[i], *starts[i], iters)
            assert it[r] == iters
            assert np.allclose(phi[r], p0, rtol=1e-11, atol=1e-14)
            assert np.allclose(mu[r], m0, rtol=1e-11, atol=1e-14)
            assert np.allclose(var[r], v0, rtol=1e-10, atol=1e-14)
            assert abs(ll[r] - hist[-1]) <= 1e-11 * abs(hist[-1]) + 1e-12
            print("  set %d (%d samples): mu %s, loglik %.12e vs %.12e" % (i, len(sets[i]), mu[r], ll[r], hist[-1]))


def test_gmm_tolerance_stop_and_batch_independence(gpu):
    """With tol > 0 each set stops on its own; a set's result does not depend on what
    else is in the batch (bitwise)."""
    g = gpu
    a = si.mixture_samples(21, 20000)
    b = si.mixture_samples(22, 70000)
    st = ([0.5, 0.5], [8.0, 25.0], [4.0, 25.0])
    pa, ma, va, la, ia = _fit_gpu(g, [a], [st], 2000, tol=1e-12)
    pb, mb, vb, lb, ib = _fit_gpu(g, [b, a], [st, st], 2000, tol=1e-12)
    assert 2 <= ia[0] < 2000
    assert np.array_equal(pa[0], pb[1]) and np.array_equal(ma[0], mb[1]) and np.array_equal(va[0], vb[1])
    assert ia[0] == ib[1] and la[0] == lb[1]
    # the stopped fit agrees with the oracle run for the same number of iterations
    p0, m0, v0, _ = gmm.fit(a, *st, int(ia[0]))
    assert np.allclose(ma[0], m0, rtol=1e-11)


def test_class_table_from_measured_pore_sizes(gpu):
    """A synthetic measured PSD of both phases (lognormal modes, medians 5 / 20 nm,
    sigma 0.5 in ln r) is fitted in ln r with two components; the smaller mode is the
    organic matter.  Its radius bins and class table reproduce those of the true modes
    to the sampling error (medians within 3 %, K within 8 %)."""
    import torch
    g = gpu
    r = si.pore_radius_samples(31, 200000)
    lr = np.log(r)
    phi, mu, var, ll, it = _fit_gpu(g, [lr], [([0.5, 0.5], [math.log(3e-9), math.log(30e-9)], [0.5, 0.5])], 500,
                                    tol=1e-13)
    o = np.argsort(mu[0])
    om, iom = o[0], o[1]
    r_om = g.glbm_radius_bins(mu[0][om], math.sqrt(var[0][om]))
    r_iom = g.glbm_radius_bins(mu[0][iom], math.sqrt(var[0][iom]))
    inst = si.shale128()
    prm = g.gas_params(inst)
    eps_fit, k_fit = g.glbm_class_table(prm, r_iom, r_om)
    eps_true, k_true = g.glbm_class_table(prm, *inst.radii())
    assert abs(math.exp(mu[0][om]) / 5e-9 - 1) < 0.03 and abs(math.exp(mu[0][iom]) / 20e-9 - 1) < 0.03
    m = np.isfinite(k_true)
    rel = np.abs(k_fit[m] / k_true[m] - 1)
    print("fitted medians %.3e / %.3e, sigma %.3f / %.3f, max K rel diff %.3f" % (
        math.exp(mu[0][om]), math.exp(mu[0][iom]), math.sqrt(var[0][om]), math.sqrt(var[0][iom]), rel.max()))
    assert rel.max() < 0.08
    assert np.array_equal(eps_fit, eps_true)


def test_gmm_vanishing_component_keeps_its_parameters(gpu):
    """Degenerate case: a component so far from every sample that its responsibilities
    underflow to zero.  After one iteration the other component is the plain sample
    mean and (population) variance with Phi = 1, and the vanished one keeps its mean and
    variance with Phi = 0; further iterations leave both unchanged."""
    g = gpu
    x = np.random.default_rng(5).standard_normal(10000) * 0.7 + 2.0
    st = ([0.5, 0.5], [0.0, 1e6], [1.0, 1.0])
    for iters in (1, 5):
        print("case iters=%d" % iters, flush=True)
        phi, mu, var, ll, it = _fit_gpu(g, [x], [st], iters)
        assert it[0] == iters
        assert phi[0][0] == 1.0 and phi[0][1] == 0.0
        assert abs(mu[0][0] - x.mean()) <= 1e-12 * abs(x.mean())
        assert abs(var[0][0] - x.var()) <= 1e-12 * x.var()
        assert mu[0][1] == 1e6 and var[0][1] == 1.0



def test_gmm_two_components_edge_arguments(gpu):
    """k = 2 sets that drive the pass's own exponential to its ends, at ragged sizes:
    components 200 standard deviations apart (the smaller term underflows to 0 and each
    responsibility is 0 or 1), components 40 apart (the exponent's argument crosses the
    -745 cutoff inside the data), and identical starting components (the exponential of
    0 must be exactly 1, every sum of the two terms is 2, and EM keeps the two
    components equal).  Parameters and log-likelihood against the oracle within the
    batch test's tolerances."""
    g = gpu
    sets = [si.mixture_samples(21, 20001, ((0.0, 1.0, 0.5), (200.0, 1.0, 0.5))),
            si.mixture_samples(22, 4099, ((0.0, 1.0, 0.5), (40.0, 1.0, 0.5))),
            si.mixture_samples(23, 12345)]
    starts = [([0.5, 0.5], [0.0, 200.0], [1.0, 1.0]),
              ([0.5, 0.5], [0.0, 40.0], [1.0, 1.0]),
              ([0.5, 0.5], [12.0, 12.0], [30.0, 30.0])]
    a = [np.abs(0.5 * ((x - m[0]) ** 2 - (x - m[1]) ** 2)) for x, (_, m, _) in zip(sets, starts)]
    assert a[0].min() > 745.0 and a[1].min() < 745.0 < a[1].max() and a[2].max() == 0.0
    iters = 20
    print("case k=2 edge sets %s" % [len(x) for x in sets], flush=True)
    phi, mu, var, ll, it = _fit_gpu(g, sets, starts, iters)
    for r in range(len(sets)):
        p0, m0, v0, hist = gmm.fit(sets[r], *starts[r], iters)
        assert it[r] == iters
        assert np.allclose(phi[r], p0, rtol=1e-11, atol=1e-14)
        assert np.allclose(mu[r], m0, rtol=1e-11, atol=1e-14)
        assert np.allclose(var[r], v0, rtol=1e-10, atol=1e-14)
        assert abs(ll[r] - hist[-1]) <= 1e-11 * abs(hist[-1]) + 1e-12
        print("  set %d (%d samples): phi %s mu %s var %s" % (r, len(sets[r]), phi[r], mu[r], var[r]))
    assert phi[2][0] == phi[2][1] and mu[2][0] == mu[2][1] and var[2][0] == var[2][1]



def test_gmm_bench_size_sampled_sets(gpu):
    """The benchmark's workload in its launch configuration: 64 sets of 2^20 log pore
    radii (seeds 9000 + k, two lognormal modes), two components from the same start, all
    sets fitted in one call.  Sets are independent, so four sampled sets (first, last and
    two between) are checked against the oracle fitted on that set alone, after three
    iterations, within the batch test's tolerances."""
    import torch
    g = gpu
    n_sets, m, iters = 64, 1 << 20, 3
    xs = [np.log(si.pore_radius_samples(9000 + k, m)) for k in range(n_sets)]
    start = ([0.5, 0.5], [math.log(3e-9), math.log(30e-9)], [0.5, 0.5])
    print("case bench size: %d sets x %d samples, %d iterations" % (n_sets, m, iters), flush=True)
    phi, mu, var, ll, it = _fit_gpu(g, xs, [start] * n_sets, iters)
    torch.cuda.empty_cache()
    assert np.all(it == iters)
    for r in (0, 21, 42, 63):
        p0, m0, v0, hist = gmm.fit(xs[r], *start, iters)
        assert np.allclose(phi[r], p0, rtol=1e-11, atol=1e-14)
        assert np.allclose(mu[r], m0, rtol=1e-11, atol=1e-14)
        assert np.allclose(var[r], v0, rtol=1e-10, atol=1e-14)
        assert abs(ll[r] - hist[-1]) <= 1e-11 * abs(hist[-1]) + 1e-12
        print("  set %d: mu %s loglik %.12e vs %.12e" % (r, mu[r], ll[r], hist[-1]))



def test_gmm_concurrent_calls(gpu):
    """Two threads fit different batches at the same time on two streams, after calls of
    other sizes in the same process: every result equals the same fit run alone, bitwise."""
    import threading
    import torch
    g = gpu
    st = ([0.5, 0.5], [8.0, 25.0], [4.0, 25.0])
    a = [si.mixture_samples(41 + i, 30000 + 777 * i) for i in range(3)]
    b = [si.mixture_samples(51 + i, 90001 + 123 * i) for i in range(5)]
    ref = {"a": _fit_gpu(g, a, [st] * len(a), 30), "b": _fit_gpu(g, b, [st] * len(b), 30)}
    again = _fit_gpu(g, a, [st] * len(a), 30)   # a smaller batch after a larger one
    for x, y in zip(again, ref["a"]):
        assert np.array_equal(x, y)
    data = {}
    for name, sets in (("a", a), ("b", b)):
        offs = np.concatenate([[0], np.cumsum([len(x) for x in sets])]).astype(np.int64)
        data[name] = (offs, torch.from_numpy(np.concatenate(sets)).cuda(), len(sets))
    streams = {"a": torch.cuda.Stream(), "b": torch.cuda.Stream()}
    torch.cuda.synchronize()
    out, err = {}, {}

    def run(name):
        try:
            offs, xd, n = data[name]
            starts = [np.tile(np.array(v, np.float64), (n, 1)) for v in st]
            out[name] = g.glbm_gmm_fit(offs, xd.data_ptr(), *starts, 30, 0.0, stream=streams[name].cuda_stream)
        except Exception as e:  # reported below
            err[name] = e

    print("case concurrent fits on two streams", flush=True)
    threads = [threading.Thread(target=run, args=(n,)) for n in ("a", "b")]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=90)
    assert not any(t.is_alive() for t in threads)
    assert not err, err
    for name in ("a", "b"):
        for x, y in zip(out[name], ref[name]):
            assert np.array_equal(x, y), name


def test_gmm_argument_errors(gpu):
    """Empty sets, k outside 1 .. GLBM_GMM_MAX_COMPONENTS and non-positive starting
    variances or weights are rejected before any work."""
    import torch
    g = gpu
    xd = torch.zeros(16, dtype=torch.float64, device="cuda")
    one = ([1.0], [0.0], [1.0])
    good = np.array([0, 16], np.int64)
    g.glbm_gmm_fit(good, xd.data_ptr(), *(np.array([v]) for v in one), 1, 0.0)
    cases = [
        (np.array([0, 0], np.int64), one),                                  # empty set
        (np.array([0, 8, 8], np.int64), None),                              # empty second set
        (good, ([1.0], [0.0], [0.0])),                                      # zero variance
        (good, ([1.0], [0.0], [-1.0])),                                     # negative variance
        (good, ([0.0], [0.0], [1.0])),                                      # zero weight
    ]
    for offs, st in cases:
        print("case offsets=%s start=%s" % (offs.tolist(), st), flush=True)
        n_sets = len(offs) - 1
        st = st or one
        arrs = [np.tile(np.array(v, np.float64), (n_sets, 1)) for v in st]
        with pytest.raises(g.GlbmError):
            g.glbm_gmm_fit(offs, xd.data_ptr(), *arrs, 1, 0.0)
    k_bad = g.GLBM_GMM_MAX_COMPONENTS + 1
    arrs = [np.full((1, k_bad), v) for v in (1.0 / k_bad, 0.0, 1.0)]
    with pytest.raises(g.GlbmError):
        g.glbm_gmm_fit(good, xd.data_ptr(), *arrs, 1, 0.0)
