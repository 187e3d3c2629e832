"""ctypes binding of libglbm (include/glbm.h): same names, argument marshalling only.

PyTorch is imported first and provides device memory and streams: the library
then binds to the HIP runtime torch has already loaded, so device pointers and
streams are shared.  Every computation runs in the library's kernels; if the
library is missing this module raises at import.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  (must precede the library load)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libglbm.so")

GLBM_D2Q9, GLBM_D3Q19 = 9, 19
GLBM_STORE_F64, GLBM_STORE_F32, GLBM_STORE_F16DEV, GLBM_STORE_F16LOC, GLBM_STORE_F32LOC = 0, 1, 2, 3, 4
GLBM_OK, GLBM_EINVAL, GLBM_ENOMEM, GLBM_EDEVICE, GLBM_ESTATE, GLBM_ENONFINITE, GLBM_ENOTCONVERGED, GLBM_EUNSTABLE = \
    0, -1, -2, -3, -4, -5, -6, -7
GLBM_WALL_CLASS = 255
GLBM_SCALE_AUTO = -2147483648
GLBM_OPT_GRAPH, GLBM_OPT_TIMING, GLBM_OPT_TILE_ROWS, GLBM_OPT_TILE_WIDTH, GLBM_OPT_CACHE = 1, 2, 3, 4, 5
GLBM_FLAG_F16DEV_OPT_IN = 1
GLBM_GMM_MAX_COMPONENTS = 8
STORE_NAMES = {"f64": GLBM_STORE_F64, "f32": GLBM_STORE_F32, "f16dev": GLBM_STORE_F16DEV,
               "f16loc": GLBM_STORE_F16LOC, "f32loc": GLBM_STORE_F32LOC}
STORE_BYTES = {GLBM_STORE_F64: 8, GLBM_STORE_F32: 4, GLBM_STORE_F16DEV: 2, GLBM_STORE_F16LOC: 2,
               GLBM_STORE_F32LOC: 4}


def bytes_per_update(q: int, store: int) -> int:
    """Algorithmic HBM bytes of one lattice update: read and write q populations
    and the class byte (F16LOC / F32LOC add the float density: 4 B written, 4 B read)."""
    return 2 * q * STORE_BYTES[store] + 1 + (8 if store in (GLBM_STORE_F16LOC, GLBM_STORE_F32LOC) else 0)

EXPORTS = ("glbm_required_bytes", "glbm_init_geometry", "glbm_set_local_perm", "glbm_step_n",
           "glbm_residual", "glbm_permeability", "glbm_set_fields", "glbm_set_fields_device",
           "glbm_get_fields", "glbm_get_populations", "glbm_state_bytes", "glbm_save_state",
           "glbm_load_state", "glbm_set_option", "glbm_sweep_time", "glbm_sweeps_per_launch", "glbm_autotune",
           "glbm_velocity_set", "glbm_destroy", "glbm_last_error", "glbm_class_table", "glbm_pore_percolates",
           "glbm_conv3x3_forward", "glbm_conv3x3_flip_weights", "glbm_conv3x3_wgrad_workspace",
           "glbm_conv3x3_backward_weight", "glbm_cnn_create", "glbm_cnn_destroy", "glbm_cnn_num_params",
           "glbm_cnn_get_params", "glbm_cnn_set_params", "glbm_cnn_get_grads", "glbm_cnn_forward",
           "glbm_cnn_backward", "glbm_cnn_train_step", "glbm_cnn_features", "glbm_cnn_targets",
           "glbm_cnn_apply", "glbm_cnn_set_grads", "glbm_cnn_adam_step", "glbm_cnn_apply_noalloc",
           "glbm_set_pressure_perm", "glbm_class_table_pressure", "glbm_gmm_fit", "glbm_radius_bins",
           "glbm_stream_copy")


class GlbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("glbm error %d: %s" % (code, msg))
        self.code = code


class glbm_instance_desc(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("store", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("wall_faces", ctypes.c_uint32),
                ("tau", ctypes.c_double), ("g", ctypes.c_double * 3),
                ("dev_scale_log2", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("pressure_axis", ctypes.c_int32),
                ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double)]


class glbm_gas_params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "pressure", "temperature", "viscosity", "molar_mass", "tortuosity", "dx", "eps_iom", "eps_om",
        "langmuir_b", "q_sat", "langmuir_vl", "toc", "d_s")]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libglbm.so is not built (%s); run python -m paper_1601_00704_amd.build"
                          % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "glbm_required_bytes": (sz, [i32, vp]),
        "glbm_init_geometry": (i32, [vp, i32, vp, vp, vp, sz, vp]),
        "glbm_set_local_perm": (i32, [vp, i32, i32, vp, vp, vp]),
        "glbm_set_pressure_perm": (i32, [vp, i32, i32, vp, vp, vp, vp, vp, f64, f64]),
        "glbm_gmm_fit": (i32, [i32, vp, vp, i32, vp, vp, vp, i32, f64, vp, vp, vp]),
        "glbm_radius_bins": (i32, [f64, f64, i32, vp]),
        "glbm_stream_copy": (i32, [vp, vp, sz, vp]),
        "glbm_class_table_pressure": (i32, [vp, i32, vp, i32, vp, vp, vp, vp, vp, vp]),
        "glbm_step_n": (i32, [vp, i64, f64]),
        "glbm_residual": (i32, [vp, vp, vp]),
        "glbm_permeability": (i32, [vp, vp]),
        "glbm_set_fields": (i32, [vp, i32, vp, vp]),
        "glbm_set_fields_device": (i32, [vp, i32, vp, vp]),
        "glbm_get_fields": (i32, [vp, i32, vp, vp]),
        "glbm_get_populations": (i32, [vp, i32, vp]),
        "glbm_state_bytes": (sz, [vp]),
        "glbm_save_state": (i32, [vp, vp, sz]),
        "glbm_load_state": (i32, [vp, vp, sz]),
        "glbm_set_option": (i32, [vp, i32, i64]),
        "glbm_sweep_time": (i32, [vp, vp, vp]),
        "glbm_sweeps_per_launch": (i32, [vp, vp]),
        "glbm_autotune": (i32, [vp, i32, vp]),
        "glbm_velocity_set": (i32, [i32, vp, vp]),
        "glbm_pore_percolates": (i32, [i32, i32, i32, i32, vp, i32, vp]),
        "glbm_destroy": (i32, [vp]),
        "glbm_last_error": (ctypes.c_char_p, []),
        "glbm_class_table": (i32, [vp, i32, vp, i32, vp, vp, vp]),
        "glbm_conv3x3_forward": (i32, [vp, i32, i32, i32, vp, vp, vp, i32, i32, i32, i32, i32, i32, i32, i32, i32,
                                       vp]),
        "glbm_conv3x3_flip_weights": (i32, [vp, i32, i32, vp, vp]),
        "glbm_conv3x3_wgrad_workspace": (sz, [i32, i32, i32, i32, i32]),
        "glbm_conv3x3_backward_weight": (i32, [vp, i32, i32, i32, vp, i32, i32, i32, vp, vp, vp, i32, i32, i32,
                                               vp]),
        "glbm_cnn_create": (i32, [vp, i32, i32, i32, ctypes.c_uint64, vp]),
        "glbm_cnn_destroy": (i32, [vp]),
        "glbm_cnn_num_params": (i64, [vp]),
        "glbm_cnn_get_params": (i32, [vp, vp]),
        "glbm_cnn_set_params": (i32, [vp, vp]),
        "glbm_cnn_get_grads": (i32, [vp, vp]),
        "glbm_cnn_forward": (i32, [vp, vp, vp, i32]),
        "glbm_cnn_backward": (i32, [vp, vp, vp, vp, i32, vp]),
        "glbm_cnn_train_step": (i32, [vp, vp, vp, vp, i32, ctypes.c_float, vp]),
        "glbm_cnn_features": (i32, [vp, i32, f64, vp]),
        "glbm_cnn_targets": (i32, [vp, i32, f64, f64, vp, vp]),
        "glbm_cnn_apply": (i32, [vp, i32, vp, f64, f64]),
        "glbm_cnn_set_grads": (i32, [vp, vp]),
        "glbm_cnn_apply_noalloc": (i32, [vp, i32, vp, f64, f64]),
        "glbm_cnn_adam_step": (i32, [vp, ctypes.c_float]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


_lib = _load()


def lib():
    return _lib


def _check(rc: int, allow=(GLBM_OK,)) -> int:
    if rc not in allow:
        raise GlbmError(rc, _lib.glbm_last_error().decode())
    return rc


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_desc(shape, lattice=GLBM_D2Q9, store=GLBM_STORE_F32, tau=1.0, g=(1e-6, 0.0, 0.0),
              wall_faces=0, dev_scale_log2=GLBM_SCALE_AUTO, check_every=100, flags=0, pressure_axis=None,
              rho_in=1.0, rho_out=1.0) -> glbm_instance_desc:
    """Descriptor of one instance; shape is (ny, nx) or (nz, ny, nx).  pressure_axis (0 = x,
    1 = y, 2 = z) puts pressure faces of densities rho_in / rho_out on that axis."""
    if len(shape) == 2:
        nz, ny, nx = 1, shape[0], shape[1]
    else:
        nz, ny, nx = shape
    d = glbm_instance_desc()
    d.lattice, d.store, d.nx, d.ny, d.nz = lattice, store, nx, ny, nz
    d.wall_faces, d.tau = wall_faces, tau
    for a in range(3):
        d.g[a] = float(g[a])
    d.dev_scale_log2, d.check_every, d.flags = dev_scale_log2, check_every, flags
    d.pressure_axis = 0 if pressure_axis is None else int(pressure_axis) + 1
    d.rho_in, d.rho_out = float(rho_in), float(rho_out)
    return d


def _desc_array(descs: Sequence[glbm_instance_desc]):
    arr = (glbm_instance_desc * len(descs))(*descs)
    return arr


def glbm_required_bytes(descs: Sequence[glbm_instance_desc]) -> int:
    return int(_lib.glbm_required_bytes(len(descs), _desc_array(descs)))


def glbm_init_geometry(descs, cls_maps, pop_dev: Optional[int] = None, pop_bytes: int = 0,
                       hip_stream: Optional[int] = None):
    """Returns the context handle (an int)."""
    arr = _desc_array(descs)
    maps = [np.ascontiguousarray(m, dtype=np.uint8) for m in cls_maps]
    ptrs = (ctypes.c_void_p * len(maps))(*[m.ctypes.data for m in maps])
    out = ctypes.c_void_p()
    _check(_lib.glbm_init_geometry(ctypes.byref(out), len(descs), arr, ptrs, pop_dev, pop_bytes, hip_stream))
    return out.value


def glbm_set_local_perm(ctx, inst: int, eps, k_lattice, f_eps=None):
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    k = np.ascontiguousarray(k_lattice, dtype=np.float64)
    fe = None if f_eps is None else np.ascontiguousarray(f_eps, dtype=np.float64)
    _check(_lib.glbm_set_local_perm(ctx, inst, len(eps), _ptr(eps), _ptr(k), None if fe is None else _ptr(fe)))


def glbm_set_pressure_perm(ctx, inst: int, eps, k_const, k_knudsen, k_surface, langmuir_b, p_in, p_out):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (eps, k_const, k_knudsen, k_surface, langmuir_b)]
    n = len(arrs[0])
    assert all(len(a) == n for a in arrs)
    _check(_lib.glbm_set_pressure_perm(ctx, inst, n, *[_ptr(a) for a in arrs], float(p_in), float(p_out)))


def glbm_step_n(ctx, n: int, tol: float = 0.0) -> int:
    return _check(_lib.glbm_step_n(ctx, int(n), float(tol)), allow=(GLBM_OK, GLBM_ENOTCONVERGED))


def glbm_residual(ctx, n_inst: int):
    r = np.zeros(n_inst)
    s = np.zeros(n_inst, dtype=np.int64)
    _check(_lib.glbm_residual(ctx, _ptr(r), _ptr(s)))
    return r, s


def glbm_permeability(ctx, n_inst: int) -> np.ndarray:
    k = np.zeros(3 * n_inst)
    _check(_lib.glbm_permeability(ctx, _ptr(k)))
    return k.reshape(n_inst, 3)


def glbm_set_fields(ctx, inst: int, rho, u):
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    _check(_lib.glbm_set_fields(ctx, inst, _ptr(rho), _ptr(u)))


def glbm_set_fields_device(ctx, inst: int, drho_dev: int, u_dev: int):
    _check(_lib.glbm_set_fields_device(ctx, inst, drho_dev, u_dev))


def glbm_get_fields(ctx, inst: int, n: int):
    rho = np.zeros(n)
    u = np.zeros(3 * n)
    _check(_lib.glbm_get_fields(ctx, inst, _ptr(rho), _ptr(u)))
    return rho, u.reshape(3, n)


def glbm_get_populations(ctx, inst: int, q: int, n: int) -> np.ndarray:
    f = np.zeros(q * n)
    _check(_lib.glbm_get_populations(ctx, inst, _ptr(f)))
    return f


def glbm_state_bytes(ctx) -> int:
    return int(_lib.glbm_state_bytes(ctx))


def glbm_save_state(ctx) -> np.ndarray:
    buf = np.zeros(glbm_state_bytes(ctx), dtype=np.uint8)
    _check(_lib.glbm_save_state(ctx, _ptr(buf), buf.size))
    return buf


def glbm_load_state(ctx, buf: np.ndarray):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(_lib.glbm_load_state(ctx, _ptr(buf), buf.size))


def glbm_set_option(ctx, option: int, value: int):
    _check(_lib.glbm_set_option(ctx, option, int(value)))


def glbm_sweep_time(ctx):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(_lib.glbm_sweep_time(ctx, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def glbm_sweeps_per_launch(ctx) -> int:
    n = ctypes.c_int32()
    _check(_lib.glbm_sweeps_per_launch(ctx, ctypes.byref(n)))
    return n.value


def glbm_pore_percolates(cls, axis: int = 1, lattice: int = None) -> bool:
    """Whether the open pores (class 0) of a class map ((ny, nx) or (nz, ny, nx)) connect
    the two faces of the drive axis (1 = x, 2 = y, 3 = z)."""
    c = np.ascontiguousarray(cls, dtype=np.uint8)
    if lattice is None:
        lattice = GLBM_D2Q9 if c.ndim == 2 else GLBM_D3Q19
    nz, ny, nx = (1,) + c.shape if c.ndim == 2 else c.shape
    out = ctypes.c_int32()
    _check(_lib.glbm_pore_percolates(lattice, nx, ny, nz, _ptr(c), axis, ctypes.byref(out)))
    return bool(out.value)


def glbm_autotune(ctx, steps: int = 20):
    """Returns the chosen (tile width, tile rows, cache policy)."""
    ch = (ctypes.c_int32 * 3)()
    _check(_lib.glbm_autotune(ctx, steps, ch))
    return tuple(ch)


def glbm_velocity_set(lattice: int):
    q = int(lattice)
    e = np.zeros(3 * q, dtype=np.int32)
    w = np.zeros(q)
    _check(_lib.glbm_velocity_set(lattice, _ptr(e), _ptr(w)))
    return e.reshape(q, 3), w


def glbm_destroy(ctx):
    _check(_lib.glbm_destroy(ctx))


def glbm_last_error() -> str:
    return _lib.glbm_last_error().decode()


def glbm_class_table(params: glbm_gas_params, r_iom, r_om):
    r_iom = np.ascontiguousarray(r_iom, dtype=np.float64)
    r_om = np.ascontiguousarray(r_om, dtype=np.float64)
    eps = np.zeros(256)
    k = np.zeros(256)
    rc = _lib.glbm_class_table(ctypes.byref(params), len(r_iom), _ptr(r_iom), len(r_om), _ptr(r_om),
                               _ptr(eps), _ptr(k))
    if rc != GLBM_OK:
        raise GlbmError(rc, "glbm_class_table: invalid parameters")
    return eps, k


def glbm_class_table_pressure(params: glbm_gas_params, r_iom, r_om):
    """(eps, k_const, k_knudsen, k_surface, b), 256 entries each (lattice units, P in Pa)."""
    r_iom = np.ascontiguousarray(r_iom, dtype=np.float64)
    r_om = np.ascontiguousarray(r_om, dtype=np.float64)
    out = [np.zeros(256) for _ in range(5)]
    rc = _lib.glbm_class_table_pressure(ctypes.byref(params), len(r_iom), _ptr(r_iom), len(r_om), _ptr(r_om),
                                        *[_ptr(a) for a in out])
    if rc != GLBM_OK:
        raise GlbmError(rc, "glbm_class_table_pressure: invalid parameters")
    return tuple(out)


def glbm_gmm_fit(offsets, x_dev, phi, mu, var, iters, tol=0.0, stream=None):
    """Batched EM fit (Eq. 20-24).  offsets: n_sets + 1 sample offsets into the device array
    x_dev (a pointer to doubles); phi, mu, var: (n_sets, k) starting points.  Returns
    (phi, mu, var, loglik, iters_done)."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    phi, mu, var = (np.array(a, dtype=np.float64, order="C", copy=True) for a in (phi, mu, var))
    n_sets, k = phi.shape
    ll = np.zeros(n_sets)
    it = np.zeros(n_sets, dtype=np.int32)
    _check(_lib.glbm_gmm_fit(n_sets, _ptr(offsets), x_dev, k, _ptr(phi), _ptr(mu), _ptr(var), int(iters), float(tol),
                             _ptr(ll), _ptr(it), _stream() if stream is None else stream))
    return phi, mu, var, ll, it


def glbm_stream_copy(src, dst, nbytes, stream=None):
    _check(_lib.glbm_stream_copy(src, dst, int(nbytes), _stream() if stream is None else stream))


def glbm_radius_bins(mu_ln, sigma_ln, n=127):
    r = np.zeros(n)
    _check(_lib.glbm_radius_bins(float(mu_ln), float(sigma_ln), int(n), _ptr(r)))
    return r


def gas_params(inst, molar_mass=0.016043) -> glbm_gas_params:
    """glbm_gas_params of a shale_inputs.Instance (an input record: plain field copy)."""
    p = glbm_gas_params()
    p.pressure, p.temperature, p.viscosity = inst.pressure, inst.temperature, inst.viscosity
    p.molar_mass, p.tortuosity, p.dx = molar_mass, inst.tortuosity, inst.dx
    p.eps_iom, p.eps_om = inst.eps_iom, inst.eps_om
    p.langmuir_b = 1.0 / inst.langmuir_pl
    p.q_sat = inst.q_sat if inst.q_sat is not None else 0.0
    p.langmuir_vl = inst.langmuir_vl if inst.langmuir_vl is not None else 0.0
    p.toc, p.d_s = inst.toc, inst.d_s
    return p


# ------------------------------------------------------------ warm-start network
def _stream():
    return torch.cuda.current_stream().cuda_stream


def glbm_conv3x3_forward(x, x_pitch, x_off, cin, w, bias, y, y_pitch, y_off, cout, relu, y_is_f32, accumulate,
                         batch, height, width, stream=None):
    """Device pointers (ints) in, see glbm_cnn.h."""
    _check(_lib.glbm_conv3x3_forward(x, x_pitch, x_off, cin, w, bias, y, y_pitch, y_off, cout, int(relu),
                                     int(y_is_f32), int(accumulate), batch, height, width,
                                     _stream() if stream is None else stream))


def glbm_conv3x3_flip_weights(w, cin, cout, wt, stream=None):
    _check(_lib.glbm_conv3x3_flip_weights(w, cin, cout, wt, _stream() if stream is None else stream))


def glbm_conv3x3_wgrad_workspace(cin, cout, batch, height, width) -> int:
    return int(_lib.glbm_conv3x3_wgrad_workspace(cin, cout, batch, height, width))


def glbm_conv3x3_backward_weight(x, x_pitch, x_off, cin, dy, dy_pitch, dy_off, cout, dw, db, workspace, batch,
                                 height, width, stream=None):
    _check(_lib.glbm_conv3x3_backward_weight(x, x_pitch, x_off, cin, dy, dy_pitch, dy_off, cout, dw, db, workspace,
                                             batch, height, width, _stream() if stream is None else stream))


def glbm_cnn_create(max_batch, height, width, seed=0, stream=None):
    out = ctypes.c_void_p()
    _check(_lib.glbm_cnn_create(ctypes.byref(out), max_batch, height, width, seed,
                                _stream() if stream is None else stream))
    return out.value


def glbm_cnn_destroy(cnn):
    _check(_lib.glbm_cnn_destroy(cnn))


def glbm_cnn_num_params(cnn) -> int:
    return int(_lib.glbm_cnn_num_params(cnn))


def glbm_cnn_get_params(cnn) -> np.ndarray:
    a = np.zeros(glbm_cnn_num_params(cnn), dtype=np.float32)
    _check(_lib.glbm_cnn_get_params(cnn, _ptr(a)))
    return a


def glbm_cnn_set_params(cnn, params):
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(_lib.glbm_cnn_set_params(cnn, _ptr(a)))


def glbm_cnn_get_grads(cnn) -> np.ndarray:
    a = np.zeros(glbm_cnn_num_params(cnn), dtype=np.float32)
    _check(_lib.glbm_cnn_get_grads(cnn, _ptr(a)))
    return a


def glbm_cnn_set_grads(cnn, grads):
    a = np.ascontiguousarray(grads, dtype=np.float32)
    _check(_lib.glbm_cnn_set_grads(cnn, _ptr(a)))


def glbm_cnn_adam_step(cnn, lr):
    _check(_lib.glbm_cnn_adam_step(cnn, float(lr)))


def glbm_cnn_forward(cnn, x, y, batch):
    _check(_lib.glbm_cnn_forward(cnn, x, y, batch))


def glbm_cnn_backward(cnn, x, target, mask, batch) -> float:
    loss = ctypes.c_double()
    _check(_lib.glbm_cnn_backward(cnn, x, target, mask, batch, ctypes.byref(loss)))
    return loss.value


def glbm_cnn_train_step(cnn, x, target, mask, batch, lr) -> float:
    loss = ctypes.c_double()
    _check(_lib.glbm_cnn_train_step(cnn, x, target, mask, batch, float(lr), ctypes.byref(loss)))
    return loss.value


def glbm_cnn_features(ctx, inst, log10_pressure_mpa, x):
    _check(_lib.glbm_cnn_features(ctx, inst, float(log10_pressure_mpa), x))


def glbm_cnn_targets(ctx, inst, rho_scale, u_scale, target, mask):
    _check(_lib.glbm_cnn_targets(ctx, inst, float(rho_scale), float(u_scale), target, mask))


def glbm_cnn_apply(ctx, inst, y, rho_scale, u_scale):
    _check(_lib.glbm_cnn_apply(ctx, inst, y, float(rho_scale), float(u_scale)))


def glbm_cnn_apply_noalloc(ctx, inst, y, rho_scale, u_scale):
    _check(_lib.glbm_cnn_apply_noalloc(ctx, inst, y, float(rho_scale), float(u_scale)))


GLBM_NOALLOC_MAX_NODES = 1 << 20


def to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """float array -> bfloat16 bit patterns (uint16), nearest even."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def from_bf16_bits(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


class Solver:
    """One context with torch-owned population memory on the current device and stream."""

    def __init__(self, descs, cls_maps, device="cuda", stream=None):
        self.descs = list(descs)
        self.n_inst = len(self.descs)
        self.q = self.descs[0].lattice
        self.shapes = [(d.nz, d.ny, d.nx) for d in self.descs]
        nbytes = glbm_required_bytes(self.descs)
        if nbytes == 0:
            raise GlbmError(GLBM_EINVAL, glbm_last_error())
        self.pop = torch.empty(nbytes, dtype=torch.uint8, device=device)
        s = stream if stream is not None else torch.cuda.current_stream(self.pop.device)
        self.stream = s
        self.ctx = glbm_init_geometry(self.descs, cls_maps, self.pop.data_ptr(), nbytes, s.cuda_stream)

    def n_nodes(self, inst=0):
        nz, ny, nx = self.shapes[inst]
        return nz * ny * nx

    def set_local_perm(self, eps, k_lattice, f_eps=None, inst=-1):
        glbm_set_local_perm(self.ctx, inst, eps, k_lattice, f_eps)

    def set_pressure_perm(self, eps, k_const, k_knudsen, k_surface, langmuir_b, p_in, p_out, inst=-1):
        glbm_set_pressure_perm(self.ctx, inst, eps, k_const, k_knudsen, k_surface, langmuir_b, p_in, p_out)

    def step(self, n, tol=0.0):
        return glbm_step_n(self.ctx, n, tol)

    def residual(self):
        return glbm_residual(self.ctx, self.n_inst)

    def permeability(self):
        return glbm_permeability(self.ctx, self.n_inst)

    def fields(self, inst=0):
        return glbm_get_fields(self.ctx, inst, self.n_nodes(inst))

    def populations(self, inst=0):
        return glbm_get_populations(self.ctx, inst, self.q, self.n_nodes(inst)).reshape(
            self.q, self.n_nodes(inst))

    def set_fields(self, rho, u, inst=0):
        glbm_set_fields(self.ctx, inst, rho, u)

    def set_option(self, opt, value):
        glbm_set_option(self.ctx, opt, value)

    def close(self):
        if self.ctx:
            glbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
