"""Thin ctypes binding of liblpc.so (the C ABI in include/lpc.h).

Argument marshalling only: every step of the method runs in liblpc's HIP kernels. PyTorch supplies device memory
and the current stream. The functions keep the C names (lpc_init_ic, lpc_pm_force, lpc_cola_step,
lpc_power_spectrum, ...). If liblpc.so is missing the import of this module fails loudly; there is no fallback.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblpc.so")

LPC_OP_INIT_IC = 1
LPC_OP_PM_FORCE = 2
LPC_OP_COLA_STEP = 3
LPC_OP_POWER_SPECTRUM = 4
LPC_OP_FFT = 5
LPC_OP_BISPECTRUM = 6
COEF_COLUMNS = ("a", "D1", "D2", "dD1", "dD2", "E", "K", "Q", "dDD1", "dDD2", "f1", "f2")

STATUS = {0: "LPC_OK", -1: "LPC_ERR_INVALID_ARG", -2: "LPC_ERR_UNSUPPORTED_SIZE", -3: "LPC_ERR_WORKSPACE",
          -4: "LPC_ERR_HIP", -5: "LPC_ERR_FIXED_OVERFLOW", -6: "LPC_ERR_NONFINITE", -7: "LPC_ERR_CAPACITY"}


class LpcError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {detail}")


class Geometry(ctypes.Structure):
    _fields_ = [("n_side", ctypes.c_int32), ("n_mesh", ctypes.c_int32), ("box", ctypes.c_double)]


class Cosmology(ctypes.Structure):
    _fields_ = [("omega_m", ctypes.c_double), ("h", ctypes.c_double), ("sigma8", ctypes.c_double),
                ("n_s", ctypes.c_double)]


class Stepping(ctypes.Structure):
    _fields_ = [("cola", ctypes.c_int32), ("modified", ctypes.c_int32), ("n_lpt", ctypes.c_double),
                ("deconv_power", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Particles(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("vel", ctypes.c_void_p), ("psi1", ctypes.c_void_p),
                ("psi2", ctypes.c_void_p), ("id", ctypes.c_void_p), ("n", ctypes.c_int64)]


class Lightcone(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("a_start", ctypes.c_double), ("rep_lo", ctypes.c_int32 * 3),
                ("rep_hi", ctypes.c_int32 * 3), ("records", ctypes.c_void_p), ("capacity", ctypes.c_int64)]


LIGHTCONE_RECORD_FIELDS = 10  # lpc_lightcone_record: 6 floats + a + index + replicate + reserved (4 bytes each)


class PngTerm(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double), ("g", ctypes.c_double)]


class Png(ctypes.Structure):
    _fields_ = [("f_nl", ctypes.c_double), ("n_terms", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("terms", PngTerm * 4)]


PNG_KINDS = {"local": 0, "equilateral": 1, "orthogonal": 2}


class BatchEntry(ctypes.Structure):
    _fields_ = [("geom", Geometry), ("particles", Particles)]


class FftTiling(ctypes.Structure):
    _fields_ = [("z_rows", ctypes.c_int32), ("axis_cols", ctypes.c_int32), ("poisson_cols", ctypes.c_int32),
                ("c2r_rows", ctypes.c_int32)]


TILING_FIELDS = tuple(f for f, _ in FftTiling._fields_)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"liblpc.so not found at {LIB_PATH}: run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "lpc_workspace_bytes": (sz, [P(Geometry), i32, i64]),
        "lpc_init_ic": (i32, [P(Geometry), P(Cosmology), ctypes.c_uint64, dbl, P(Particles), vp, sz, vp]),
        "lpc_init_ic_png": (i32, [P(Geometry), P(Cosmology), ctypes.c_uint64, dbl, P(Png), P(Particles), vp, sz, vp]),
        "lpc_png_preset": (i32, [i32, dbl, P(Png)]),
        "lpc_pm_force": (i32, [P(Geometry), P(Stepping), vp, i64, vp, vp, vp, sz, vp]),
        "lpc_pm_force_noalloc": (i32, [P(Geometry), P(Stepping), vp, i64, vp, vp, vp]),
        "lpc_cola_step": (i32, [P(Geometry), P(Cosmology), P(Stepping), P(dbl), i32, P(Particles), vp, sz, vp]),
        "lpc_cola_step_lightcone": (i32, [P(Geometry), P(Cosmology), P(Stepping), P(dbl), i32, P(Particles),
                                          P(Lightcone), P(i64), vp, sz, vp]),
        "lpc_comoving_distance": (i32, [P(Cosmology), P(dbl), i32, P(dbl)]),
        "lpc_workspace_bytes_batched": (sz, [P(BatchEntry), i32]),
        "lpc_cola_step_batched": (i32, [P(BatchEntry), i32, P(Cosmology), P(Stepping), P(dbl), i32, vp, sz, vp]),
        "lpc_graph_enable": (i32, [i32]),
        "lpc_net_param_count": (i64, []),
        "lpc_net_init": (i32, [P(ctypes.c_float), ctypes.c_uint64]),
        "lpc_net_workspace_bytes": (sz, [i32]),
        "lpc_net_features": (i32, [P(Geometry), vp, vp, i64, vp, vp, vp, vp, sz, vp]),
        "lpc_net_forward": (i32, [i32, vp, vp, vp, vp, sz, vp]),
        "lpc_net_loss_grad": (i32, [i32, vp, vp, vp, vp, P(dbl), vp, sz, vp]),
        "lpc_net_symmetry": (i32, [i32, i32, i32, vp, vp, vp]),
        "lpc_net_scale_output": (i32, [vp, ctypes.c_float, vp]),
        "lpc_net_adam": (i32, [vp, vp, vp, vp, i64, ctypes.c_float, vp]),
        "lpc_net_apply": (i32, [P(Geometry), vp, P(Particles), vp, sz, vp]),
        "lpc_power_spectrum": (i32, [P(Geometry), vp, i64, dbl, i32, P(dbl), P(dbl), P(i64), vp, sz, vp]),
        "lpc_bispectrum": (i32, [P(Geometry), vp, i64, P(dbl), i32, dbl, P(dbl), P(dbl), P(dbl), vp, sz, vp]),
        "lpc_cola_coefficients": (i32, [P(Cosmology), P(Stepping), P(dbl), i32, P(dbl)]),
        "lpc_linear_power": (i32, [P(Cosmology), P(dbl), i32, P(dbl)]),
        "lpc_fft_r2c": (i32, [i32, vp, vp, vp, sz, vp]),
        "lpc_fft_c2r": (i32, [i32, vp, vp, vp, sz, vp]),
        "lpc_fft_pitch": (i32, [i32]),
        "lpc_fft_tiling_default": (i32, [i32, P(FftTiling)]),
        "lpc_fft_tiling_get": (i32, [i32, P(FftTiling)]),
        "lpc_fft_tiling_set": (i32, [i32, P(FftTiling)]),
        "lpc_fft_tiling_reset": (i32, []),
        "lpc_profile_enable": (i32, [i32]),
        "lpc_profile_reset": (i32, []),
        "lpc_profile_count": (i32, []),
        "lpc_profile_get": (i32, [i32, P(ctypes.c_char_p), P(i64), P(dbl)]),
        "lpc_status_string": (ctypes.c_char_p, [i32]),
        "lpc_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()
EXPORTED = ("lpc_workspace_bytes", "lpc_init_ic", "lpc_init_ic_png", "lpc_png_preset", "lpc_pm_force",
            "lpc_pm_force_noalloc", "lpc_cola_step",
            "lpc_cola_step_lightcone", "lpc_comoving_distance",
            "lpc_workspace_bytes_batched",
            "lpc_cola_step_batched", "lpc_graph_enable", "lpc_power_spectrum", "lpc_bispectrum",
            "lpc_net_param_count", "lpc_net_init", "lpc_net_workspace_bytes", "lpc_net_features", "lpc_net_forward",
            "lpc_net_loss_grad", "lpc_net_symmetry", "lpc_net_scale_output", "lpc_net_adam", "lpc_net_apply",
            "lpc_cola_coefficients", "lpc_linear_power", "lpc_fft_r2c", "lpc_fft_c2r", "lpc_fft_pitch",
            "lpc_fft_tiling_default", "lpc_fft_tiling_get", "lpc_fft_tiling_set", "lpc_fft_tiling_reset",
            "lpc_profile_enable", "lpc_profile_reset", "lpc_profile_count", "lpc_profile_get",
            "lpc_status_string", "lpc_last_error")


def _check(status):
    if status != 0:
        raise LpcError(status, LIB.lpc_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def geometry(n_side, n_mesh, box):
    return Geometry(int(n_side), int(n_mesh), float(box))


def cosmology(omega_m=0.31, h=0.68, sigma8=0.8, n_s=0.96):
    return Cosmology(omega_m, h, sigma8, n_s)


def stepping(cola=1, modified=1, n_lpt=-2.5, deconv_power=1):
    return Stepping(int(cola), int(modified), float(n_lpt), int(deconv_power), 0)


def lpc_workspace_bytes(geom, op, n_particles=0):
    return int(LIB.lpc_workspace_bytes(ctypes.byref(geom), int(op), int(n_particles)))


def workspace(geom, op, device="cuda", n_particles=None):
    """A caller-owned workspace tensor (uint8) for operation `op`; n_particles defaults to n_side^3."""
    import torch
    if n_particles is None:
        n_particles = int(geom.n_side) ** 3
    nbytes = lpc_workspace_bytes(geom, op, n_particles)
    if nbytes == 0:
        raise LpcError(-2, f"unsupported geometry {geom.n_side}/{geom.n_mesh} for op {op}")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


class ParticleSet:
    """Device SoA particles: pos/vel/psi1/psi2 float32 [3, n], id int32 [n] (torch tensors)."""

    def __init__(self, pos, vel, psi1=None, psi2=None, id=None):
        self.pos, self.vel, self.psi1, self.psi2, self.id = pos, vel, psi1, psi2, id

    @classmethod
    def empty(cls, n, device="cuda"):
        import torch
        f = lambda: torch.empty((3, n), dtype=torch.float32, device=device)
        return cls(f(), f(), f(), f(), torch.empty(n, dtype=torch.int32, device=device))

    @property
    def n(self):
        return int(self.pos.shape[1])

    def c_struct(self):
        for t in (self.pos, self.vel, self.psi1, self.psi2):
            if t is not None and not t.is_contiguous():
                raise ValueError("particle arrays must be contiguous")
        return Particles(_ptr(self.pos), _ptr(self.vel), _ptr(self.psi1), _ptr(self.psi2), _ptr(self.id), self.n)


def lpc_init_ic(geom, cosmo, seed, a_init, particles, ws, stream=None):
    p = particles.c_struct()
    _check(LIB.lpc_init_ic(ctypes.byref(geom), ctypes.byref(cosmo), ctypes.c_uint64(seed), float(a_init),
                           ctypes.byref(p), _ptr(ws), ws.numel(), _stream(stream)))


def png(f_nl, kind=None, terms=None):
    """An lpc_png: a preset kind ("local", "equilateral", "orthogonal") or explicit terms [(c, a, b, g), ...]."""
    p = Png()
    if kind is not None:
        _check(LIB.lpc_png_preset(PNG_KINDS[kind], float(f_nl), ctypes.byref(p)))
        return p
    p.f_nl = float(f_nl)
    p.n_terms = len(terms)
    for t, (c, a, b, g) in enumerate(terms):
        p.terms[t] = PngTerm(float(c), float(a), float(b), float(g))
    return p


def lpc_init_ic_png(geom, cosmo, seed, a_init, png_params, particles, ws, stream=None):
    p = particles.c_struct()
    _check(LIB.lpc_init_ic_png(ctypes.byref(geom), ctypes.byref(cosmo), ctypes.c_uint64(seed), float(a_init),
                               ctypes.byref(png_params), ctypes.byref(p), _ptr(ws), ws.numel(), _stream(stream)))


def lpc_pm_force(geom, step, pos, grad_out, ws, density_out=None, stream=None):
    _check(LIB.lpc_pm_force(ctypes.byref(geom), ctypes.byref(step), _ptr(pos), int(pos.shape[1]), _ptr(grad_out),
                            _ptr(density_out), _ptr(ws), ws.numel(), _stream(stream)))


NOALLOC_SCRATCH_BYTES = 64 << 20  # LPC_NOALLOC_SCRATCH_BYTES


def lpc_pm_force_noalloc(geom, step, pos, grad_out, density_out=None, stream=None):
    """lpc_pm_force on the library's static per-GPU scratch (no workspace argument, no allocation)."""
    _check(LIB.lpc_pm_force_noalloc(ctypes.byref(geom), ctypes.byref(step), _ptr(pos), int(pos.shape[1]),
                                    _ptr(grad_out), _ptr(density_out), _stream(stream)))


def lpc_cola_step(geom, cosmo, step, a_list, particles, ws, stream=None):
    a = np.ascontiguousarray(a_list, dtype=np.float64)
    p = particles.c_struct()
    _check(LIB.lpc_cola_step(ctypes.byref(geom), ctypes.byref(cosmo), ctypes.byref(step),
                             a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(a.size), ctypes.byref(p),
                             _ptr(ws), ws.numel(), _stream(stream)))


def lightcone(origin, a_start, records=None, rep_lo=(0, 0, 0), rep_hi=(0, 0, 0)):
    """An lpc_lightcone; `records` is a device tensor of shape (capacity, 10) with 4-byte elements (float32 or int32
    view of lpc_lightcone_record), or None for capacity 0. Keep the tensor referenced while the struct is used."""
    cap = 0 if records is None else int(records.shape[0])
    if records is not None and (records.element_size() != 4 or records.shape[1] != LIGHTCONE_RECORD_FIELDS
                                or not records.is_contiguous()):
        raise ValueError("records must be a contiguous (capacity, 10) tensor of 4-byte elements")
    return Lightcone((ctypes.c_double * 3)(*origin), float(a_start), (ctypes.c_int32 * 3)(*rep_lo),
                     (ctypes.c_int32 * 3)(*rep_hi), _ptr(records).value, cap)


def lpc_cola_step_lightcone(geom, cosmo, step, a_list, particles, lc, ws, stream=None):
    """lpc_cola_step with the lightcone drift; returns the number of records (raises LpcError with status -7 when it
    exceeds the capacity)."""
    a = np.ascontiguousarray(a_list, dtype=np.float64)
    p = particles.c_struct()
    count = ctypes.c_int64(0)
    status = LIB.lpc_cola_step_lightcone(ctypes.byref(geom), ctypes.byref(cosmo), ctypes.byref(step),
                                         a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(a.size),
                                         ctypes.byref(p), ctypes.byref(lc), ctypes.byref(count), _ptr(ws), ws.numel(),
                                         _stream(stream))
    if status != 0:
        err = LpcError(status, LIB.lpc_last_error().decode())
        err.count = int(count.value)
        raise err
    return int(count.value)


def lpc_comoving_distance(cosmo, a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = np.empty_like(a)
    D = ctypes.POINTER(ctypes.c_double)
    _check(LIB.lpc_comoving_distance(ctypes.byref(cosmo), a.ctypes.data_as(D), int(a.size), out.ctypes.data_as(D)))
    return out


def _entries(boxes):
    """boxes: sequence of (geometry, ParticleSet) -> ctypes array of BatchEntry (the particle sets stay referenced
    by the caller)."""
    arr = (BatchEntry * len(boxes))()
    for i, (g, ps) in enumerate(boxes):
        arr[i].geom = g
        arr[i].particles = ps.c_struct()
    return arr


def lpc_workspace_bytes_batched(boxes):
    return int(LIB.lpc_workspace_bytes_batched(_entries(boxes), len(boxes)))


def workspace_batched(boxes, device="cuda"):
    import torch
    nbytes = lpc_workspace_bytes_batched(boxes)
    if nbytes == 0:
        raise LpcError(-2, "unsupported geometry in batch")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def lpc_cola_step_batched(boxes, cosmo, step, a_list, ws, stream=None):
    """One lpc_cola_step run for every (geometry, ParticleSet) in `boxes`, all stages batched across boxes."""
    a = np.ascontiguousarray(a_list, dtype=np.float64)
    e = _entries(boxes)
    _check(LIB.lpc_cola_step_batched(e, len(boxes), ctypes.byref(cosmo), ctypes.byref(step),
                                     a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(a.size), _ptr(ws),
                                     ws.numel(), _stream(stream)))


def lpc_graph_enable(on=True):
    _check(LIB.lpc_graph_enable(1 if on else 0))


def lpc_power_spectrum(geom, pos, k_max, n_bins, ws, stream=None):
    k = np.empty(n_bins, dtype=np.float64)
    pk = np.empty(n_bins, dtype=np.float64)
    cnt = np.empty(n_bins, dtype=np.int64)
    D = ctypes.POINTER(ctypes.c_double)
    _check(LIB.lpc_power_spectrum(ctypes.byref(geom), _ptr(pos), int(pos.shape[1]), float(k_max), int(n_bins),
                                  k.ctypes.data_as(D), pk.ctypes.data_as(D),
                                  cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return k, pk, cnt


def lpc_bispectrum(geom, pos, triangles, dk, ws, stream=None):
    """Reduced bispectrum of particles pos[3][n] on the geom.n_mesh estimator mesh: triangles is a sequence of
    (k1, k2, k3) shell centres (h/Mpc), dk the shell width. Returns (B, Q, P) numpy arrays ([m], [m], [m][3])."""
    k123 = np.ascontiguousarray(np.asarray(triangles, dtype=np.float64).reshape(-1, 3))
    m = k123.shape[0]
    B = np.empty(m, dtype=np.float64)
    Q = np.empty(m, dtype=np.float64)
    P = np.empty((m, 3), dtype=np.float64)
    D = ctypes.POINTER(ctypes.c_double)
    _check(LIB.lpc_bispectrum(ctypes.byref(geom), _ptr(pos), int(pos.shape[1]), k123.ctypes.data_as(D), int(m),
                              float(dk), B.ctypes.data_as(D), Q.ctypes.data_as(D), P.ctypes.data_as(D), _ptr(ws),
                              ws.numel(), _stream(stream)))
    return B, Q, P


def lpc_cola_coefficients(cosmo, step, a_list):
    a = np.ascontiguousarray(a_list, dtype=np.float64)
    out = np.empty((a.size, len(COEF_COLUMNS)), dtype=np.float64)
    D = ctypes.POINTER(ctypes.c_double)
    _check(LIB.lpc_cola_coefficients(ctypes.byref(cosmo), ctypes.byref(step), a.ctypes.data_as(D), int(a.size),
                                     out.ctypes.data_as(D)))
    return out


def lpc_linear_power(cosmo, k):
    k = np.ascontiguousarray(k, dtype=np.float64)
    out = np.empty_like(k)
    D = ctypes.POINTER(ctypes.c_double)
    _check(LIB.lpc_linear_power(ctypes.byref(cosmo), k.ctypes.data_as(D), int(k.size), out.ctypes.data_as(D)))
    return out


def lpc_fft_pitch(n):
    return int(LIB.lpc_fft_pitch(int(n)))


def lpc_fft_r2c(n, real_in, complex_out, ws, stream=None):
    _check(LIB.lpc_fft_r2c(int(n), _ptr(real_in), _ptr(complex_out), _ptr(ws), ws.numel(), _stream(stream)))


def lpc_fft_c2r(n, complex_in, real_out, ws, stream=None):
    _check(LIB.lpc_fft_c2r(int(n), _ptr(complex_in), _ptr(real_out), _ptr(ws), ws.numel(), _stream(stream)))


def _tiling_dict(t):
    return {f: int(getattr(t, f)) for f in TILING_FIELDS}


def lpc_fft_tiling_default(n_mesh):
    """Built-in FFT tile widths of mesh size n_mesh, as a dict of the lpc_fft_tiling fields."""
    t = FftTiling()
    _check(LIB.lpc_fft_tiling_default(int(n_mesh), ctypes.byref(t)))
    return _tiling_dict(t)


def lpc_fft_tiling_get(n_mesh):
    t = FftTiling()
    _check(LIB.lpc_fft_tiling_get(int(n_mesh), ctypes.byref(t)))
    return _tiling_dict(t)


def lpc_fft_tiling_set(n_mesh, tiling):
    """Override the tile widths of n_mesh (a dict with every lpc_fft_tiling field), or remove the override (None)."""
    if tiling is None:
        _check(LIB.lpc_fft_tiling_set(int(n_mesh), None))
        return
    t = FftTiling(*(int(tiling[f]) for f in TILING_FIELDS))
    _check(LIB.lpc_fft_tiling_set(int(n_mesh), ctypes.byref(t)))


def lpc_fft_tiling_reset():
    _check(LIB.lpc_fft_tiling_reset())


# --- learned correction ---------------------------------------------------------------------------------------

def lpc_net_param_count():
    return int(LIB.lpc_net_param_count())


def lpc_net_init(seed):
    """Initial parameters (host NumPy float32)."""
    p = np.empty(lpc_net_param_count(), dtype=np.float32)
    _check(LIB.lpc_net_init(p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.c_uint64(seed)))
    return p


def lpc_net_workspace_bytes(n_side):
    return int(LIB.lpc_net_workspace_bytes(int(n_side)))


def net_workspace(n_side, device="cuda"):
    import torch
    nbytes = lpc_net_workspace_bytes(n_side)
    if nbytes == 0:
        raise LpcError(-2, f"unsupported n_side {n_side} for the network")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


NET_INPUT_CHANNELS = 6


def lpc_net_features(geom, pos, ids, out, ws, ref_pos=None, psi1=None, stream=None):
    """Input grid [N^3][6] (psi1 given) or target grid [N^3][3] (ref_pos given) into the device tensor out."""
    _check(LIB.lpc_net_features(ctypes.byref(geom), _ptr(pos), _ptr(ids), int(pos.shape[1]), _ptr(ref_pos), _ptr(psi1),
                                _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))


def lpc_net_forward(n_side, params, feat, out, ws, stream=None):
    _check(LIB.lpc_net_forward(int(n_side), _ptr(params), _ptr(feat), _ptr(out), _ptr(ws), ws.numel(),
                               _stream(stream)))


def lpc_net_loss_grad(n_side, params, feat, target, grad, ws, stream=None):
    loss = ctypes.c_double()
    _check(LIB.lpc_net_loss_grad(int(n_side), _ptr(params), _ptr(feat), _ptr(target), _ptr(grad),
                                 ctypes.byref(loss), _ptr(ws), ws.numel(), _stream(stream)))
    return float(loss.value)


def lpc_net_symmetry(n_side, k, grid, out=None, stream=None):
    """The k-th cube symmetry of a lattice field grid [n_side^3][channels] (FP32, contiguous); returns out (a new
    tensor unless given)."""
    import torch
    if grid.dtype != torch.float32 or not grid.is_contiguous() or grid.dim() != 2:
        raise ValueError("grid must be a contiguous FP32 [n_side^3][channels] tensor")
    if out is None:
        out = torch.empty_like(grid)
    elif out.shape != grid.shape or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous FP32 tensor of the grid's shape")
    if grid.shape[0] != int(n_side) ** 3:
        raise ValueError("grid must have n_side^3 rows")
    _check(LIB.lpc_net_symmetry(int(n_side), int(k), int(grid.shape[1]), _ptr(grid), _ptr(out), _stream(stream)))
    return out


def lpc_net_scale_output(params, gain, stream=None):
    """Multiply the output layer of params (device, in place) by gain."""
    _check(LIB.lpc_net_scale_output(_ptr(params), ctypes.c_float(gain), _stream(stream)))


def lpc_net_adam(params, m, v, grad, step, lr, stream=None):
    _check(LIB.lpc_net_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(step), ctypes.c_float(lr),
                            _stream(stream)))


def lpc_net_apply(geom, params, particles, ws, stream=None):
    p = particles.c_struct()
    _check(LIB.lpc_net_apply(ctypes.byref(geom), _ptr(params), ctypes.byref(p), _ptr(ws), ws.numel(),
                             _stream(stream)))


def lpc_status_string(status):
    return LIB.lpc_status_string(int(status)).decode()


def lpc_profile_enable(on=True):
    _check(LIB.lpc_profile_enable(1 if on else 0))


def lpc_profile_reset():
    _check(LIB.lpc_profile_reset())


def lpc_profile_stats():
    """{stage name: (launches, total_ms)} accumulated since the last reset."""
    out = {}
    for i in range(LIB.lpc_profile_count()):
        name = ctypes.c_char_p()
        launches = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(LIB.lpc_profile_get(i, ctypes.byref(name), ctypes.byref(launches), ctypes.byref(ms)))
        out[name.value.decode()] = (int(launches.value), float(ms.value))
    return out
