"""CPU-only checks of the C ABI: the library loads, exports every symbol include/lpc.h declares, host-only entry
points agree with the oracle, and argument errors come back as status codes (no GPU call is made)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import cosmology as ocosmo
from oracle import ic as oic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpc.h")
LIBFILE = os.path.join(ROOT, "paper_1506_03737_amd", "liblpc.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIBFILE), reason="liblpc.so not built")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\*]+\s+)+\**(lpc_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIBFILE)
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_1506_03737_amd import lpc
    assert set(declared_functions()) == set(lpc.EXPORTED)


@pytest.mark.parametrize("modified", [0, 1])
def test_coefficients_match_oracle(modified):
    from paper_1506_03737_amd import lpc
    c = synth.COSMOLOGY
    step = lpc.stepping(modified=modified)
    got = lpc.lpc_cola_coefficients(lpc.cosmology(**c), step, synth.A_LIST)
    ref = ocosmo.coefficient_table(synth.A_LIST, c["omega_m"], bool(modified), -2.5)
    assert got.shape == ref.shape
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-14)


def test_coefficients_eds_closed_form():
    from paper_1506_03737_amd import lpc
    got = lpc.lpc_cola_coefficients(lpc.cosmology(omega_m=1.0), lpc.stepping(modified=0), [0.25, 0.5, 1.0])
    assert got[0, 7] == pytest.approx(2 * (0.25**-0.5 - 0.5**-0.5), rel=1e-13)       # Q
    assert got[1, 6] == pytest.approx(2 * (0.75**0.5 - 0.375**0.5), rel=1e-13)      # K
    assert got[2, 1] == pytest.approx(1.0, rel=1e-13)                               # D1(1)


def test_comoving_distance_matches_oracle():
    from oracle import lightcone as olc
    from paper_1506_03737_amd import lpc
    c = synth.COSMOLOGY
    a = np.array([0.1, 0.55, 0.82, 0.91, 0.999, 1.0])
    got = lpc.lpc_comoving_distance(lpc.cosmology(**c), a)
    ref = np.array([olc.comoving_distance(x, c["omega_m"]) for x in a])
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-9)
    with pytest.raises(lpc.LpcError):
        lpc.lpc_comoving_distance(lpc.cosmology(**c), [1.5])


def test_linear_power_matches_oracle():
    from paper_1506_03737_amd import lpc
    c = synth.COSMOLOGY
    k = np.logspace(-3, 1, 40)
    got = lpc.lpc_linear_power(lpc.cosmology(**c), k)
    ref = oic.linear_pk(k, **c)
    assert np.allclose(got, ref, rtol=1e-9)


def test_workspace_sizes_and_rejections():
    from paper_1506_03737_amd import lpc
    g = lpc.geometry(32, 64, 256.0)
    n = 32**3
    cola = lpc.lpc_workspace_bytes(g, lpc.LPC_OP_COLA_STEP, n)
    force = lpc.lpc_workspace_bytes(g, lpc.LPC_OP_PM_FORCE, n)
    assert force > 64**3 * 12 + 3 * 64 * 64 * 40 * 8 + 16 * n      # meshes + one sorted copy (pos, index)
    assert cola - force == 2 * 52 * n - 16 * n                       # two full sorted copies instead of one
    assert lpc.lpc_workspace_bytes(g, lpc.LPC_OP_COLA_STEP, 0) == 0  # a particle op needs a particle count
    assert lpc.lpc_workspace_bytes(g, lpc.LPC_OP_FFT, 0) > 0
    assert lpc.lpc_workspace_bytes(g, 99, n) == 0
    assert lpc.lpc_workspace_bytes(lpc.geometry(32, 14, 256.0), lpc.LPC_OP_PM_FORCE, n) == 0   # 7 is not 2/3/5-smooth
    assert lpc.lpc_workspace_bytes(lpc.geometry(32, 2048, 256.0), lpc.LPC_OP_PM_FORCE, n) == 0
    assert lpc.lpc_fft_pitch(768) == 392 and lpc.lpc_fft_pitch(64) == 40


def test_batched_workspace_layout():
    """Flags + job region, then per box 12 Nm^3 bytes (int64 counts / AoS float3 force) and three half spectra, then
    the sort space (two tile-sorted copies of every box's pos/vel/psi1/psi2/index, keys, ranks, tile counts and
    starts), each array 256-byte aligned; an unsupported mesh anywhere in the batch gives 0."""
    from paper_1506_03737_amd import lpc

    def entry(nm, n, box=100.0):
        e = lpc.BatchEntry()
        e.geom = lpc.geometry(0, nm, box)
        e.particles.n = n
        return e

    def r256(x):
        return (x + 255) // 256 * 256

    def per_box(nm):
        return r256(12 * nm**3) + 3 * r256(nm * nm * lpc.lpc_fft_pitch(nm) * 8)

    def sort_space(nms, ns):
        copies = 2 * sum(4 * r256(12 * n) + r256(4 * n) for n in ns)
        # two buckets per tile of 16 x 8 x 32 cells, plus one per box
        G = sum(2 * (-(-nm // 16)) * (-(-nm // 8)) * (-(-nm // 32)) + 1 for nm in nms)
        return copies + 2 * r256(4 * sum(ns)) + r256(4 * G) + r256(4 * (G + 1)) + r256(4 * -(-G // 2048))

    one = (lpc.BatchEntry * 1)(entry(64, 1000))
    base = lpc.LIB.lpc_workspace_bytes_batched(one, 1) - per_box(64) - sort_space([64], [1000])
    assert base == 256 + (1 << 20)
    arr = (lpc.BatchEntry * 3)(entry(192, 96**3), entry(40, 777), entry(320, 160**3))
    want = base + per_box(192) + per_box(40) + per_box(320) + sort_space([192, 40, 320], [96**3, 777, 160**3])
    assert lpc.LIB.lpc_workspace_bytes_batched(arr, 3) == want
    arr[1] = entry(14, 777)
    assert lpc.LIB.lpc_workspace_bytes_batched(arr, 3) == 0
    arr[1] = entry(40, 0)
    assert lpc.LIB.lpc_workspace_bytes_batched(arr, 3) == 0
    assert lpc.LIB.lpc_workspace_bytes_batched(arr, 0) == 0


def test_argument_errors_are_status_codes():
    from paper_1506_03737_amd import lpc
    c = lpc.cosmology()
    with pytest.raises(lpc.LpcError) as e:
        lpc.lpc_cola_coefficients(c, lpc.stepping(), [0.5, 0.4])
    assert e.value.status == -1 and "increasing" in str(e.value)
    with pytest.raises(lpc.LpcError) as e:
        lpc.lpc_cola_coefficients(lpc.cosmology(omega_m=-1.0), lpc.stepping(), [0.1, 0.2])
    assert e.value.status == -1
    # unsupported mesh: rejected before any device work
    lib = lpc.LIB
    g = lpc.geometry(32, 14, 256.0)
    st = lib.lpc_pm_force(ctypes.byref(g), ctypes.byref(lpc.stepping()), ctypes.c_void_p(8), 10,
                          ctypes.c_void_p(8), None, ctypes.c_void_p(256), 1 << 20, None)
    assert st == -2
    # workspace too small / misaligned
    g = lpc.geometry(32, 64, 256.0)
    st = lib.lpc_pm_force(ctypes.byref(g), ctypes.byref(lpc.stepping()), ctypes.c_void_p(8), 10,
                          ctypes.c_void_p(8), None, ctypes.c_void_p(256), 1024, None)
    assert st == -3
    st = lib.lpc_pm_force(ctypes.byref(g), ctypes.byref(lpc.stepping()), ctypes.c_void_p(8), 10,
                          ctypes.c_void_p(8), None, ctypes.c_void_p(100), 1 << 30, None)
    assert st == -3
    # deconvolution power out of range, n = 0, NULL positions
    st = lib.lpc_pm_force(ctypes.byref(g), ctypes.byref(lpc.stepping(deconv_power=3)), ctypes.c_void_p(8), 10,
                          ctypes.c_void_p(8), None, ctypes.c_void_p(256), 1 << 30, None)
    assert st == -1
    st = lib.lpc_pm_force(ctypes.byref(g), ctypes.byref(lpc.stepping()), ctypes.c_void_p(8), 0,
                          ctypes.c_void_p(8), None, ctypes.c_void_p(256), 1 << 30, None)
    assert st == -1
    st = lib.lpc_pm_force(ctypes.byref(g), ctypes.byref(lpc.stepping()), None, 10,
                          ctypes.c_void_p(8), None, ctypes.c_void_p(256), 1 << 30, None)
    assert st == -1
    assert lpc.lpc_status_string(-5) == "LPC_ERR_FIXED_OVERFLOW"
    # init_ic with mismatched particle count
    p = lpc.Particles(8, 8, 8, 8, 8, 100)
    st = lib.lpc_init_ic(ctypes.byref(g), ctypes.byref(c), 1, 0.1, ctypes.byref(p), ctypes.c_void_p(256), 1 << 30,
                         None)
    assert st == -1 and b"n_side^3" in lib.lpc_last_error()


def test_net_parameter_count_and_workspace_sizes():
    from oracle import net as onet
    from paper_1506_03737_amd import lpc
    assert lpc.lpc_net_param_count() == onet.param_count()
    p = lpc.lpc_net_init(7)
    assert p.shape == (onet.param_count(),) and np.all(np.isfinite(p))
    sl = onet.layer_slices()
    assert np.all(p[sl["e0b"][1]] == 0.0)                          # biases start at zero
    assert np.abs(p[sl["e0b"][0]]).max() <= np.sqrt(6.0 / (27 * 16)) + 1e-7
    assert np.array_equal(p, lpc.lpc_net_init(7)) and not np.array_equal(p, lpc.lpc_net_init(8))
    assert lpc.lpc_net_workspace_bytes(16) > 0 and lpc.lpc_net_workspace_bytes(6) == 0
    assert lpc.lpc_net_workspace_bytes(18) == 0 and lpc.lpc_net_workspace_bytes(1024) == 0


def _supported_meshes():
    def smooth(n):
        for r in (2, 3, 5):
            while n % r == 0:
                n //= r
        return n == 1
    return [n for n in range(8, 1025, 2) if smooth(n)]


def _fits(field, n, w):
    """Capacity of the FFT tiles, restated from the kernels' limits: 512 threads, 16 complex values per thread per
    stage (8192 per tile), one extra value per thread in the z passes' loads, 160 KiB of LDS (8-byte complex)."""
    h = n // 2
    lds = 160 * 1024

    def rows(B):
        return B * (h + 1) <= 8192 + 512 and h * B <= 16 * (512 // B) * B

    if field == "z_rows":
        return (w in (8, 16, 32) and rows(w) and 8 * (h * (w + 1) + 2 * h + 1) <= lds
                and 8 * ((h + 1) * (w + 1) + 2 * h + 1) <= lds)
    pitch = w if w == 8 else w + 1  # row pitch of a strided tile (8-column tiles unpadded)
    if field == "axis_cols":
        return w in (8, 16, 32) and n * w <= 8192 and 8 * (n * pitch + n) <= lds
    if field == "poisson_cols":
        # the transformed delta_hat stays in registers (one LDS tile) up to 12 points per thread, else a second tile
        tiles = 1 if -(-n * w // 512) <= 12 else 2
        return w in (4, 8, 16) and n * w <= 8192 and 8 * (tiles * n * pitch + n) + 4 * (h + 1) <= lds
    return w in (4, 8, 16) and rows(3 * w) and 8 * ((h + 1) * (3 * w + 1) + 2 * h + 1) <= lds


def test_fft_tiling_defaults_overrides_and_rejections():
    from paper_1506_03737_amd import lpc
    lpc.lpc_fft_tiling_reset()
    fields = lpc.TILING_FIELDS
    try:
        for n in _supported_meshes():
            d = lpc.lpc_fft_tiling_default(n)
            assert lpc.lpc_fft_tiling_get(n) == d
            for f in fields:
                assert _fits(f, n, d[f]), (n, f, d[f])
                for w in (0, 2, 4, 8, 12, 16, 32, 64):
                    ok = _fits(f, n, w)
                    try:
                        lpc.lpc_fft_tiling_set(n, dict(d, **{f: w}))
                        accepted = True
                    except lpc.LpcError as e:
                        accepted = False
                        assert e.status == -1 and f in str(e)
                    assert accepted == ok, (n, f, w)
                lpc.lpc_fft_tiling_set(n, None)
        # the largest widths that fit the single-box mesh
        assert lpc.lpc_fft_tiling_default(768) == dict(z_rows=16, axis_cols=8, poisson_cols=8, c2r_rows=4)
        # an override sticks, a rejected one leaves it in place, None and reset remove it
        t = dict(z_rows=8, axis_cols=8, poisson_cols=4, c2r_rows=4)
        lpc.lpc_fft_tiling_set(768, t)
        with pytest.raises(lpc.LpcError):
            lpc.lpc_fft_tiling_set(768, dict(t, axis_cols=16))
        assert lpc.lpc_fft_tiling_get(768) == t
        assert lpc.lpc_fft_tiling_get(384) == lpc.lpc_fft_tiling_default(384)
        lpc.lpc_fft_tiling_set(768, None)
        assert lpc.lpc_fft_tiling_get(768) == lpc.lpc_fft_tiling_default(768)
        lpc.lpc_fft_tiling_set(768, t)
        lpc.lpc_fft_tiling_reset()
        assert lpc.lpc_fft_tiling_get(768) == lpc.lpc_fft_tiling_default(768)
        for bad in (7, 14, 1026, 0, -8):
            with pytest.raises(lpc.LpcError) as e:
                lpc.lpc_fft_tiling_default(bad)
            assert e.value.status == -2
    finally:
        lpc.lpc_fft_tiling_reset()


def test_net_entry_points_reject_misaligned_params():
    """The network's down/up layers read weights as 16-byte vectors: a params pointer off a 16-byte boundary is an
    argument error, reported before any device work (the fake pointers below are never dereferenced)."""
    from paper_1506_03737_amd import lpc
    lib = lpc.LIB
    loss = ctypes.c_double()
    vp = ctypes.c_void_p
    bad = vp(0x100004)
    ok = vp(0x100000)
    st = lib.lpc_net_forward(16, bad, ok, ok, ok, 1 << 20, None)
    assert st == -1 and b"16-byte" in lib.lpc_last_error()
    st = lib.lpc_net_loss_grad(16, bad, ok, ok, ok, ctypes.byref(loss), ok, 1 << 20, None)
    assert st == -1 and b"16-byte" in lib.lpc_last_error()


def test_png_presets_match_oracle():
    from oracle import png as opng
    from paper_1506_03737_amd import lpc
    for kind, terms in opng.PRESETS.items():
        p = lpc.png(12.5, kind=kind)
        assert p.f_nl == 12.5 and p.n_terms == len(terms) and p.reserved == 0
        got = [(p.terms[t].c, p.terms[t].a, p.terms[t].b, p.terms[t].g) for t in range(p.n_terms)]
        assert got == [tuple(map(float, t)) for t in terms]
    with pytest.raises(lpc.LpcError):
        lpc._check(lpc.LIB.lpc_png_preset(7, 1.0, ctypes.byref(lpc.Png())))


def test_net_symmetry_rejects_bad_arguments():
    """Argument checks of lpc_net_symmetry run before any device work: k and channels out of range, aliasing."""
    import ctypes
    from paper_1506_03737_amd import lpc
    n, C = 4, 6
    a = ctypes.create_string_buffer(n**3 * C * 4 * 2)
    base = ctypes.addressof(a)
    other = base + n**3 * C * 4
    for args in ((n, 48, C, base, other), (n, -1, C, base, other), (n, 0, 4, base, other), (n, 0, 51, base, other),
                 (0, 0, C, base, other), (n, 0, C, base, base + 8), (n, 0, C, None, other)):
        st = lpc.LIB.lpc_net_symmetry(*args, None)
        assert st == -1, args  # LPC_ERR_INVALID_ARG


def test_bispectrum_arguments_and_workspace():
    """lpc_bispectrum's checks run before any device work; its workspace holds the P(k) path's plus three real
    meshes and a spectrum."""
    from paper_1506_03737_amd import lpc
    g = lpc.geometry(0, 64, 500.0)
    wb = lpc.lpc_workspace_bytes(g, lpc.LPC_OP_BISPECTRUM, 1000)
    wp = lpc.lpc_workspace_bytes(g, lpc.LPC_OP_POWER_SPECTRUM, 1000)
    assert wb >= wp + 3 * 64**3 * 4 + 64 * 64 * lpc.lpc_fft_pitch(64) * 8
    assert lpc.lpc_workspace_bytes(g, lpc.LPC_OP_BISPECTRUM, 0) == 0
    D = ctypes.POINTER(ctypes.c_double)
    k = (ctypes.c_double * 6)(0.1, 0.1, 0.1, 0.1, 0.2, 0.0)
    out = (ctypes.c_double * 8)()
    fake = ctypes.c_void_p(0x100000)
    lib = lpc.LIB
    for args in ((fake, 1000, k, 1, 0.0), (fake, 1000, k, 0, 0.01), (fake, 1000, k, 257, 0.01),
                 (fake, 1000, k, 2, 0.01), (fake, 0, k, 1, 0.01), (None, 1000, k, 1, 0.01)):
        st = lib.lpc_bispectrum(ctypes.byref(g), args[0], args[1], ctypes.cast(args[2], D), args[3], args[4],
                                ctypes.cast(out, D), ctypes.cast(out, D), None, fake, 1 << 30, None)
        assert st == -1, args


def test_autotune_pick_prefers_the_wider_of_tied_widths():
    """The tuner's choice from one round of timings: the fastest width, unless a wider one is within 3 % of it."""
    from paper_1506_03737_amd import autotune
    assert autotune.pick({8: 0.100, 16: 0.200, 32: 0.300}) == 8
    assert autotune.pick({4: 0.178, 8: 0.1799, 16: 0.1846}) == 8      # 8 within 1.1 %, 16 at 3.7 %
    assert autotune.pick({8: 0.0805, 16: 0.0578, 32: 0.058}) == 32     # 16 and 32 tied
    assert autotune.pick({4: 0.190, 8: 0.092, 16: 0.111}) == 8         # a narrower fastest width still wins
    assert autotune.pick({8: 1.0}) == 8
    assert autotune.pick({8: 0.1, 16: 0.1, 32: 0.1}, tie=0.0) == 32
