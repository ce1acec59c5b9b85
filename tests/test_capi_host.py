"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every declared symbol, and the plan's host logic agrees with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def moff():
    import paper_1510_08318_amd as m
    if not os.path.exists(m.library_path()):
        pytest.fail("libmoff.so is not built (run __graft_entry__.build())")
    return m


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "moff.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(moff_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(moff):
    lib = ctypes.CDLL(moff.library_path())
    names = declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    from paper_1510_08318_amd import _lib
    assert set(names) == set(_lib.SIGNATURES)


def test_abi_version_and_status_strings(moff):
    from paper_1510_08318_amd import _lib
    assert _lib.moff_abi_version() == 1
    for s in range(7):
        assert len(_lib.moff_status_str(s)) > 0


def host_plan(moff, geom):
    return moff.Plan.from_geometry(geom, device=-1)


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5])
def test_cells_bit_exact_vs_oracle(moff, cfg):
    w = synth.make_config(cfg, n_time=1, n_chan=4 if cfg != 1 else 1)
    P = oracle.plan(w.geom)
    with host_plan(moff, w.geom) as p:
        cells = p.cells()
        assert p.cell_m() == P["cell_m"]                       # bit-exact float64
        assert np.array_equal(cells[:, 0], P["ix0"])
        assert np.array_equal(cells[:, 1], P["iy0"])
        assert np.array_equal(p.lm_per_pixel(), P["lm_per_pixel"])


def test_cells_exact_ties(moff):
    cell = 0.5
    xy = np.array([[0.25, -0.25], [-1.25, 0.75], [2.0, -3.0], [1.75, 0.0], [0.0, 0.0], [0.5, 0.5]])
    kern = [np.ones((1, 1), np.complex64), np.ones((2, 2), np.complex64), np.ones((3, 3), np.complex64)]
    types = np.array([0, 1, 2, 0, 1, 2], np.int32)
    geom = synth.Geometry(ant_xy=xy, ktype_k=[1, 2, 3], ktype_vals=kern, ant_ktype=types,
                          freq_hz=np.array([50e6]), grid_n=64, cell_m=cell)
    P = oracle.plan(geom)
    with host_plan(moff, geom) as p:
        c = p.cells()
    assert np.array_equal(c[:, 0], P["ix0"]) and np.array_equal(c[:, 1], P["iy0"])


@pytest.mark.parametrize("cfg", [1, 5])
def test_power_patterns_vs_oracle(moff, cfg):
    w = synth.make_config(cfg, n_time=1, n_chan=1)
    with host_plan(moff, w.geom) as p:
        for t, K in enumerate(w.geom.ktype_vals):
            ref = oracle.power_pattern(K, w.geom.grid_n)
            got = p.power_pattern(t)
            assert np.max(np.abs(got - ref)) <= 1e-12 * ref.max()


def _status_of(moff, fn):
    with pytest.raises(moff.MoffError) as ei:
        fn()
    return ei.value.status


def test_error_codes(moff):
    w = synth.make_config(1, n_time=1)
    g = w.geom
    mk = lambda **kw: moff.Plan(**{**dict(ant_xy=g.ant_xy, ktype_k=g.ktype_k, ktype_vals=g.ktype_vals,
                                          ant_ktype=g.ant_ktype, freq_hz=g.freq_hz, grid_n=g.grid_n,
                                          cell_m=0.0, flags=g.flags, device=-1), **kw})
    assert _status_of(moff, lambda: mk(grid_n=48)) == 2
    assert _status_of(moff, lambda: mk(grid_n=512)) == 2
    with mk(grid_n=8) as p8:                                     # the default rule widens the cell to fit
        span = max(np.ptp(g.ant_xy[:, 0]), np.ptp(g.ant_xy[:, 1]))
        assert p8.cell_m() == span / (4 - 2 - 1)
    assert _status_of(moff, lambda: mk(cell_m=0.1)) == 3         # explicit fine grid: array does not fit
    assert _status_of(moff, lambda: mk(flags=64)) == 1
    assert _status_of(moff, lambda: mk(ant_ktype=np.full(16, 3, np.int32))) == 1
    assert _status_of(moff, lambda: mk(freq_hz=np.array([-1.0]))) == 1
    assert _status_of(moff, lambda: mk(ant_xy=g.ant_xy[:1], ant_ktype=g.ant_ktype[:1])) == 1
    # compute calls on a host-only plan are refused before touching any device
    from paper_1510_08318_amd import _lib
    with mk() as p:
        st = _lib.lib().moff_image(p.handle, None, 1, None, None, None)
        assert st == 4


@pytest.mark.parametrize("case", ["config1", "config2", "config3", "config5", "hetero_small", "n8", "n16"])
def test_gather_program_replays_oracle_grid(moff, case):
    """Replaying the fused kernel's gather program on the CPU (float64) gives the
    oracle's gridded field, transposed (folded-grid row = aperture column x) and
    folded along y onto the workgroup's class of image rows."""
    rng = np.random.default_rng(5)
    if case == "config1":
        w = synth.make_config(1, n_time=2)
    elif case == "config2":
        w = synth.make_config(2, n_time=2, n_chan=1)
    elif case == "config3":
        w = synth.make_config(3, n_time=1, n_chan=1)
    elif case == "config5":
        w = synth.make_config(5, n_time=1, n_chan=1)
    elif case == "hetero_small":
        w = synth.random_case(3, 9, 32, 1, 2, [synth.random_kernel(rng, 3), synth.random_kernel(rng, 2)],
                              extent_m=4.0, cell_m=1.0)
    else:
        N = 8 if case == "n8" else 16
        w = synth.random_case(4, 5, N, 1, 2, [synth.random_kernel(rng, 2)], extent_m=1.5, cell_m=1.0)
    P = oracle.plan(w.geom)
    e = oracle.calibrated_field(w.E, w.gains, w.geom.flags, 0)
    Eg = oracle.grid_field(e, P)[0].T           # [ix][iy]: the fused programs' transposed aperture
    N, L = P["N"], P["L"]
    with host_plan(moff, w.geom) as p:
      for variant in (0, 1):
        if variant == 1 and N not in (128, 256):
            continue
        prog0, _, info = p.gather_program(0, variant)
        SX = info["n_classes"]
        M = N // SX
        NZR = min(L, M)
        ZP = info["row_pitch"]
        ev = np.concatenate([e[0], [0.0]])
        for cls in range(SX):
            prog, wts, info = p.gather_program(cls, variant)
            x = prog[..., 0].astype(np.int64)
            y = prog[..., 1].astype(np.int64)
            ant = x & 0xFFF
            wi = (x >> 12) & 0x7FF
            st = (x >> 31) & 1
            assert ant.max() <= w.geom.n_ant and wi.max() < len(wts)
            G = np.full(L * ZP, np.nan, complex)
            stored = np.zeros(L * ZP, int)
            acc = np.zeros(prog.shape[1], complex)
            for k in range(prog.shape[0]):
                acc = acc + ev[ant[k]] * wts[wi[k]].astype(np.complex128)
                s = st[k] == 1
                assert (y[k][s] < L * ZP).all()
                G[y[k][s]] = acc[s]
                stored[y[k][s]] += 1
                acc[s] = 0
            # folded reference: sum_j exp(2 pi i j w / SX) Eg^T[ix, n + j M]
            ref = np.zeros((L, NZR), complex)
            for j in range(max(1, L // M)):
                ref += np.exp(2j * np.pi * j * cls / SX) * Eg[:, j * M:j * M + NZR]
            iy = np.arange(L)[:, None]
            n = np.arange(NZR)[None, :]
            slot = iy * ZP + n
            got = G[slot]
            assert (stored[slot] == 1).all() and stored.sum() == L * NZR
            assert np.max(np.abs(got - ref)) <= 1e-6 * max(1.0, np.abs(ref).max())
            # The device keeps only the x words: a lane's k-th store goes to the
            # folded cell after its first one, so each lane's stores must fill
            # consecutive cells (row-major over (iy, n')), and batches of four
            # entries must tile the program.
            assert prog.shape[0] % 4 == 0
            for lane in range(prog.shape[1]):
                dst = y[:, lane][st[:, lane] == 1]
                if len(dst) == 0:
                    continue
                cells = (dst // ZP) * NZR + dst % ZP
                assert (dst % ZP < NZR).all()
                assert (np.diff(cells) == 1).all(), (cls, lane)


def test_uv_rule_flag_validation(moff):
    w = synth.make_config(1, n_time=2)
    with pytest.raises(moff.MoffError) as ei:
        moff.Plan.from_geometry(w.geom, device=-1, extra_flags=synth.AUTOCORR_UV | synth.AUTOCORR_NONE)
    assert ei.value.status == 1
    with moff.Plan.from_geometry(w.geom, device=-1, extra_flags=synth.AUTOCORR_UV) as p:
        assert p.N == 32


def test_host_only_plan_rejects_compute(moff):
    """A plan built without a device answers compute calls with
    MOFF_ERR_UNSUPPORTED before touching any device."""
    from paper_1510_08318_amd import _lib
    w = synth.make_config(1, n_time=2)
    with moff.Plan.from_geometry(w.geom, device=-1) as p:
        L = _lib.lib()
        dummy = ctypes.c_void_p(16)
        assert L.moff_image(p.handle, dummy, 2, None, dummy, None) == 4
        assert L.moff_accumulate(p.handle, dummy, 2, None, dummy, dummy, None) == 4
        assert L.moff_gain_vjp(p.handle, dummy, 2, None, dummy, dummy, None) == 4
        assert L.moff_image_staged(p.handle, dummy, 2, None, dummy, None) == 4


def test_wave_owned_rows_hera(moff):
    """On the HERA-shaped layout the 512-thread shape's program gives every wave
    exactly the 16 folded rows that wave transforms in the row stage (wave w:
    rows 8 w .. 8 w + 7 from the upper half and 8 (8 + (w xor 1)) .. + 7 from
    the lower half), which lets the kernel skip the workgroup barrier between
    the gather and the row stage; every row is covered."""
    w = synth.make_config(3, n_time=1, n_chan=1)
    with host_plan(moff, w.geom) as p:
        for cls in range(2):
            prog, _, info = p.gather_program(cls, 1)
            assert info["n_threads"] == 512
            ZP = info["row_pitch"]
            x, y = prog[..., 0], prog[..., 1]
            rows_seen = set()
            for lane in range(512):
                dst = y[:, lane][(x[:, lane] >> 31) == 1]
                rows = set((dst // ZP).tolist())
                wave = lane // 64
                lower = 8 * (8 + (wave ^ 1))
                own = set(range(8 * wave, 8 * wave + 8)) | set(range(lower, lower + 8))
                assert rows <= own, (cls, lane)
                rows_seen |= rows
            assert rows_seen == set(range(128))
