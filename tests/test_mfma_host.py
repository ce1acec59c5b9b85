"""Host-side checks of the reduced-precision (matrix-core) path's tables:
plan validation, the gather program over non-empty aperture cells replayed on
the CPU against the oracle's gridded field, and the 16-bit phase-factor operands
against their definition, correctly rounded."""
import numpy as np
import pytest

import oracle
import synth

MFMA = {"f16": synth.MFMA_F16, "bf16": synth.MFMA_BF16}


@pytest.fixture(scope="module")
def moff():
    import paper_1510_08318_amd as m
    m._lib.lib()
    return m


def _case(name):
    rng = np.random.default_rng(9)
    if name == "config2_n128":
        return synth.make_config(2, n_time=2, n_chan=1)
    if name == "config2_n64":
        return synth.make_config(2, n_time=2, n_chan=1, grid_n=64)
    if name == "hetero_n64":
        return synth.random_case(6, 40, 64, 1, 2, [synth.random_kernel(rng, 3), synth.random_kernel(rng, 5)],
                                 extent_m=40.0, cell_m=1.5)
    return synth.make_config(5, n_time=1, n_chan=1, grid_n=128)


def test_lds_bound_on_antennas(moff):
    """On the 128 grid the double-buffered LDS layout bounds the antenna count:
    4000 antennas are rejected at plan creation (MOFF_ERR_UNSUPPORTED), 1400 fit."""
    rng = np.random.default_rng(40)
    tabs = [synth.random_kernel(rng, 3), synth.random_kernel(rng, 1)]
    for n_ant, ok in ((4000, False), (1400, True)):
        w = synth.random_case(41, n_ant, 128, 1, 2, tabs, extent_m=60 * 0.8, cell_m=0.8)
        if ok:
            with moff.Plan.from_geometry(w.geom, device=-1, extra_flags=synth.MFMA_F16):
                pass
        else:
            with pytest.raises(moff.MoffError) as ei:
                moff.Plan.from_geometry(w.geom, device=-1, extra_flags=synth.MFMA_F16)
            assert ei.value.status == 4


def test_plan_validation(moff):
    w = synth.make_config(1, n_time=2)       # grid_n 32
    with pytest.raises(moff.MoffError) as ei:
        moff.Plan.from_geometry(w.geom, device=-1, extra_flags=synth.MFMA_F16)
    assert ei.value.status == 4               # MOFF_ERR_UNSUPPORTED: only grid_n 64 and 128
    w = synth.make_config(2, n_time=2, n_chan=1)
    with pytest.raises(moff.MoffError) as ei:
        moff.Plan.from_geometry(w.geom, device=-1, extra_flags=synth.MFMA_F16 | synth.MFMA_BF16)
    assert ei.value.status == 1               # MOFF_ERR_INVALID_ARG: both precisions
    with moff.Plan.from_geometry(w.geom, device=-1) as p:
        with pytest.raises(moff.MoffError) as ei:
            p.mfma_tables()
        assert ei.value.status == 4


@pytest.mark.parametrize("name", ["config2_n128", "config2_n64", "hetero_n64", "config5_n128"])
def test_mfma_gather_program_replays_oracle_grid(moff, name):
    w = _case(name)
    P = oracle.plan(w.geom)
    N, L = P["N"], P["L"]
    e = oracle.calibrated_field(w.E, w.gains, w.geom.flags, 0)[0]
    Eg = oracle.grid_field(e[None], P)[0]
    taps = np.concatenate([np.asarray(K, np.complex64).ravel() for K in P["kernels"]]).astype(np.complex128)
    with moff.Plan.from_geometry(w.geom, device=-1, extra_flags=synth.MFMA_F16) as p:
        prog, _, info = p.mfma_tables()
    pitch, base, na = info["row_pitch"], info["grid_base"], w.geom.n_ant
    assert info["n_threads"] == (256 if N == 128 else 128) and pitch == 2 * L + 8   # gather lanes
    assert base % 16 == 0 and base >= 8 * (2 * (na + 1) + len(taps))
    x = prog[..., 0].astype(np.int64)
    y = prog[..., 1].astype(np.int64)
    eoff, koff = x & 0xFFFF, x >> 16
    assert (eoff % 8 == 0).all() and (koff % 8 == 0).all()
    ant, tap = eoff // 8, koff // 8 - 2 * (na + 1)   # taps follow two sample buffers
    st = y != 0
    assert ant.max() <= na and tap.min() >= 0 and tap.max() < len(taps)
    slot = (y - base) // 2
    assert ((y[st] - base) % 2 == 0).all() and (slot[st] >= 0).all() and (slot[st] + L < L * pitch).all()
    ev = np.concatenate([e, [0.0]])
    G = np.zeros(L * pitch, complex)
    stored = np.zeros(L * pitch, int)
    acc = np.zeros(prog.shape[1], complex)
    for k in range(prog.shape[0]):
        acc = acc + ev[ant[k]] * taps[tap[k]]
        s = st[k]
        G[slot[k][s]] = acc[s]
        stored[slot[k][s]] += 1
        acc[s] = 0
    # every lane ends on a stored cell (no partial sum is dropped)
    assert np.all(np.abs(acc) == 0)
    slot = np.arange(L)[:, None] * pitch + np.arange(L)[None, :]
    # cells some nonzero table entry reaches (exactly-zero entries are not gridded)
    nonempty = np.zeros((L, L), bool)
    for a in range(w.geom.n_ant):
        K = np.asarray(P["kernels"][P["ant_ktype"][a]])
        k = K.shape[0]
        nonempty[P["iy0"][a]:P["iy0"][a] + k, P["ix0"][a]:P["ix0"][a] + k] |= K != 0
    assert (stored[slot] == nonempty.astype(int)).all() and stored.sum() == nonempty.sum()
    assert np.max(np.abs(G[slot] - Eg)) <= 1e-6 * max(1.0, np.abs(Eg).max())


def _phase(j, n, N):
    """exp(+2 pi i j (n - N/2) / N), exact on the quarter turns."""
    m = np.mod(j * (n - N // 2), N)
    c, s = np.cos(2 * np.pi * m / N), np.sin(2 * np.pi * m / N)
    q = (4 * m) % N == 0
    c = np.where(q, np.round(c), c)
    s = np.where(q, np.round(s), s)
    return c + 1j * s


def _expected_operands(N):
    """float64 [2, N/64, 2, N/64, 2, 64, 8] operand values by their definition:
    the base half (index n < N/2) of each transform's phase vectors, real part
    then imaginary part; index 0 carries the two real self-conjugate vectors, of
    n - N/2 = -N/2 (real part) and of n - N/2 = 0 (imaginary part)."""
    L, NRB, KS2 = N // 2, N // 64, N // 64
    st, b, hf, ks, part, ln, i = np.meshgrid(np.arange(2), np.arange(NRB), np.arange(2), np.arange(KS2),
                                             np.arange(2), np.arange(64), np.arange(8), indexing="ij")
    j = 32 * ks + 8 * (ln // 16) + i
    n = 32 * b + 16 * hf + ln % 16
    f = _phase(j, n, N)
    shared = _phase(j, 0, N).real + 1j * _phase(j, L, N).real
    f = np.where(n == 0, shared, f) * np.where(st == 0, 1.0 / L, 1.0)
    return np.where(part == 0, f.real, f.imag)


def test_conjugate_pairs_give_the_full_transform():
    """The pairing the tables rely on, checked in float64 on a random input: the
    four real products of the base half reproduce the full complex matrix
    product for the base rows, their conjugate partners N - n, and the two real
    self-conjugate rows through the shared slot."""
    rng = np.random.default_rng(5)
    for N in (64, 128):
        L = N // 2
        j = np.arange(L)
        full = np.stack([_phase(j, n, N) for n in range(N)])                 # [n][j]
        x = rng.standard_normal(L) + 1j * rng.standard_normal(L)
        want = full @ x
        ops = _expected_operands(N)[1]                                       # column stage, scale 1
        u = np.zeros((L, L), complex)
        for b in range(N // 64):
            for hf in range(2):
                for ks in range(N // 64):
                    for ln in range(64):
                        for i in range(8):
                            u[32 * b + 16 * hf + ln % 16, 32 * ks + 8 * (ln // 16) + i] = (
                                ops[b, hf, ks, 0, ln, i] + 1j * ops[b, hf, ks, 1, ln, i])
        P1, P2 = u.real @ x.real, u.imag @ x.imag
        P3, P4 = u.imag @ x.real, u.real @ x.imag
        base, part = (P1 - P2) + 1j * (P3 + P4), (P1 + P2) + 1j * (P4 - P3)
        assert np.allclose(base[1:], want[1:L], atol=1e-9)
        assert np.allclose(part[1:], want[N - np.arange(1, L)], atol=1e-9)
        assert np.isclose(P1[0] + 1j * P4[0], want[0]) and np.isclose(P3[0] + 1j * P2[0], want[L])


def _bf16_decode(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("N", [64, 128])
@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_mfma_phase_operands_correctly_rounded(moff, N, prec):
    w = synth.make_config(2, n_time=2, n_chan=1, grid_n=N)
    with moff.Plan.from_geometry(w.geom, device=-1, extra_flags=MFMA[prec]) as p:
        _, dft, _ = p.mfma_tables()
    exact = _expected_operands(N)
    assert dft.shape == exact.shape
    if prec == "f16":
        # numpy rounds float64 -> binary16 to nearest even in one step
        want = exact.astype(np.float16).view(np.uint16)
        zero = exact == 0
        assert np.array_equal(dft[~zero], want[~zero])
        assert np.all((dft[zero] & 0x7FFF) == 0)
    else:
        got = _bf16_decode(dft)
        ax = np.abs(exact)
        e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
        half_ulp = np.where(ax > 0, 2.0 ** (e - 8), 0.0)
        assert np.all(np.abs(got - exact) <= half_ulp)
        assert np.all(np.sign(got) * np.sign(exact) >= 0)
