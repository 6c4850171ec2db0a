"""Pins of the FP64 oracle against facts fixed by mathematics and by the paper.

Each test names the property it pins.  A plausible mistake in the oracle (a
dropped term, a wrong sign or index, a transposed operand, a wrong scale)
fails at least one of them:

* brute force: recursive FFT == direct O(N^2) DFT for every N = 2..512;
* library routine: == numpy.fft (pocketfft), an independent implementation;
* invariants: Parseval, inverse round trip, linearity;
* closed forms: DC, alternating, impulse, the quadratic Gauss sum;
* the paper's overflow mechanism (Sec. III-B) and BFP fix (Eq. (1));
* adjoint identity and entropy-gradient invariance for autofocus.
"""
import numpy as np
import pytest

import oracle
from paper_2605_28451_amd import scenes


def _rand(rows, n, seed):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((2, rows, n))
    return g[0] + 1j * g[1]


@pytest.mark.parametrize("n", [2 ** k for k in range(1, 10)])
def test_fft_matches_direct_dft(n):
    x = _rand(1, n, n)[0]
    X = oracle.fft(x[None])[0]
    D = oracle.dft_direct(x)
    assert np.max(np.abs(X - D)) <= 1e-12 * n * np.max(np.abs(x))
    Xi = oracle.fft(x[None], inverse=True)[0]
    Di = oracle.dft_direct(x, inverse=True)
    assert np.max(np.abs(Xi - Di)) <= 1e-12 * np.max(np.abs(x))


def test_direct_dft_odd_length_closed_form():
    # a non-power-of-two length exercises the exact argument reduction
    n = 12
    x = np.zeros(n, complex)
    x[5] = 1.0
    D = oracle.dft_direct(x)
    k = np.arange(n)
    assert np.allclose(D, np.exp(-2j * np.pi * 5 * k / n), atol=1e-15)


@pytest.mark.parametrize("n", [8, 256, 4096, 16384])
def test_fft_matches_numpy(n):
    x = _rand(3, n, 7)
    X = oracle.fft(x)
    ref = np.fft.fft(x, axis=-1)
    rel = np.linalg.norm(X - ref) / np.linalg.norm(ref)
    assert rel <= 1e-13


@pytest.mark.parametrize("n", [64, 4096])
def test_parseval_and_round_trip(n):
    x = _rand(4, n, 11)
    X = oracle.fft(x)
    assert abs(np.sum(np.abs(X) ** 2) - n * np.sum(np.abs(x) ** 2)) <= 1e-13 * n * np.sum(np.abs(x) ** 2)
    back = oracle.fft(X, inverse=True)
    assert np.max(np.abs(back - x)) <= 1e-14 * np.max(np.abs(x)) * np.log2(n)


def test_linearity():
    n = 1024
    a, b = _rand(2, n, 3)
    lhs = oracle.fft((2.5 * a - 1j * b)[None])[0]
    rhs = 2.5 * oracle.fft(a[None])[0] - 1j * oracle.fft(b[None])[0]
    assert np.max(np.abs(lhs - rhs)) < 1e-10


@pytest.mark.parametrize("n", [256, 4096, 16384])
def test_dc_and_alternating_exact(n):
    # all-ones -> N delta[k]; (-1)^n -> N delta[k - N/2]; exact in FP64
    x = np.ones((1, n), complex)
    X = oracle.fft(x)[0]
    expect = np.zeros(n, complex)
    expect[0] = n
    assert np.array_equal(X, expect)
    alt = ((-1.0) ** np.arange(n))[None].astype(complex)
    A = oracle.fft(alt)[0]
    expect = np.zeros(n, complex)
    expect[n // 2] = n
    assert np.array_equal(A, expect)


@pytest.mark.parametrize("n0", [0, 1, 1000, 4095])
def test_impulse_closed_form(n0):
    n = 4096
    x = np.zeros((1, n), complex)
    x[0, n0] = 1.0
    X = oracle.fft(x)[0]
    k = np.arange(n)
    assert np.max(np.abs(X - np.exp(-2j * np.pi * ((n0 * k) % n) / n))) < 1e-13


def test_roots_exact_at_quarter_turns():
    for n in (4, 256, 4096, 16384):
        assert oracle.root(0, n) == complex(1, 0)
        assert oracle.root(n // 4, n) == complex(0, -1)
        assert oracle.root(n // 2, n) == complex(-1, 0)
        assert oracle.root(3 * n // 4, n) == complex(0, 1)
    w = np.array([oracle.root(k, 4096) for k in range(4096)])
    assert np.max(np.abs(np.abs(w) - 1)) <= 2.3e-16
    assert np.max(np.abs(w - np.exp(-2j * np.pi * np.arange(4096) / 4096))) < 1e-15


@pytest.mark.parametrize("n", [1024, 4096])
def test_gauss_sum_lfm_spectrum(n):
    # h[m] = exp(i pi m^2 / N), N even: DFT = sqrt(N) e^{i pi/4} e^{-i pi k^2 / N}
    m = np.arange(n)
    h = np.exp(1j * np.pi * ((m * m) % (2 * n)) / n)
    H = oracle.fft(h[None])[0]
    k = np.arange(n)
    expect = np.sqrt(n) * np.exp(1j * np.pi / 4) * np.exp(-1j * np.pi * ((k * k) % (2 * n)) / n)
    assert np.max(np.abs(H - expect)) < 1e-9


def test_matched_filter_normalised_and_peaks_at_delay():
    n, L = 4096, 1024
    h = scenes.range_replica_padded(n, L)
    H = oracle.matched_filter(h, n)
    assert abs(np.max(np.abs(H)) - 1.0) < 1e-15
    ref = np.conj(np.fft.fft(h))
    ref = ref / np.max(np.abs(ref))
    assert np.max(np.abs(H - ref)) < 1e-12
    for d in (0, 17, 3072):
        x = np.zeros((1, n), complex)
        x[0, d:d + L] = h[:L]
        y = oracle.compress(x, H)[0]
        assert int(np.argmax(np.abs(y))) == d
        # peak = sum|h|^2 / max|DFT h| (matched gain)
        assert abs(np.abs(y[d]) - L / np.max(np.abs(np.fft.fft(h)))) < 1e-9


def test_compress_equals_circular_correlation():
    # y = IDFT(DFT(x) conj(DFT(h))) / c is the circular cross-correlation / c
    n = 64
    rng = np.random.default_rng(5)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    h = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    H = oracle.matched_filter(h, n)
    c = np.max(np.abs(np.fft.fft(h)))
    y = oracle.compress(x[None], H)[0]
    corr = np.array([np.sum(x * np.conj(np.roll(h, d))) for d in range(n)]) / c
    assert np.max(np.abs(y - corr)) < 1e-12


def test_zadoff_chu_overflow_mechanism():
    # Sec. III-B: with |DFT x| = sqrt(N) flat and |H| = 1 the compressed output
    # is sqrt(N) delta; the unscaled inverse peaks at N^1.5 > 65504.
    n = 4096
    m = np.arange(n)
    x = np.exp(-1j * np.pi * ((m * m) % (2 * n)) / n)
    X = oracle.fft(x[None])[0]
    assert np.allclose(np.abs(X), np.sqrt(n), rtol=1e-12)
    H = np.conj(X) / np.sqrt(n)
    y = oracle.compress(x[None], H)[0]
    expect = np.zeros(n, complex)
    expect[0] = np.sqrt(n)
    assert np.max(np.abs(y - expect)) < 1e-10
    unscaled = oracle.fft(np.conj(X * H)[None])[0]
    assert np.max(np.abs(unscaled)) == pytest.approx(n ** 1.5, rel=1e-12)
    assert n ** 1.5 > 65504


def test_transpose_and_sar_chain_composition():
    rng = np.random.default_rng(9)
    npul, nr = 32, 64
    echo = rng.standard_normal((npul, nr)) + 1j * rng.standard_normal((npul, nr))
    Hr = oracle.matched_filter(rng.standard_normal(nr) + 1j * rng.standard_normal(nr), nr)
    Ha = oracle.matched_filter(rng.standard_normal(npul) + 1j * rng.standard_normal(npul), npul)
    img, rct = oracle.sar_image(echo, Hr, Ha, return_rc=True)
    # independent composition with numpy's FFT
    rc = np.fft.ifft(np.fft.fft(echo, axis=1) * Hr[None], axis=1)
    assert np.max(np.abs(rct - rc.T)) < 1e-12
    ref = np.fft.ifft(np.fft.fft(rc.T, axis=1) * Ha[None], axis=1)
    assert img.shape == (nr, npul)
    assert np.max(np.abs(img - ref)) < 1e-12
    phi = rng.uniform(-3, 3, npul)
    img2 = oracle.sar_image(echo, Hr, Ha, phi=phi)
    ref2 = np.fft.ifft(np.fft.fft(rc.T * np.exp(1j * phi)[None], axis=1) * Ha[None], axis=1)
    assert np.max(np.abs(img2 - ref2)) < 1e-12


def test_adjoint_identity():
    # <A x, y> = <x, A^H y>, A^H = same chain with conj(H)
    n = 256
    rng = np.random.default_rng(2)
    H = oracle.matched_filter(rng.standard_normal(n) + 1j * rng.standard_normal(n), n)
    x = _rand(3, n, 4)
    y = _rand(3, n, 5)
    Ax = oracle.compress(x, H)
    AHy = oracle.compress(y, H, conj_filter=True)
    lhs = np.vdot(y, Ax)
    rhs = np.vdot(AHy, x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_entropy_definition_and_gradient():
    rng = np.random.default_rng(8)
    I = rng.standard_normal((4, 8)) + 1j * rng.standard_normal((4, 8))
    I[0, 0] = 0.0  # 0 ln 0 = 0
    E, G = oracle.entropy(I, want_grad=True)
    p = np.abs(I) ** 2 / np.sum(np.abs(I) ** 2)
    nz = p > 0
    assert E == pytest.approx(-np.sum(p[nz] * np.log(p[nz])), rel=1e-14)
    # uniform magnitudes give the maximum ln(count)
    assert oracle.entropy(np.exp(1j * rng.uniform(0, 6, 32))) == pytest.approx(np.log(32), rel=1e-14)
    # real-pair gradient vs central differences on Re and Im parts
    h = 1e-6
    for (i, j) in [(1, 2), (3, 7)]:
        for unit in (1.0, 1j):
            Ip = I.copy(); Ip[i, j] += h * unit
            Im = I.copy(); Im[i, j] -= h * unit
            fd = (oracle.entropy(Ip) - oracle.entropy(Im)) / (2 * h)
            an = G[i, j].real if unit == 1.0 else G[i, j].imag
            assert fd == pytest.approx(an, rel=1e-6, abs=1e-10)


def test_autofocus_gradient_fd_and_invariance():
    rng = np.random.default_rng(6)
    nr, npul = 16, 64
    rc = rng.standard_normal((nr, npul)) + 1j * rng.standard_normal((nr, npul))
    Ha = oracle.matched_filter(scenes.azimuth_replica_centred(npul, 16), npul)
    phi = rng.uniform(-1, 1, npul)
    E, g = oracle.autofocus(rc, Ha, phi)
    # constant-phase invariance: sum_m dE/dphi_m = 0
    assert abs(np.sum(g)) <= 1e-10 * np.sum(np.abs(g))
    h = 1e-4  # central differences: O(h^2) truncation, ~1e-11 roundoff
    for m in (0, 5, 63):
        pp = phi.copy(); pp[m] += h
        pm = phi.copy(); pm[m] -= h
        fd = (oracle.autofocus(rc, Ha, pp)[0] - oracle.autofocus(rc, Ha, pm)[0]) / (2 * h)
        assert fd == pytest.approx(g[m], rel=1e-6, abs=1e-10)


# Adam (Kingma & Ba, 2015, Algorithm 1) for the autofocus phase.  Pins: the
# library routine torch.optim.Adam (FP64 on the CPU) over a sequence of
# gradients, and the closed form under a constant gradient, where the bias
# corrections make both moment estimates exact: every step moves each
# element by lr g / (|g| + eps).

def test_adam_matches_torch_optimizer():
    import torch
    rng = np.random.default_rng(11)
    n, lr, betas, eps = 257, 0.3, (0.9, 0.999), 1e-8
    phi0 = rng.standard_normal(n)
    grads = [rng.standard_normal(n) * s for s in (1.0, 0.1, 3.0, 0.5, 2.0)]
    p = torch.tensor(phi0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=lr, betas=betas, eps=eps)
    phi, m, v = phi0, np.zeros(n), np.zeros(n)
    for k, g in enumerate(grads, start=1):
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        phi, m, v = oracle.adam_step(phi, g, m, v, k, lr, betas[0], betas[1], eps)
        np.testing.assert_allclose(phi, p.detach().numpy(), rtol=1e-13, atol=1e-14)


def test_adam_constant_gradient_closed_form():
    g = np.array([2.0, -0.5, 1e-3, -7.0])
    lr, eps = 0.1, 1e-8
    phi, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for k in range(1, 6):
        phi, m, v = oracle.adam_step(phi, g, m, v, k, lr, eps=eps)
        np.testing.assert_allclose(phi, -k * lr * g / (np.abs(g) + eps), rtol=1e-12)


# ---------------------------------------------------- weighted apertures ----
# Tapers for the weighted matched filters of Sec. VIII (limitations: deeply
# weighted apertures with sidelobes near -40 dB).  Pins: the library routine
# scipy.signal.windows, and closed-form facts of the tapers' transforms.

def _transform_pslr(w, pad=64):
    """Highest sidelobe of |DFT(w)|^2 (zero-padded) outside the first minima."""
    P = np.fft.fftshift(np.abs(np.fft.fft(w, w.size * pad)) ** 2)
    k = int(np.argmax(P))
    lo, hi = k, k
    while lo > 0 and P[lo - 1] < P[lo]:
        lo -= 1
    while hi < P.size - 1 and P[hi + 1] < P[hi]:
        hi += 1
    return 10.0 * np.log10(np.concatenate([P[:lo], P[hi + 1:]]).max() / P[k])


@pytest.mark.parametrize("length", [1, 2, 16, 127, 1024])
def test_tapers_match_scipy(length):
    from scipy.signal import windows as sw
    from oracle import windows as W
    assert np.max(np.abs(W.hamming(length) - sw.hamming(length, sym=True))) <= 1e-14
    for nbar, sll in ((1, 30.0), (4, 30.0), (5, 40.0), (8, 50.0)):
        want = sw.taylor(length, nbar, sll, norm=True, sym=True)
        assert np.max(np.abs(W.taylor(length, nbar, sll) - want)) <= 1e-13, (nbar, sll)


def test_taper_sidelobes_closed_form():
    from oracle import windows as W
    # uniform aperture: -13.26 dB; Hamming 0.54 / 0.46: -42.7 dB
    assert abs(_transform_pslr(np.ones(1024)) + 13.26) <= 0.05
    assert abs(_transform_pslr(W.hamming(1024)) + 42.7) <= 0.1
    # Taylor: the nearest sidelobes at the design level
    for nbar, sll in ((4, 30.0), (5, 40.0), (8, 50.0)):
        assert abs(_transform_pslr(W.taylor(1024, nbar, sll)) + sll) <= 0.4, (nbar, sll)


def test_weighted_point_target_sidelobes_and_broadening():
    # the oracle's range compression of an LFM target (L = 1024, b = 0.8)
    # with a weighted filter: sidelobes at the taper's level (the chirp's
    # spectrum is nearly flat over its band), and the Hamming -3 dB width
    # 1.47 times the uniform one (1.30 / 0.886 bins)
    from oracle import windows as W
    from paper_2605_28451_amd import metrics
    n = 4096
    x = np.zeros((1, n), dtype=np.complex128)
    x[0, :1024] = scenes.lfm_chirp(1024)
    res = {}
    for name, w in (("rect", np.ones(1024)), ("hamming", W.hamming(1024)),
                    ("taylor", W.taylor(1024, 5, 40.0))):
        H = oracle.matched_filter(scenes.weighted_range_replica(n, w), n)
        res[name] = metrics.cut_metrics_1d(oracle.compress(x, H)[0])
    assert abs(res["rect"][0] + 13.26) <= 0.1
    assert abs(res["hamming"][0] + 42.7) <= 0.3
    assert abs(res["taylor"][0] + 40.0) <= 0.7
    assert abs(res["hamming"][2] / res["rect"][2] - 1.47) <= 0.03
    assert res["rect"][2] < res["taylor"][2] < res["hamming"][2]


def test_adaptive_exponent_rule():
    # smallest k in [-15, 14] with sqrt(2) n M 2^-k < 2^15, as k - log2 n
    n = 4096
    at = lambda m: int(oracle.adaptive_exponent(np.array([[m + 0j]]), n)[0]) + 12
    assert at(0.0) == -15                                # an all-zero row: the floor
    edge = 2.0 ** 15 / (np.sqrt(2.0) * n)                # sqrt(2) n M = 2^15 exactly
    assert at(edge * (1 - 1e-12)) == 0 and at(edge) == 1
    assert at(edge * 2 * (1 - 1e-12)) == 1 and at(edge * 2) == 2
    assert at(edge / 8) == -2 and at(edge / 8 * (1 - 1e-12)) == -3
    assert at(1.0) == -2                                 # sqrt(2) 4096 = 2^12.5: 2^14.5 < 2^15
    assert at(64.0) == 4                                 # 2^18.5: 2^14.5 < 2^15 <= 2^15.5
    assert at(1e-30) == -15
    assert at(1e30) == 14                                # capped
    # the component maximum, not the modulus, and per row
    z = np.array([[3.0 + 4.0j, -5.0 + 0j], [0.0 + 0.0j, 0.0 + 0.0j]])
    e = oracle.adaptive_exponent(z, n)
    assert e[1] == -15 - 12 and e[0] == oracle.adaptive_exponent(np.array([[5.0 + 0j]]), n)[0]
    # bound and minimality on random rows
    rng = np.random.default_rng(9)
    rows = (rng.standard_normal((50, n)) + 1j * rng.standard_normal((50, n))) * 10.0 ** rng.uniform(-6, 2, (50, 1))
    for row, ex in zip(rows, oracle.adaptive_exponent(rows, n)):
        k = ex + 12
        b = np.sqrt(2.0) * n * max(np.abs(row.real).max(), np.abs(row.imag).max())
        assert -15 <= k <= 14 and b * 2.0 ** -k < 2.0 ** 15
        assert k == -15 or b * 2.0 ** -(k - 1) >= 2.0 ** 15


# ------------------------------------------ range cell migration (RCMC) ----

def test_rcmc_shift_is_band_limited_interpolation():
    n = 256
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    one = np.ones(n, dtype=np.complex128)
    # integer shifts: a circular roll toward smaller index
    y = oracle.rcmc_compress(x, one, [3.0, -7.0, 0.0])
    for r, s in enumerate((3, -7, 0)):
        assert np.max(np.abs(y[r] - np.roll(x[r], -s))) <= 1e-12
    # a fractional shift of a complex exponential below Nyquist is exact
    k0, s = 37, 2.375
    e = np.exp(2j * np.pi * k0 * np.arange(n) / n)
    y = oracle.rcmc_compress(e[None], one, [s])[0]
    assert np.max(np.abs(y - np.exp(2j * np.pi * k0 * (np.arange(n) + s) / n))) <= 1e-12
    k1 = n - 21   # a negative frequency takes the signed bin
    e = np.exp(2j * np.pi * k1 * np.arange(n) / n)
    y = oracle.rcmc_compress(e[None], one, [s])[0]
    assert np.max(np.abs(y - np.exp(2j * np.pi * (k1 - n) * (np.arange(n) + s) / n))) <= 1e-12


def test_rcmc_focuses_migrating_targets():
    # hyperbolic migration of 6.4 range bins at the aperture edge: with the
    # correction every target focuses to the unweighted point-target figures
    # (PSLR -13.26 dB, IRW 0.886 / 0.8 = 1.107 samples); without it the
    # azimuth response smears to more than twice its width
    from paper_2605_28451_amd import metrics
    sc = scenes.migration_scene()
    n = 4096
    Hr = oracle.matched_filter(sc.range_replica, n)
    Ha = oracle.matched_filter(sc.azimuth_replica, n)
    img = oracle.rda_rcmc_image(sc.echo, Hr, Ha, sc.rcmc_shift)
    raw = oracle.rda_rcmc_image(sc.echo, Hr, Ha, np.zeros(n))
    for (r0, a0) in sc.targets[::4]:
        m = metrics.point_target(img, r0, a0)
        assert m["peak_rc"] == (r0, a0)
        for k in ("pslr_range", "pslr_azimuth"):
            assert abs(m[k] + 13.26) <= 0.3, (r0, a0, k, m[k])
        for k in ("irw_range", "irw_azimuth"):
            assert abs(m[k] - 1.107) <= 0.03, (r0, a0, k, m[k])
        u = metrics.point_target(raw, r0, a0)
        assert u["irw_azimuth"] > 2.0 * m["irw_azimuth"] and u["pslr_range"] > m["pslr_range"] + 3.0


def test_magnitude_budget_closed_forms():
    # The cascade of Sec. IV-B: each stage's output magnitude bounds the next
    # stage's input, and with |H| <= 1 every intermediate of the chains stays
    # far below the FP16 limit 65504.  Closed forms: a unit target's
    # range-compressed peak is sum|h|^2 / max|DFT h| = L / max|DFT h|
    # (Parseval), the focused image peak the product of that with
    # A / max|DFT g| for the azimuth replica; the forward spectrum obeys
    # |X| <= N max|x|.
    n, L, A = 4096, 1024, 512
    rs = scenes.range_scene(seed=2, n_pulses=64)
    Mr = np.abs(oracle.fft(rs.replica[None])[0]).max()
    X = oracle.fft(rs.echo)
    assert np.abs(X).max() <= n * np.abs(rs.echo).max()
    Hr = oracle.matched_filter(rs.replica, n)
    rc = oracle.compress(rs.echo, Hr)
    # each of the 5 targets peaks at its delay at L / max|DFT h| (about 24)
    for d in rs.delays:
        assert abs(np.abs(rc[:, d]).mean() - L / Mr) <= 0.02 * L / Mr
    assert np.abs(X * Hr[None]).max() / n < 1.0 and np.abs(rc).max() < 64.0
    sc = scenes.sar_scene(seed=3)
    Ma = np.abs(oracle.fft(sc.azimuth_replica[None])[0]).max()
    Ha = oracle.matched_filter(sc.azimuth_replica, n)
    img, rct = oracle.sar_image(sc.echo, Hr, Ha, return_rc=True)
    peak = (L / Mr) * (A / Ma)
    for (r0, a0) in sc.targets:
        assert abs(np.abs(img[r0, a0]) - peak) <= 0.02 * peak
    # the largest input of the azimuth stage (three targets share a range
    # bin) and every output stay below 4096, far inside FP16
    assert np.abs(oracle.fft(rct)).max() < 4096.0 and np.abs(img).max() < 4096.0
