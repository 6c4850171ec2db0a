"""Seeded input generators and storage encoders (host only)."""
import numpy as np
import pytest
import torch

from oracle import emulator
from paper_2605_28451_amd import scenes


def _probe_values():
    rng = np.random.default_rng(1)
    v = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.uniform(-6, 5, 20000),
        [0.0, -0.0, 448.0, 449.0, 464.0, 480.0, 1e6, -1e6, 57344.0, 6e4, 2.0 ** -9, 2.0 ** -10,
         3 * 2.0 ** -11, 2.0 ** -16, 2.0 ** -17, 3 * 2.0 ** -18, 0.0625 * 1.0625],
    ])
    return v


@pytest.mark.parametrize("fmt,tdtype", [("e4m3", torch.float8_e4m3fn), ("e5m2", torch.float8_e5m2)])
def test_fp8_encoder_matches_torch_and_emulator(fmt, tdtype):
    v = _probe_values()
    vmax = 448.0 if fmt == "e4m3" else 57344.0
    enc = scenes.encode(v.astype(np.complex128), fmt)[..., 0]
    # torch's cast is RNE without saturation: clamp first (library routine)
    t = torch.from_numpy(np.clip(v, -vmax, vmax)).to(tdtype)
    assert np.array_equal(enc, t.view(torch.uint8).numpy())
    dec = scenes.decode(np.stack([enc, enc], -1), fmt).real
    assert np.array_equal(dec, emulator.round_to_format(v, fmt))
    assert np.array_equal(dec, t.to(torch.float64).numpy())
    # NaN encodings decode to NaN, and NaN encodes to NaN
    nan_code = scenes.encode(np.array([complex(np.nan, 1.0)]), fmt)
    assert np.isnan(scenes.decode(nan_code, fmt).real[0])
    assert np.isnan(torch.from_numpy(nan_code[..., 0].copy()).view(tdtype).to(torch.float32).numpy()[0])


def test_fp16_fp32_encoders_round_nearest_even():
    v = _probe_values()
    with np.errstate(over="ignore"):
        assert np.array_equal(scenes.encode(v.astype(complex), "fp16")[..., 0], v.astype(np.float16))
    assert np.array_equal(scenes.encode(v.astype(complex), "fp32")[..., 0], v.astype(np.float32))
    x = v[:100] + 1j * v[100:200]
    for fmt in ("fp16", "fp32", "e4m3", "e5m2"):
        with np.errstate(over="ignore"):
            e = scenes.encode(x, fmt)
        assert e.shape == x.shape + (2,)
        with np.errstate(over="ignore"):
            q = scenes.quantize(x, fmt)
        assert np.array_equal(q.real, scenes.decode(e, fmt).real)


def test_chirp_exact_phase_reduction():
    L = 1024
    h = scenes.lfm_chirp(L)
    n = np.arange(L) - L // 2
    direct = np.exp(1j * np.pi * 0.8 * n.astype(float) ** 2 / L)
    assert np.max(np.abs(h - direct)) < 1e-11
    assert np.allclose(np.abs(h), 1.0, atol=1e-15)
    g = scenes.azimuth_replica_centred(4096, 512)
    assert np.count_nonzero(g) == 512 and g[0] == 1.0
    assert np.allclose(g[1], np.exp(-1j * np.pi * 0.8 / 512))


def test_scenes_are_seeded_and_shaped():
    a = scenes.range_scene(seed=2, n_pulses=8)
    b = scenes.range_scene(seed=2, n_pulses=8)
    assert np.array_equal(a.echo, b.echo) and a.echo.shape == (8, 4096)
    assert len(a.delays) == 5 and np.all(a.delays <= 4096 - 1024)
    ub = scenes.uneven_batch(seed=4, count=100)
    assert ub.x.size == int(np.sum(1 << ub.log2n.astype(np.int64)))
    assert set(np.unique(ub.log2n)) <= set(range(8, 15)) and set(np.unique(ub.inverse)) <= {0, 1}
    phi = scenes.autofocus_phase_error(n_pulse=4096)
    # quadratic of 4 pi at +/-256 pulses around the centre (plus N(0, 0.3) jitter)
    assert abs(phi[2048 + 256] - phi[2048] - 4 * np.pi) < 3.0
    sc = scenes.sar_scene(seed=3, n=512, ranges=(100,), azimuths=(256,), length=64, aperture=32)
    assert sc.echo.shape == (512, 512) and sc.targets == [(100, 256)]


def test_weighted_replicas_taper_the_support_only():
    n = 4096
    w = np.linspace(0.5, 1.0, 1024)
    h = scenes.weighted_range_replica(n, w)
    h0 = scenes.range_replica_padded(n)
    assert np.array_equal(h[:1024], h0[:1024] * w) and not np.any(h[1024:])
    wa = np.linspace(0.25, 1.0, 512)
    g = scenes.weighted_azimuth_replica(n, wa)
    g0 = scenes.azimuth_replica_centred(n)
    m = np.arange(-256, 256)
    assert np.array_equal(g[m % n], g0[m % n] * wa)
    assert np.count_nonzero(g) == 512


def test_migration_scene_geometry():
    sc = scenes.migration_scene(ranges=(2048,), azimuths=(2048,))
    assert abs(sc.migration_edge_bins - 6.4) < 1e-12
    f = np.fft.fftfreq(4096)
    # the migration curve is even in Doppler, zero at f = 0 and about
    # A b_a / (8 mu) = 6.4 bins at the band edge f = 0.4
    assert sc.rcmc_shift[0] == 0.0
    assert np.allclose(sc.rcmc_shift[1:2048], sc.rcmc_shift[:2048:-1][:2047])
    k = int(np.argmin(np.abs(f - 0.4)))
    assert abs(sc.rcmc_shift[k] - 6.4) < 0.01
    # the echo holds the delayed chirp: at closest approach it starts at the
    # target's range start, at the aperture edge 6.4 bins later
    p0 = sc.echo[2048] - 0  # closest approach
    assert np.abs(p0[2048]) > 0.5 and np.abs(p0[2040]) < 0.5
