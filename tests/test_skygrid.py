"""Sky grids (Sec. "Grid in the sky", Eqs. gammalong, gammalat, ND, Nsky;
appendix on the construction of the coarse grid; Sec. "Refined grid in the
sky")."""
import math

import numpy as np
import pytest

from paper_1407_8333_amd import skygrid


def test_doppler_bins_matches_the_orbital_doppler_band():
    # N_D = B_D / delta f with B_D = f0 v_orb / c, |v_orb| / c ~ 1e-4
    nd = skygrid.doppler_bins(200.0, 1024.0)
    assert nd == pytest.approx(200.0 * 1e-4 * 1024.0, rel=0.01)


@pytest.mark.parametrize("n_d", [3.3, 20.35, 81.4, 407.0])
def test_latitudes_follow_the_recurrence_and_land_on_the_equator(n_d):
    beta, k = skygrid.latitudes(n_d)
    n = len(beta)
    assert n % 2 == 1
    assert beta[0] == 0.5 * math.pi and beta[-1] == -0.5 * math.pi and beta[n // 2] == 0.0
    np.testing.assert_allclose(beta, -beta[::-1], atol=0)
    assert np.all(np.diff(beta) < 0)
    north = beta[: n // 2 + 1]
    # every step beta_{i-1} - beta_i = K / (N_D sin beta_{i-1}) with one K <= 1
    ks = (north[:-1] - north[1:]) * n_d * np.sin(north[:-1])
    assert 0 < k <= 1
    np.testing.assert_allclose(ks, k, rtol=1e-9)
    # K is the largest that lands on the equator: at K = 1 the same number of
    # steps reaches or passes it, and a slightly larger K overshoots
    m = len(north) - 1
    b = 0.5 * math.pi
    for _ in range(m):
        b -= 1.0 / (n_d * math.sin(b))
        if b <= 0:
            break
    assert b <= 0
    if k < 1:
        b = 0.5 * math.pi
        for _ in range(m):
            b -= (k * (1 + 1e-9)) / (n_d * math.sin(b))
            if b <= 0:
                break
        assert b < 0


@pytest.mark.parametrize("n_d", [20.35, 81.4])
def test_longitude_spacing_is_the_largest_submultiple_of_2pi_within_resolution(n_d):
    beta, _ = skygrid.latitudes(n_d)
    n = skygrid.ring_sizes(beta, n_d)
    for b, m in zip(beta, n):
        if abs(b) == 0.5 * math.pi:
            assert m == 1
            continue
        res = 1.0 / (n_d * math.cos(b))  # Eq. gammalong
        assert 2 * math.pi / m <= res * (1 + 1e-12)
        assert m == 1 or 2 * math.pi / (m - 1) > res


def test_adjacent_grid_points_differ_by_at_most_one_frequency_bin():
    # the defining criterion: the maximum Doppler difference between
    # neighbouring directions is delta f = 1 / T_FFT
    f0, t_fft = 200.0, 1024.0
    g = skygrid.coarse_grid(f0, t_fft)
    v = skygrid.V_ORB_OVER_C
    df_lon = f0 * v * g.dlam * np.cos(g.beta) * t_fft
    assert df_lon.max() <= 1.0 + 1e-9
    inner = np.abs(g.beta) > 1e-9
    df_lat = f0 * v * g.dbeta[inner] * np.abs(np.sin(g.beta[inner])) * t_fft
    # the ring spacing uses sin at the ring nearer the pole: the step is
    # K / (N_D sin beta) at the poleward ring, so at most one bin there
    assert df_lat.max() <= 1.0 / np.sin(np.abs(g.beta[inner])).min() + 1e-9


def test_point_count_tends_to_the_continuum_count_of_the_construction():
    """Cells of 1/(N_D cos b) x 1/(N_D sin b) tile the sphere with
    2 pi N_D^2 points in the high-frequency limit (the rounding up of ring
    sizes adds about N_D); Eq. Nsky quotes 4 pi K_sky N_D^2 from a
    simulation, a factor 2 the construction does not reproduce (recorded as
    a reading)."""
    ratios = []
    for f0, t_fft in [(200.0, 1024.0), (500.0, 4096.0), (1000.0, 8192.0)]:
        g = skygrid.coarse_grid(f0, t_fft)
        nd = g.n_d
        ratios.append(len(g) / (2 * math.pi * nd * nd))
        assert 1.0 <= ratios[-1] < 1.15
    assert ratios[0] > ratios[1] > ratios[2]
    assert ratios[2] == pytest.approx(1.0, abs=0.01)
    # K_sky scales the count
    g1 = skygrid.coarse_grid(500.0, 4096.0)
    g2 = skygrid.coarse_grid(500.0, 4096.0, k_sky=2.0)
    assert len(g2) / len(g1) == pytest.approx(2.0, rel=0.02)


def test_ecliptic_to_equatorial_axes():
    eps = skygrid.OBLIQUITY
    n = skygrid.ecliptic_to_equatorial([0.0, 0.0, 0.5 * math.pi], [0.0, 0.5 * math.pi, 0.0])
    np.testing.assert_allclose(n[0], [1, 0, 0], atol=1e-15)
    np.testing.assert_allclose(n[1], [0, -math.sin(eps), math.cos(eps)], atol=1e-15)
    np.testing.assert_allclose(n[2], [0, math.cos(eps), math.sin(eps)], atol=1e-15)
    g = skygrid.coarse_grid(100.0, 1024.0)
    np.testing.assert_allclose(np.linalg.norm(g.nhat(), axis=1), 1.0, atol=1e-15)


def test_refined_points_form_k_hat_squared_layers():
    lam, beta = skygrid.refined_points(1.0, 0.3, 0.05, 0.04, 5)
    assert len(lam) == 25  # K_hat = 5, two layers (the paper's example)
    assert (lam[12], beta[12]) == (1.0, 0.3)  # the centre
    np.testing.assert_allclose(np.unique(np.round(lam, 12)), 1.0 + np.arange(-2, 3) * 0.01)
    np.testing.assert_allclose(np.unique(np.round(beta, 12)), 0.3 + np.arange(-2, 3) * 0.008)
    with pytest.raises(ValueError):
        skygrid.refined_points(1.0, 0.3, 0.05, 0.04, 4)
