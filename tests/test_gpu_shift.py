"""Per-FFT shift variant of the Doppler correction (fh_ctx_set_doppler mode
1) against the oracle's shift mode: unweighted maps and candidates
bit-exact, weighted maps within 1e-5 relative."""
import numpy as np
import pytest

import oracle
from paper_1407_8333_amd import synth
from test_gpu_parity import _assert_weighted_close, _check_candidates, _gpu_map

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1407_8333_amd import api
    c = api.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("seed", range(4))
def test_shift_maps_match_the_oracle(ctx, seed):
    rng = synth.rng_for(900 + seed)
    kf = [1, 10, 10, 37][seed]
    t_fft = [1024.0, 4096.0, 8192.0, 2048.0][seed]
    n_fft = int(rng.integers(5, 60))
    k_lo = int(rng.integers(20_000, 400_000))
    pm = synth.random_peakmap(n_fft, t_fft, k_lo, k_lo + 600, 0.08, rng)
    f_lo = (k_lo + 60) / t_fft
    f_hi = (k_lo + 60 + int(rng.integers(50, 480))) / t_fft
    grid = synth.make_grid(pm, f_lo, f_hi, -3e-8, 2e-9, kf=kf)
    nhat = synth.sky_uniform(1, rng)[0]
    f_ref = 0.0 if seed % 2 else (k_lo + 100.25) / t_fft
    ctx.set_doppler("shift", f_ref)
    try:
        got = _gpu_map(ctx, pm, grid, nhat)
        ref = oracle.hough_map(pm, grid, nhat, doppler="shift", f_ref=f_ref or None)
        np.testing.assert_array_equal(got, ref.astype(np.int32))
        wts = rng.uniform(0.5, 1.5, pm.n_fft).astype(np.float32)
        gotw = _gpu_map(ctx, pm, grid, nhat, weights=wts)
        refw = oracle.hough_map(pm, grid, nhat, weights=wts.astype(np.float64), doppler="shift",
                                f_ref=f_ref or None)
        _assert_weighted_close(gotw, refw, wts)
        # the unfused window methods read the same edges
        for m in (0, 1):
            ctx.set_option("window_method", m)
            np.testing.assert_array_equal(_gpu_map(ctx, pm, grid, nhat), ref.astype(np.int32))
        ctx.set_option("window_method", 2)
    finally:
        ctx.set_doppler("exact")
    # back to the exact correction
    np.testing.assert_array_equal(_gpu_map(ctx, pm, grid, nhat), oracle.hough_map(pm, grid, nhat).astype(np.int32))


def test_shift_candidates_100hz_full_size(ctx):
    """The 1 Hz band at 100 Hz (3140 FFTs, 118 rows) for one direction:
    candidates of the shift variant equal the oracle's."""
    from paper_1407_8333_amd import api
    w = synth.workload("sky-100hz")
    dpm = ctx.upload(w.pm)
    sel = synth.Selection(width=int(round(0.1 * w.grid.kf * w.pm.t_fft)))
    ctx.set_doppler("shift")
    try:
        dec = api.decode_candidates(api.fh_hough_candidates(ctx, dpm, w.sky, w.grid, sel))
    finally:
        ctx.set_doppler("exact")
    ref_map = oracle.hough_map(w.pm, w.grid, w.sky[0], doppler="shift")
    idx, val = oracle.candidates(ref_map, sel.width, sel.excl, sel.sep)
    _check_candidates(dec, 0, idx, val, w.pm.n_fft, sel.theta)
    dpm.release()


def test_set_doppler_rejects_bad_arguments(ctx):
    from paper_1407_8333_amd import _lib
    from paper_1407_8333_amd._lib import FHError, check
    with pytest.raises(FHError):
        check(_lib.fh_ctx_set_doppler(ctx.handle, 2, 0.0))
    with pytest.raises(FHError):
        check(_lib.fh_ctx_set_doppler(ctx.handle, 1, float("nan")))
