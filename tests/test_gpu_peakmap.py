"""GPU peakmap construction against the oracle: bit-exact CSR."""
import numpy as np
import pytest

from oracle import peakmap
from paper_1407_8333_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_fft,n_bins,with_ar", [(1, 3, False), (7, 257, True), (300, 8500, True),
                                                   (3140, 1000, False)])
def test_peakmap_from_spectra_matches_oracle(n_fft, n_bins, with_ar):
    import torch
    from paper_1407_8333_amd import api
    rng = synth.rng_for(n_fft + n_bins)
    ar = rng.uniform(0.5, 2.0, (n_fft, n_bins)).astype(np.float32)
    sp = (rng.standard_exponential((n_fft, n_bins)).astype(np.float32) * ar).astype(np.float32)
    if not with_ar:
        sp = rng.standard_exponential((n_fft, n_bins)).astype(np.float32)
    t = synth.fft_times(n_fft, 1024.0)
    v = synth.detector_velocity(t, rng)
    with api.Context(0) as ctx:
        dsp = torch.as_tensor(sp, device="cuda")
        dar = torch.as_tensor(ar, device="cuda") if with_ar else None
        dpm = api.DevicePeakmap.from_spectra(ctx, dsp, 12345, 2.5, t, v, 1024.0, sar=dar)
        off, bins = dpm.download()
        ref_off, ref_bins = peakmap.peakmap_from_spectra(sp, ar if with_ar else None, 12345, 2.5)
        np.testing.assert_array_equal(off, ref_off)
        np.testing.assert_array_equal(bins, ref_bins)
        dpm.release()


def test_built_peakmap_feeds_the_hough_map():
    """The GPU-built peakmap gives the same Hough map as the uploaded one."""
    import torch
    from paper_1407_8333_amd import api
    rng = synth.rng_for(8)
    n_fft, t_fft = 400, 4096.0
    k_lo, n_bins = 300 * 4096 - 200, 1400
    sp = rng.standard_exponential((n_fft, n_bins)).astype(np.float32)
    t = synth.fft_times(n_fft, t_fft)
    v = synth.detector_velocity(t, rng)
    off, bins = peakmap.peakmap_from_spectra(sp, None, k_lo, 2.5)
    pm = synth.Peakmap(t_fft, t, v, off, bins)
    grid = synth.make_grid(pm, 300.0, 300.2, -1e-8, 1e-9)
    with api.Context(0) as ctx:
        built = api.DevicePeakmap.from_spectra(ctx, torch.as_tensor(sp, device="cuda"), k_lo, 2.5, t, v, t_fft)
        up = ctx.upload(pm)
        n = synth.sky_uniform(1, rng)[0]
        a = api.fh_hough_map_i32(ctx, built, n, grid)
        b = api.fh_hough_map_i32(ctx, up, n, grid)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        built.release()
        up.release()
