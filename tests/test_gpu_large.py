"""Large-band configuration at full size (1024-1034 Hz, T_FFT 1024 s, 25 000
FFTs, ~20 M peaks per direction, 147 spin-down rows, 102 400 fine bins,
weighted, 100 injected signals): the persistent batched search against the
oracle on sampled directions, and recovery of injected signals at their own
sky directions."""
import numpy as np
import pytest

import oracle
from paper_1407_8333_amd import synth

from test_gpu_parity import _candidates_ref, _check_candidates

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def large():
    import torch
    from paper_1407_8333_amd import api
    w = synth.workload("large-1024hz", n_sky=4)
    # four grid directions, then the directions of two injected signals
    sky = np.concatenate([w.sky[:4], np.stack([w.injections[0].nhat, w.injections[1].nhat])])
    ctx = api.Context(0)
    dpm = ctx.upload(w.pm)
    wt = torch.as_tensor(w.weights, device="cuda")
    raw_u = api.fh_hough_candidates(ctx, dpm, sky, w.grid, w.sel, schedule=1)
    raw_w = api.fh_hough_candidates(ctx, dpm, sky, w.grid, w.sel, weights=wt, schedule=1)
    torch.cuda.synchronize()
    ctx.check()
    out = (w, sky, api.decode_candidates(raw_u), api.decode_candidates(raw_w))
    dpm.release()
    ctx.close()
    return out


def test_large_band_unweighted_candidates_bit_exact(large):
    w, sky, dec_u, _ = large
    _, idx, val = _candidates_ref(w.pm, w.grid, sky[1], w.sel)
    _check_candidates(dec_u, 1, idx, val, w.pm.n_fft, w.sel.theta)


def test_large_band_weighted_candidates(large):
    w, sky, _, dec_w = large
    m, idx, val = _candidates_ref(w.pm, w.grid, sky[4], w.sel, weights=w.weights)
    _check_candidates(dec_w, 4, idx, val, w.pm.n_fft, w.sel.theta, weighted_map=m, weights=w.weights)


@pytest.mark.parametrize("k", [0, 1])
def test_large_band_injection_recovered(large, k):
    """At the injected direction, the first candidate of the sub-band holding
    the signal lies within one stripe width and two spin-down rows of the
    injected (f0, fdot), with a critical ratio far above noise."""
    w, sky, dec_u, _ = large
    g, inj = w.grid, w.injections[k]
    b_true = inj.f0 * g.kf * w.pm.t_fft - g.b0
    s_true = (inj.fdot - g.fdot0) / g.dfdot
    sb = int(b_true) // w.sel.width
    s = 4 + k
    assert dec_u["valid"][s, sb, 0] == 1
    assert abs(int(dec_u["bin"][s, sb, 0]) - b_true) <= g.kf
    assert abs(int(dec_u["row"][s, sb, 0]) - s_true) <= 2
    assert dec_u["cr"][s, sb, 0] > 10.0
