"""Refined grid around coarse candidates (Sec. "Refined Grid in the parameter
space") and peakmap slicing, against the oracle run on the full peakmap."""
import math

import numpy as np
import pytest

import oracle
from paper_1407_8333_amd import skygrid, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1407_8333_amd import api
    c = api.Context(0)
    yield c
    c.close()


def _signal_band():
    """400 FFTs of 8192 s at 100-100.2 Hz with Doppler and one signal of
    known direction, frequency and spin-down."""
    rng = synth.rng_for(4242)
    t_fft, n = 8192.0, 400
    nhat = synth.sky_uniform(1, rng)[0]
    t = synth.fft_times(n, t_fft)
    t0 = 0.5 * (t[0] + t[-1])
    inj = synth.Injection(100.0913, -3.3e-10, nhat, lam=2.5)
    pm = synth.make_noise_peakmap(n, t_fft, int(100.0 * t_fft) - 120, int(100.2 * t_fft) + 120, seed=11,
                                  injections=[inj], t0=t0)
    grid = synth.make_grid(pm, 100.0, 100.2, -1e-9, 1e-10, t0=t0)
    return pm, grid, inj


def _reference_directions(lam_c, beta_c, dlam, dbeta, k_sky):
    """The refined directions written out with the scalar functions the
    library uses, in the same order (so both sides get identical vectors)."""
    L = (k_sky - 1) // 2
    eps = math.radians(23.44)
    ce, se = math.cos(eps), math.sin(eps)
    out = []
    for j in range(-L, L + 1):
        for i in range(-L, L + 1):
            lam = lam_c + i * (dlam / k_sky)
            bet = beta_c + j * (dbeta / k_sky)
            if abs(bet) > 0.5 * math.pi:
                lam += math.pi
                bet = (math.pi if bet > 0 else -math.pi) - bet
            lam = math.fmod(lam, 2.0 * math.pi)
            if lam < 0:
                lam += 2.0 * math.pi
            x, ye, ze = math.cos(bet) * math.cos(lam), math.cos(bet) * math.sin(lam), math.sin(bet)
            n = [x, ye * ce - ze * se, ye * se + ze * ce]
            r = math.sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2])
            out.append((lam, bet, [n[0] / r, n[1] / r, n[2] / r]))
    return out


def _oracle_refined(pm, cand, kf, k_fdot, k_sky, dfdot, t0, w=None):
    """Best cell of the refined volume by the oracle on the full peakmap:
    larger value, then smaller direction index, smaller bin, smaller row."""
    f0c, fdc = cand[0], cand[1]
    rgrid = synth.Grid(kf=kf, b0=int(round(f0c * kf * pm.t_fft)) - kf, nf=2 * kf + 1, ns=4 * k_fdot,
                       fdot0=fdc - 2 * dfdot, dfdot=dfdot / k_fdot, t0=t0)
    dirs = _reference_directions(*cand[2:], k_sky)
    best = None
    for d, (lam, bet, n) in enumerate(dirs):
        m = oracle.hough_map(pm, rgrid, np.array(n), weights=None if w is None else w.astype(np.float64))
        vmax = m.max()
        rows, bins = np.nonzero(m == vmax)
        k = np.lexsort((rows, bins))[0]
        if best is None or vmax > best[0]:
            best = (vmax, d, int(bins[k]), int(rows[k]))
    return best, rgrid, dirs


def test_peakmap_slice_matches_a_host_selection(ctx):
    import torch
    from paper_1407_8333_amd import api
    pm, _, _ = _signal_band()
    dpm = ctx.upload(pm)
    k_lo, k_hi = int(100.05 * pm.t_fft), int(100.12 * pm.t_fft)
    sub = dpm.slice(k_lo, k_hi)
    torch.cuda.synchronize()
    off, bins = sub.download()
    want_off = [0]
    want = []
    for i in range(pm.n_fft):
        b = pm.bins[pm.offsets[i]:pm.offsets[i + 1]]
        sel = b[(b >= k_lo) & (b < k_hi)]
        want.extend(sel.tolist())
        want_off.append(len(want))
    np.testing.assert_array_equal(off, np.array(want_off))
    np.testing.assert_array_equal(bins, np.array(want, dtype=np.int32))
    sub.release()
    dpm.release()


@pytest.mark.parametrize("weighted", [False, True])
def test_refined_candidate_is_the_best_cell_of_the_refined_volume(ctx, weighted):
    import torch
    from paper_1407_8333_amd import api
    pm, grid, inj = _signal_band()
    dpm = ctx.upload(pm)
    w = synth.fft_weights(pm.n_fft, synth.rng_for(5)) if weighted else None
    wt = None if w is None else torch.as_tensor(w, device="cuda")
    # coarse candidate: the coarse sky point nearest the signal, its best cell
    # in the sub-band of the signal
    g = skygrid.coarse_grid(100.2, pm.t_fft)
    nh = g.nhat()
    c = int(np.argmax(nh @ inj.nhat))
    sel = synth.Selection(width=int(round(0.01 * grid.kf * pm.t_fft)))
    raw = api.fh_hough_candidates(ctx, dpm, nh[c:c + 1], grid, sel, weights=wt)
    dec = api.decode_candidates(raw)
    sb = int(inj.f0 * grid.kf * pm.t_fft - grid.b0) // sel.width
    b, s = int(dec["bin"][0, sb, 0]), int(dec["row"][0, sb, 0])
    f0c = (grid.b0 + b) / (grid.kf * pm.t_fft)
    fdc = grid.fdot0 + s * grid.dfdot
    kf, k_fdot, k_sky = grid.kf, 3, 5
    cand = [f0c, fdc, g.lam[c], g.beta[c], g.dlam[c], g.dbeta[c]]
    out = api.decode_refined(api.refine(ctx, dpm, [cand], kf, k_fdot, k_sky, grid.dfdot, grid.t0,
                                        weights=wt))[0]
    torch.cuda.synchronize()
    best, rgrid, dirs = _oracle_refined(pm, cand, kf, k_fdot, k_sky, grid.dfdot, grid.t0, w)
    assert out["valid"] == 1
    if w is None:
        assert (float(out["value"]), int(out["sky"]), int(out["bin"]), int(out["row"])) == \
            (float(best[0]), best[1], best[2], best[3])
    else:
        tol = 1e-5 * max(best[0], float(np.mean(w)))
        assert float(out["value"]) == pytest.approx(best[0], abs=2 * tol)
    lam, bet, _ = dirs[int(out["sky"])]
    assert (out["lambda"], out["beta"]) == (lam, bet)
    assert out["f0"] == pytest.approx((rgrid.b0 + int(out["bin"])) / (kf * pm.t_fft), rel=0, abs=1e-12)
    assert out["fdot"] == pytest.approx(rgrid.fdot0 + int(out["row"]) * rgrid.dfdot, rel=1e-12)
    # the refined cell lies on the signal: within one natural bin in frequency
    # and one and a half coarse spin-down steps
    assert abs(out["f0"] - inj.f0) <= 1.0 / pm.t_fft
    assert abs(out["fdot"] - inj.fdot) <= 1.5 * grid.dfdot
    dpm.release()


def test_several_candidates_in_one_call(ctx):
    """Candidates in different sub-bands and one whose refined sky crosses
    the north pole; each result is the oracle's best cell of its own volume."""
    from paper_1407_8333_amd import api
    pm, grid, inj = _signal_band()
    dpm = ctx.upload(pm)
    g = skygrid.coarse_grid(100.2, pm.t_fft)
    rng = synth.rng_for(77)
    c_sig = int(np.argmax(g.nhat() @ inj.nhat))
    c_rand = int(rng.integers(len(g)))
    c_pole = 1  # first ring below the pole
    cands = [
        [inj.f0, inj.fdot + 0.4 * grid.dfdot, g.lam[c_sig], g.beta[c_sig], g.dlam[c_sig], g.dbeta[c_sig]],
        [100.031, -5.0e-10, g.lam[c_rand], g.beta[c_rand], g.dlam[c_rand], g.dbeta[c_rand]],
        [100.17, 0.0, g.lam[c_pole], g.beta[c_pole], g.dlam[c_pole], 3.0 * g.dbeta[c_pole]],
    ]
    kf, k_fdot, k_sky = grid.kf, 2, 7
    out = api.decode_refined(api.refine(ctx, dpm, cands, kf, k_fdot, k_sky, grid.dfdot, grid.t0))
    assert [int(x) for x in out["cand"]] == [0, 1, 2]
    for c, cand in enumerate(cands):
        best, rgrid, dirs = _oracle_refined(pm, cand, kf, k_fdot, k_sky, grid.dfdot, grid.t0)
        o = out[c]
        assert o["valid"] == 1
        assert (float(o["value"]), int(o["sky"]), int(o["bin"]), int(o["row"])) == \
            (float(best[0]), best[1], best[2], best[3])
        assert (o["lambda"], o["beta"]) == dirs[int(o["sky"])][:2]
    # the third volume reaches past the pole (its latitudes fold back)
    assert cands[2][3] + (k_sky - 1) // 2 * cands[2][5] / k_sky > 0.5 * math.pi
    dpm.release()


def test_refine_edge_cases(ctx):
    """No candidates is a no-op; an even k_sky, a zero spin-down step and a
    candidate below bin 0 are rejected before any launch."""
    from paper_1407_8333_amd import api
    from paper_1407_8333_amd._lib import FHError
    pm, grid, _ = _signal_band()
    dpm = ctx.upload(pm)
    assert api.refine(ctx, dpm, np.zeros((0, 6)), grid.kf, 2, 5, grid.dfdot, grid.t0).numel() == 0
    good = [100.1, 0.0, 1.0, 0.2, 0.05, 0.05]
    for kw, cand in [(dict(k_sky=4), good), (dict(dfdot=0.0), good),
                     (dict(), [1e-9, 0.0, 1.0, 0.2, 0.05, 0.05])]:
        args = dict(kf=grid.kf, k_fdot=2, k_sky=5, dfdot=grid.dfdot, t0=grid.t0)
        args.update(kw)
        with pytest.raises(FHError):
            api.refine(ctx, dpm, [cand], **args)
    dpm.release()
