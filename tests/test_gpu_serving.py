"""Continuous-batching server: each request's candidates are identical alone
and in the mix and match the oracle on sampled directions; admission respects
the HBM budget (the arena holds the workspaces of the running requests);
queued requests cancel."""
import math

import numpy as np
import pytest

import oracle
from paper_1407_8333_amd import synth

pytestmark = pytest.mark.gpu
REL_TOL = 1e-5


def _check_against_oracle(dec, s, pm, grid, sel, nhat, weights=None):
    """Candidates of direction s of a served request against the oracle's map:
    bit-exact unweighted; weighted within 1e-5 max(|H|, mean w), CR included."""
    w64 = None if weights is None else np.asarray(weights, np.float64)
    m = oracle.hough_map(pm, grid, nhat, weights=w64)
    idx, val = oracle.candidates(m, sel.width, sel.excl, sel.sep)
    q = oracle.p0(sel.theta)
    for sb in range(idx.shape[0]):
        for r in range(2):
            valid = int(dec["valid"][s, sb, r])
            assert valid == idx[sb, r, 0], (s, sb, r)
            if not valid:
                continue
            if w64 is None:
                assert (dec["bin"][s, sb, r], dec["row"][s, sb, r]) == (idx[sb, r, 1], idx[sb, r, 2])
                assert dec["value"][s, sb, r] == val[sb, r]
                cr = float(oracle.critical_ratio(val[sb, r], pm.n_fft, sel.theta))
                assert dec["cr"][s, sb, r] == pytest.approx(cr, rel=1e-5, abs=1e-5)
            else:
                b, row = int(dec["bin"][s, sb, r]), int(dec["row"][s, sb, r])
                tol = REL_TOL * max(val[sb, r], float(np.mean(w64)))
                assert m[row, b] >= val[sb, r] - 2 * tol
                assert dec["value"][s, sb, r] == pytest.approx(val[sb, r], abs=2 * tol)
                ws, w2 = float(w64.sum()), float((w64 * w64).sum())
                cr = float(oracle.critical_ratio_weighted(val[sb, r], ws, w2, sel.theta))
                sigma = math.sqrt(q * (1 - q) * w2)
                assert abs(float(dec["cr"][s, sb, r]) - cr) <= 2 * tol / sigma + 1e-5 * (1 + abs(cr))


def _band(seed, t_fft, f_lo, n_fft):
    pm = synth.make_noise_peakmap(n_fft, t_fft, int(f_lo * t_fft) - 60, int((f_lo + 0.25) * t_fft) + 60,
                                  seed=seed)
    return pm


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_1407_8333_amd import api
    ctx = api.Context(0)
    bands = [_band(1, 8192.0, 60.0, 300), _band(2, 4096.0, 300.0, 500), _band(3, 1024.0, 700.0, 900)]
    dpms = [ctx.upload(pm) for pm in bands]
    yield ctx, bands, dpms
    for d in dpms:
        d.release()
    ctx.close()


def _requests(bands, rng):
    reqs = []
    for k in range(14):
        bi = k % 3
        pm = bands[bi]
        f_lo = pm.k_lo / pm.t_fft + 0.01
        rng_sd = [(-1e-9, 1e-10), (-1e-8, 1e-9)][k % 2]
        grid = synth.make_grid(pm, f_lo, f_lo + 0.2, *rng_sd)
        sel = synth.Selection(width=max(64, grid.nf // 8))
        n_sky = int(rng.integers(1, 24))
        sky = synth.sky_uniform(n_sky, rng)
        weighted = k % 4 == 3
        reqs.append((bi, grid, sel, sky, weighted))
    return reqs


def test_alone_equals_mix(setup):
    import torch
    from paper_1407_8333_amd import api
    ctx, bands, dpms = setup
    rng = synth.rng_for(3)
    reqs = _requests(bands, rng)
    wts = [torch.as_tensor(synth.fft_weights(pm.n_fft, rng), device="cuda") for pm in bands]
    alone = []
    for bi, grid, sel, sky, weighted in reqs:
        alone.append(api.fh_hough_candidates(ctx, dpms[bi], sky, grid, sel,
                                             weights=wts[bi] if weighted else None))
    torch.cuda.synchronize()
    srv = api.Server(ctx, hbm_budget=1 << 30, lanes=3)
    outs, ids = [], []
    done = {}
    for k, (bi, grid, sel, sky, weighted) in enumerate(reqs):
        out = torch.full((len(sky), api.n_subbands(grid, sel), 2, 8), -7, dtype=torch.int32, device="cuda")
        outs.append(out)
        ids.append(srv.submit(dpms[bi], sky, grid, sel, out, weights=wts[bi] if weighted else None, tag=k))
        if k % 3 == 2:  # requests keep arriving while others run
            for c in srv.poll():
                done[c["tag"]] = c
    for _ in range(100000):
        for c in srv.poll():
            done[c["tag"]] = c
        if len(done) == len(reqs):
            break
    srv.close()
    torch.cuda.synchronize()
    assert len(done) == len(reqs)
    lanes_used = {c["lane"] for c in done.values()}
    assert len(lanes_used) > 1
    for k in range(len(reqs)):
        assert done[k]["status"] == 0
        assert done[k]["latency_ms"] >= done[k]["queue_ms"] >= 0
        assert torch.equal(outs[k], alone[k]), k
    # every served request against the oracle on its first and last direction
    wts_host = [w.cpu().numpy() for w in wts]
    for k, (bi, grid, sel, sky, weighted) in enumerate(reqs):
        dec = api.decode_candidates(outs[k])
        for s in sorted({0, len(sky) - 1}):
            _check_against_oracle(dec, s, bands[bi], grid, sel, sky[s],
                                  weights=wts_host[bi] if weighted else None)


def test_arena_admits_by_footprint(setup):
    """Two lanes but an arena that holds one request's workspace (each request
    runs its directions one at a time, the smallest chunk): the second request
    waits for memory, not for a lane, and both finish with the results of the
    request run alone."""
    import torch
    from paper_1407_8333_amd import api
    ctx, bands, dpms = setup
    pm = bands[2]
    f_lo = pm.k_lo / pm.t_fft + 0.01
    grid = synth.make_grid(pm, f_lo, f_lo + 0.2, -1e-8, 1e-9)
    sel = synth.Selection(width=512)
    sky = synth.sky_uniform(6, synth.rng_for(12))
    ref = api.fh_hough_candidates(ctx, dpms[2], sky, grid, sel)
    one = torch.empty((1, api.n_subbands(grid, sel), 2, 8), dtype=torch.int32, device="cuda")
    big = api.Server(ctx, hbm_budget=1 << 30, lanes=2)
    big.submit(dpms[2], sky[:1], grid, sel, one, tag=0)
    big.drain()
    (c0,) = big.poll()
    big.close()
    f1 = int(c0["footprint"])  # workspace of a one-direction chunk
    assert 0 < f1 < (1 << 30)
    budget = f1 + f1 // 2
    srv = api.Server(ctx, hbm_budget=budget, lanes=2)
    outs = [torch.full_like(ref, -7) for _ in range(2)]
    srv.submit(dpms[2], sky, grid, sel, outs[0], tag=1)
    srv.submit(dpms[2], sky, grid, sel, outs[1], tag=2)
    done = {c["tag"]: c for c in srv.poll()}  # admits what fits
    st = srv.stats()
    assert st["running"] + len(done) == 1 and st["queued"] == 1, st
    assert 0 < st["bytes_in_flight"] <= budget
    for _ in range(100000):
        for c in srv.poll():
            done[c["tag"]] = c
        if len(done) == 2:
            break
    srv.close()
    assert done[1]["status"] == 0 and done[2]["status"] == 0
    assert done[1]["footprint"] == f1 and done[2]["footprint"] == f1
    torch.cuda.synchronize()
    assert torch.equal(outs[0], ref) and torch.equal(outs[1], ref)


def test_budget_admission_and_cancel(setup):
    import torch
    from paper_1407_8333_amd import _lib, api
    ctx, bands, dpms = setup
    pm = bands[1]
    f_lo = pm.k_lo / pm.t_fft + 0.01
    grid = synth.make_grid(pm, f_lo, f_lo + 0.2, -1e-8, 1e-9)
    sel = synth.Selection(width=512)
    sky = synth.sky_uniform(4, synth.rng_for(5))
    out0 = torch.empty((4, api.n_subbands(grid, sel), 2, 8), dtype=torch.int32, device="cuda")
    # a budget below one request's footprint is refused at submit
    tiny = api.Server(ctx, hbm_budget=1 << 16, lanes=2)
    with pytest.raises(_lib.FHError) as e:
        tiny.submit(dpms[1], sky, grid, sel, out0)
    assert e.value.status == _lib.FH_E_UNSUPPORTED
    tiny.close()
    # one lane: the second and third requests wait in the queue
    srv = api.Server(ctx, hbm_budget=1 << 30, lanes=1)
    outs = [torch.empty_like(out0) for _ in range(3)]
    ids = [srv.submit(dpms[1], sky, grid, sel, o, tag=k) for k, o in enumerate(outs)]
    assert srv.cancel(ids[2]) == 0
    st = srv.stats()
    assert st["queued"] + st["running"] <= 2
    done = {}
    for _ in range(100000):
        for c in srv.poll():
            done[c["tag"]] = c
        if len(done) == 3:
            break
    srv.close()
    assert done[2]["status"] == _lib.FH_E_CANCELLED
    assert done[0]["status"] == 0 and done[1]["status"] == 0
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


def test_drain_runs_every_queued_request(setup):
    import torch
    from paper_1407_8333_amd import api
    ctx, bands, dpms = setup
    pm = bands[0]
    f_lo = pm.k_lo / pm.t_fft + 0.02
    grid = synth.make_grid(pm, f_lo, f_lo + 0.1, -1e-9, 1e-10)
    sel = synth.Selection(width=256)
    skies = [synth.sky_uniform(3, synth.rng_for(40 + k)) for k in range(5)]
    outs = [torch.empty((3, api.n_subbands(grid, sel), 2, 8), dtype=torch.int32, device="cuda")
            for _ in range(5)]
    srv = api.Server(ctx, hbm_budget=1 << 30, lanes=2)
    for k in range(5):
        srv.submit(dpms[0], skies[k], grid, sel, outs[k], tag=k)
    srv.drain()
    st = srv.stats()
    assert st["queued"] == 0 and st["running"] == 0 and st["finished"] == 5
    done = srv.poll()
    assert sorted(c["tag"] for c in done) == list(range(5)) and all(c["status"] == 0 for c in done)
    srv.close()
    for k in range(5):
        ref = api.fh_hough_candidates(ctx, dpms[0], skies[k], grid, sel)
        torch.cuda.synchronize()
        assert torch.equal(outs[k], ref)
