"""GPU path (through the C ABI) against the CPU oracle.

Unweighted maps and candidates must be bit-exact.  Weighted maps must satisfy
|H - H_ref| <= 1e-5 * max(|H_ref|, mean weight) cell by cell.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1407_8333_amd import synth

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    from paper_1407_8333_amd import api
    c = api.Context(0)
    yield c
    c.close()


def _api():
    from paper_1407_8333_amd import api
    return api


def _gpu_map(ctx, pm, grid, nhat, weights=None):
    import torch
    api = _api()
    dpm = ctx.upload(pm)
    if weights is None:
        m = api.fh_hough_map_i32(ctx, dpm, nhat, grid)
    else:
        w = torch.as_tensor(np.asarray(weights, np.float32), device="cuda")
        m = api.fh_hough_map_f32(ctx, dpm, nhat, w, grid)
    torch.cuda.synchronize()
    ctx.check()
    out = m.cpu().numpy()
    dpm.release()
    return out


def _assert_weighted_close(got, ref, weights):
    wbar = float(np.mean(weights))
    tol = REL_TOL * np.maximum(np.abs(ref), wbar)
    err = np.abs(got.astype(np.float64) - ref)
    bad = err > tol
    assert not bad.any(), "max err %g at %s (ref %g)" % (err.max(), np.unravel_index(err.argmax(), err.shape),
                                                        ref.flat[err.argmax()])


def test_plain_map_no_doppler_200_ffts(ctx):
    w = synth.workload("plain-50hz")
    got = _gpu_map(ctx, w.pm, w.grid, w.sky[0])
    ref = oracle.hough_map(w.pm, w.grid, w.sky[0])
    np.testing.assert_array_equal(got, ref.astype(np.int32))


def test_map_100hz_single_sky_full_size(ctx):
    w = synth.workload("sky-100hz")
    got = _gpu_map(ctx, w.pm, w.grid, w.sky[0])
    ref = oracle.hough_map(w.pm, w.grid, w.sky[0])
    np.testing.assert_array_equal(got, ref.astype(np.int32))


def test_weighted_map_100hz_full_size(ctx):
    w = synth.workload("sky-100hz")
    got = _gpu_map(ctx, w.pm, w.grid, w.sky[0], weights=w.weights)
    ref = oracle.hough_map(w.pm, w.grid, w.sky[0], weights=w.weights.astype(np.float64))
    _assert_weighted_close(got, ref, w.weights)


def _fixed_point_bits(weights, n_fft, adjacent):
    """F of the library's weight fixed point: the largest F <= 40 with
    2^(F+1) <= ((2^32 - 1) / m - N / 2) / sum w (m = 2 with adjacent bins)."""
    m = 2 if adjacent else 1
    lim = (4294967295.0 / m - 0.5 * n_fft) / float(np.sum(np.asarray(weights, np.float64)))
    f = 0
    while f < 40 and 2.0 ** (f + 1) <= lim:
        f += 1
    return f


@pytest.mark.parametrize("name,n_fft", [("sky-100hz", 1500), ("batch-256hz", None)])
def test_weighted_map_wide_weight_range(ctx, name, n_fft):
    """Weights U(0.02, 1.5), as adaptive weights near an antenna-pattern zero
    produce.  Every cell is within the stated fixed-point bound
    n_c 2^-(F+1) + 2^-24 |H| (n_c: contributions to the cell), and within
    1e-5 max(|H|, mean w) on these inputs; the candidates and their CR follow."""
    import torch
    api = _api()
    w = synth.workload(name, seed=77, n_fft=n_fft, n_sky=1)
    print("case: wide weights", name, w.pm.n_fft, flush=True)
    rng = synth.rng_for(78)
    wts = rng.uniform(0.02, 1.5, w.pm.n_fft).astype(np.float32)
    nhat = w.sky[0]
    got = _gpu_map(ctx, w.pm, w.grid, nhat, weights=wts)
    ref = oracle.hough_map(w.pm, w.grid, nhat, weights=wts.astype(np.float64))
    n_c = oracle.hough_map(w.pm, w.grid, nhat)
    adjacent = any(np.any(np.diff(w.pm.bins[w.pm.offsets[i]:w.pm.offsets[i + 1]]) == 1)
                   for i in range(w.pm.n_fft))
    F = _fixed_point_bits(wts, w.pm.n_fft, adjacent)
    err = np.abs(got.astype(np.float64) - ref)
    bound = n_c * 2.0 ** -(F + 1) + 2.0 ** -24 * np.abs(ref) + 1e-12
    assert np.all(err <= bound), (F, float((err - bound).max()))
    _assert_weighted_close(got, ref, wts)
    dpm = ctx.upload(w.pm)
    raw = api.fh_hough_candidates(ctx, dpm, w.sky, w.grid, w.sel, weights=torch.as_tensor(wts, device="cuda"))
    torch.cuda.synchronize()
    ctx.check()
    dec = api.decode_candidates(raw)
    idx, val = oracle.candidates(ref, w.sel.width, w.sel.excl, w.sel.sep)
    _check_candidates(dec, 0, idx, val, w.pm.n_fft, w.sel.theta, weighted_map=ref, weights=wts)
    dpm.release()


@pytest.mark.parametrize("seed", range(6))
def test_random_small_maps_edge_cases(ctx, seed):
    """Ragged tiles, rows not a multiple of 16, K_f from 1 to 64, empty FFTs,
    peaks far outside the band, reference time at the first FFT."""
    rng = synth.rng_for(500 + seed)
    kf = [1, 2, 10, 10, 37, 64][seed]
    n_fft = int(rng.integers(1, 40))
    t_fft = float([1024, 2048, 4096, 8192][seed % 4])
    k_lo = int(rng.integers(10_000, 200_000))
    pm = synth.random_peakmap(n_fft, t_fft, k_lo, k_lo + 300, 0.08, rng)
    if n_fft > 3:  # an empty FFT in the middle
        pm = pm.subset_ffts([i for i in range(n_fft) if i != n_fft // 2])
    f_lo = (k_lo + 40) / t_fft
    f_hi = (k_lo + 40 + int(rng.integers(1, 200))) / t_fft
    grid = synth.make_grid(pm, f_lo, f_hi, -3e-8, 2e-9, kf=kf,
                           t0=float(pm.t[0]) if seed % 2 else None)
    nhat = synth.sky_uniform(1, rng)[0]
    got = _gpu_map(ctx, pm, grid, nhat)
    ref = oracle.hough_map(pm, grid, nhat)
    np.testing.assert_array_equal(got, ref.astype(np.int32))
    wts = rng.uniform(0.5, 1.5, pm.n_fft).astype(np.float32)
    gotw = _gpu_map(ctx, pm, grid, nhat, weights=wts)
    refw = oracle.hough_map(pm, grid, nhat, weights=wts.astype(np.float64))
    _assert_weighted_close(gotw, refw, wts)


@pytest.mark.parametrize("ns,kf", [(1, 10), (2, 1), (5, 10), (6, 37), (7, 10), (17, 10), (18, 1), (19, 3), (21, 2),
                                   (22, 10), (33, 10), (38, 10), (65, 10), (67, 37)])
def test_short_last_row_block(ctx, ns, kf):
    """Grids whose last 16-row block is partly empty (1 to 15 rows of it
    exist; 1-3 rows after a full block are folded into the tiles of the block
    before, 65 and 67 rows with the folded rows past a row group): maps,
    weighted maps, candidates of both schedules and column maxima against the
    oracle."""
    import torch
    api = _api()
    rng = synth.rng_for(700 + ns * 3 + kf)
    print("case: short last row block ns=%d kf=%d" % (ns, kf), flush=True)
    t_fft = 2048.0
    pm = synth.random_peakmap(90, t_fft, 60_000, 60_400, 0.08, rng)
    dfd = (1.0 / t_fft) / (90 * t_fft / 2)
    grid = synth.Grid(kf=kf, b0=kf * 60_050, nf=kf * 300, ns=ns, fdot0=-(ns // 2) * dfd, dfdot=dfd,
                      t0=float(pm.t[45]))
    nhat = synth.sky_uniform(1, rng)[0]
    ref = oracle.hough_map(pm, grid, nhat)
    np.testing.assert_array_equal(_gpu_map(ctx, pm, grid, nhat), ref.astype(np.int32))
    wts = rng.uniform(0.5, 1.5, pm.n_fft).astype(np.float32)
    refw = oracle.hough_map(pm, grid, nhat, weights=wts.astype(np.float64))
    _assert_weighted_close(_gpu_map(ctx, pm, grid, nhat, weights=wts), refw, wts)
    sky = np.concatenate([nhat[None, :], synth.sky_uniform(2, rng)])
    sel = synth.Selection(width=max(1, grid.nf // 4))
    dpm = ctx.upload(pm)
    raw_p = api.fh_hough_candidates(ctx, dpm, sky, grid, sel, schedule=1)
    raw_0 = api.fh_hough_candidates(ctx, dpm, sky, grid, sel, schedule=0)
    torch.cuda.synchronize()
    assert torch.equal(raw_p, raw_0)
    dec = api.decode_candidates(raw_p)
    idx, val = oracle.candidates(ref, sel.width, sel.excl, sel.sep)
    _check_candidates(dec, 0, idx, val, pm.n_fft, sel.theta)
    val_c, row_c = api.fh_hough_colmax(ctx, dpm, sky[:1], grid)
    torch.cuda.synchronize()
    top = ref.max(axis=0)
    np.testing.assert_array_equal(val_c.cpu().numpy()[0], top.astype(np.float32))
    np.testing.assert_array_equal(row_c.cpu().numpy()[0], np.argmax(ref == top[None, :], axis=0))
    dpm.release()


@pytest.mark.parametrize("ns", [17, 19, 65])
def test_folded_tail_rows_equal_a_row_block_of_their_own(ctx, ns):
    """The same grid with its last 1-3 rows folded into the tiles of the row
    block before (library-chosen width) and run as a row block of their own
    (the widest 16-row tile, which leaves no LDS for them): identical
    candidates and column maxima, and the oracle's."""
    import torch
    api = _api()
    rng = synth.rng_for(900 + ns)
    print("case: folded tail ns=%d" % ns, flush=True)
    t_fft = 2048.0
    pm = synth.random_peakmap(120, t_fft, 60_000, 60_500, 0.08, rng)
    dfd = (1.0 / t_fft) / (120 * t_fft / 2)
    grid = synth.Grid(kf=10, b0=10 * 60_020, nf=10 * 450, ns=ns, fdot0=-(ns // 2) * dfd, dfdot=dfd,
                      t0=float(pm.t[60]))
    dpm = ctx.upload(pm)
    folded = ctx.plan(dpm, grid, tile_bins=1280)
    wide = ctx.plan(dpm, grid, tile_bins=4096)
    assert folded["n_row_blocks"] == (ns + 15) // 16 - 1, folded
    assert wide["n_row_blocks"] == (ns + 15) // 16 and wide["tile_bins"] == 2496, wide
    sky = synth.sky_uniform(5, rng)
    sel = synth.Selection(width=300)
    a = api.fh_hough_candidates(ctx, dpm, sky, grid, sel, tile_bins=1280)
    b = api.fh_hough_candidates(ctx, dpm, sky, grid, sel, tile_bins=4096)
    va, ra = api.fh_hough_colmax(ctx, dpm, sky, grid, tile_bins=1280)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    ref = oracle.hough_map(pm, grid, sky[2])
    top = ref.max(axis=0)
    np.testing.assert_array_equal(va.cpu().numpy()[2], top.astype(np.float32))
    np.testing.assert_array_equal(ra.cpu().numpy()[2], np.argmax(ref == top[None, :], axis=0))
    idx, val = oracle.candidates(ref, sel.width, sel.excl, sel.sep)
    _check_candidates(api.decode_candidates(a), 2, idx, val, pm.n_fft, sel.theta)
    dpm.release()


@pytest.mark.parametrize("n_fft,n_bins,nf,ns", [(48, 6000, 5600, 20), (16_500, 1000, 900, 4)])
def test_windows_of_more_than_127_peaks(ctx, n_fft, n_bins, nf, ns):
    """K_f = 1 with the widest tile: windows of hundreds of peaks, beyond the
    sizes that the window sort's counting buckets order (from 127 peaks up
    they share one bucket, ranked apart; with 16 500 FFTs the rows are sorted
    in pieces): maps, weighted maps and candidates of both schedules against
    the oracle."""
    import torch
    api = _api()
    rng = synth.rng_for(1270 + n_fft)
    print("case: windows of more than 127 peaks, %d FFTs" % n_fft, flush=True)
    t_fft = 1024.0
    pm = synth.random_peakmap(n_fft, t_fft, 60_000, 60_000 + n_bins, 0.3, rng)
    assert np.diff(pm.offsets).min() > 127
    dfd = (1.0 / t_fft) / (n_fft * t_fft / 2)
    grid = synth.Grid(kf=1, b0=60_000 + (n_bins - nf) // 2, nf=nf, ns=ns, fdot0=-(ns // 2) * dfd, dfdot=dfd,
                      t0=float(pm.t[n_fft // 2]))
    nhat = synth.sky_uniform(1, rng)[0]
    dpm = ctx.upload(pm)
    assert ctx.plan(dpm, grid)["tile_bins"] >= min(nf, 2496)
    ref = oracle.hough_map(pm, grid, nhat)
    np.testing.assert_array_equal(_gpu_map(ctx, pm, grid, nhat), ref.astype(np.int32))
    wts = rng.uniform(0.5, 1.5, pm.n_fft).astype(np.float32)
    refw = oracle.hough_map(pm, grid, nhat, weights=wts.astype(np.float64))
    _assert_weighted_close(_gpu_map(ctx, pm, grid, nhat, weights=wts), refw, wts)
    sky = np.concatenate([nhat[None, :], synth.sky_uniform(3, rng)])
    sel = synth.Selection(width=max(1, nf // 8))
    raw_p = api.fh_hough_candidates(ctx, dpm, sky, grid, sel, schedule=1, tile_bins=nf)
    raw_0 = api.fh_hough_candidates(ctx, dpm, sky, grid, sel, schedule=0, tile_bins=nf)
    torch.cuda.synchronize()
    assert torch.equal(raw_p, raw_0)
    idx, val = oracle.candidates(ref, sel.width, sel.excl, sel.sep)
    _check_candidates(api.decode_candidates(raw_p), 0, idx, val, pm.n_fft, sel.theta)
    dpm.release()


@pytest.mark.parametrize("sign,ns", [(-1.0, 19), (-1.0, 40), (0.0, 17), (0.0, 3)])
def test_descending_and_flat_spin_down_rows(ctx, sign, ns):
    """Rows whose spin-down decreases (dfdot < 0, the row terms change sign)
    and rows that all coincide (dfdot = 0: every row equals row 0, so the
    column maxima pick row 0 on the ties), with and without folded tail
    rows: maps, weighted maps, candidates and column maxima against the
    oracle."""
    import torch
    api = _api()
    rng = synth.rng_for(3300 + ns + int(sign))
    print("case: dfdot sign %g, %d rows" % (sign, ns), flush=True)
    t_fft = 2048.0
    pm = synth.random_peakmap(80, t_fft, 70_000, 70_500, 0.08, rng)
    dfd = sign * (1.0 / t_fft) / (80 * t_fft / 2)
    grid = synth.Grid(kf=10, b0=10 * 70_050, nf=10 * 400, ns=ns, fdot0=(ns // 2) * abs(dfd), dfdot=dfd,
                      t0=float(pm.t[20]))
    nhat = synth.sky_uniform(1, rng)[0]
    ref = oracle.hough_map(pm, grid, nhat)
    np.testing.assert_array_equal(_gpu_map(ctx, pm, grid, nhat), ref.astype(np.int32))
    wts = rng.uniform(0.5, 1.5, pm.n_fft).astype(np.float32)
    _assert_weighted_close(_gpu_map(ctx, pm, grid, nhat, weights=wts),
                           oracle.hough_map(pm, grid, nhat, weights=wts.astype(np.float64)), wts)
    dpm = ctx.upload(pm)
    sel = synth.Selection(width=500)
    raw = api.fh_hough_candidates(ctx, dpm, nhat[None, :], grid, sel, tile_bins=1280)
    val_c, row_c = api.fh_hough_colmax(ctx, dpm, nhat[None, :], grid, tile_bins=1280)
    torch.cuda.synchronize()
    idx, val = oracle.candidates(ref, sel.width, sel.excl, sel.sep)
    _check_candidates(api.decode_candidates(raw), 0, idx, val, pm.n_fft, sel.theta)
    top = ref.max(axis=0)
    np.testing.assert_array_equal(val_c.cpu().numpy()[0], top.astype(np.float32))
    np.testing.assert_array_equal(row_c.cpu().numpy()[0], np.argmax(ref == top[None, :], axis=0))
    if sign == 0.0:
        assert (row_c.cpu().numpy()[0] == 0).all()
    dpm.release()


def test_fft_count_limit_of_the_tile_runs(ctx):
    """A tile run holds every 16th FFT, its place in 15 bits: 524 160 FFTs are
    searched, one more is refused with FH_E_UNSUPPORTED (the peakmaps have no
    peaks; only the plan is asked for)."""
    from paper_1407_8333_amd import _lib
    for n_fft, ok in ((524_160, True), (524_161, False)):
        t = synth.fft_times(n_fft, 1024.0)
        pm = synth.Peakmap(1024.0, t, np.zeros((n_fft, 3)), np.zeros(n_fft + 1, np.int64), np.zeros(0, np.int32))
        grid = synth.Grid(kf=10, b0=10 * 60_000, nf=1000, ns=4, fdot0=0.0, dfdot=1e-12, t0=float(t[n_fft // 2]))
        dpm = ctx.upload(pm)
        if ok:
            assert ctx.plan(dpm, grid)["n_row_blocks"] == 1
        else:
            with pytest.raises(_lib.FHError) as e:
                ctx.plan(dpm, grid)
            assert e.value.status == _lib.FH_E_UNSUPPORTED
        dpm.release()


def test_zero_peaks_gives_zero_map(ctx):
    t = synth.fft_times(5, 1024.0)
    pm = synth.Peakmap(1024.0, t, np.zeros((5, 3)), np.zeros(6, np.int64), np.zeros(0, np.int32))
    grid = synth.Grid(kf=10, b0=1_000_000, nf=333, ns=19, fdot0=-1e-9, dfdot=1e-10, t0=2048.0)
    got = _gpu_map(ctx, pm, grid, np.array([0.0, 0.0, 1.0]))
    assert got.shape == (19, 333) and not got.any()


def test_noiseless_injection_reaches_n_fft(ctx):
    rng = synth.rng_for(42)
    t_fft, n_fft = 8192.0, 150
    t = synth.fft_times(n_fft, t_fft)
    v = synth.detector_velocity(t, rng)
    t0 = 0.5 * (t[0] + t[-1])
    tmp = synth.Peakmap(t_fft, t, v, np.zeros(n_fft + 1, np.int64), np.zeros(0, np.int32))
    grid = synth.make_grid(tmp, 120.0, 120.1, -1e-9, 1e-10, t0=t0)
    for _ in range(500):
        b_star = int(rng.integers(100, grid.nf - 100))
        s_star = int(rng.integers(0, grid.ns))
        inj = synth.Injection((grid.b0 + b_star) / (grid.kf * t_fft),
                              grid.fdot0 + s_star * grid.dfdot, synth.sky_uniform(1, rng)[0])
        if synth.track_is_clean(t, v, t_fft, inj, t0):
            break
    pm = synth.make_track_peakmap(t, v, t_fft, [inj], t0)
    got = _gpu_map(ctx, pm, grid, inj.nhat)
    assert got[s_star, b_star] == n_fft and got.max() == n_fft


def _candidates_ref(pm, grid, nhat, sel, weights=None):
    m = oracle.hough_map(pm, grid, nhat, weights=None if weights is None else weights.astype(np.float64))
    idx, val = oracle.candidates(m, sel.width, sel.excl, sel.sep)
    return m, idx, val


def _check_candidates(dec, s, ref_idx, ref_val, n_fft, theta, weighted_map=None, weights=None):
    n_sb = ref_idx.shape[0]
    for sb in range(n_sb):
        for r in range(2):
            valid = int(dec["valid"][s, sb, r])
            assert valid == ref_idx[sb, r, 0], (s, sb, r)
            if not valid:
                continue
            if weighted_map is None:
                assert (dec["bin"][s, sb, r], dec["row"][s, sb, r]) == (ref_idx[sb, r, 1], ref_idx[sb, r, 2])
                assert dec["value"][s, sb, r] == ref_val[sb, r]
                cr = oracle.critical_ratio(ref_val[sb, r], n_fft, theta)
                assert dec["cr"][s, sb, r] == pytest.approx(cr, rel=1e-5, abs=1e-5)
            else:
                b, row = int(dec["bin"][s, sb, r]), int(dec["row"][s, sb, r])
                # the chosen cell's exact value is within tolerance of the best
                tol = REL_TOL * max(ref_val[sb, r], float(np.mean(weights)))
                assert weighted_map[row, b] >= ref_val[sb, r] - 2 * tol
                assert dec["value"][s, sb, r] == pytest.approx(ref_val[sb, r], abs=2 * tol)
                # weighted critical ratio of the oracle's best value; the GPU's
                # value may differ by 2 tol, which moves CR by 2 tol / sigma
                w64 = np.asarray(weights, np.float64)
                ws, w2 = float(w64.sum()), float((w64 * w64).sum())
                q = oracle.p0(theta)
                sigma = math.sqrt(q * (1 - q) * w2)
                cr = float(oracle.critical_ratio_weighted(ref_val[sb, r], ws, w2, theta))
                assert abs(float(dec["cr"][s, sb, r]) - cr) <= 2 * tol / sigma + 1e-5 * (1 + abs(cr)), (sb, r)


@pytest.mark.parametrize("schedule", [0, 1])
def test_candidates_plain_50hz(ctx, schedule):
    api = _api()
    w = synth.workload("plain-50hz")
    dpm = ctx.upload(w.pm)
    raw = api.fh_hough_candidates(ctx, dpm, w.sky, w.grid, w.sel, schedule=schedule)
    dec = api.decode_candidates(raw)
    _, idx, val = _candidates_ref(w.pm, w.grid, w.sky[0], w.sel)
    _check_candidates(dec, 0, idx, val, w.pm.n_fft, w.sel.theta)
    dpm.release()


def test_candidates_batch_256hz_sampled_skies(ctx):
    """Batched (persistent) search of 12 sky directions at full size; plain and
    persistent schedules agree exactly; three directions against the oracle."""
    import torch
    api = _api()
    w = synth.workload("batch-256hz", n_sky=12)
    dpm = ctx.upload(w.pm)
    raw_p = api.fh_hough_candidates(ctx, dpm, w.sky, w.grid, w.sel, schedule=1)
    raw_0 = api.fh_hough_candidates(ctx, dpm, w.sky, w.grid, w.sel, schedule=0)
    torch.cuda.synchronize()
    assert torch.equal(raw_p, raw_0)
    dec = api.decode_candidates(raw_p)
    for s in (0, 5, 11):
        _, idx, val = _candidates_ref(w.pm, w.grid, w.sky[s], w.sel)
        _check_candidates(dec, s, idx, val, w.pm.n_fft, w.sel.theta)
    dpm.release()


def _colmax_ref(m):
    """Per-bin maximum over rows and the smallest row holding it."""
    top = m.max(axis=0)
    row = np.argmax(m == top[None, :], axis=0)
    return top, row


def test_column_maxima_batch_256hz_every_bin(ctx):
    """Column maxima of four directions at full size (583 rows = 37 row blocks
    merged by 64-bit atomics, 40960 bins), unweighted, bit for bit against the
    oracle's map in every bin; both schedules; one weighted direction within
    tolerance."""
    import torch
    api = _api()
    w = synth.workload("batch-256hz", n_sky=4)
    print("case: column maxima batch-256hz, 4 directions", flush=True)
    dpm = ctx.upload(w.pm)
    val, row = api.fh_hough_colmax(ctx, dpm, w.sky, w.grid, schedule=1)
    val0, row0 = api.fh_hough_colmax(ctx, dpm, w.sky, w.grid, schedule=0)
    torch.cuda.synchronize()
    assert torch.equal(val, val0) and torch.equal(row, row0)
    val, row = val.cpu().numpy(), row.cpu().numpy()
    for s in range(4):
        top, arg = _colmax_ref(oracle.hough_map(w.pm, w.grid, w.sky[s]))
        np.testing.assert_array_equal(val[s], top.astype(np.float32))
        np.testing.assert_array_equal(row[s], arg)
    wt = torch.as_tensor(w.weights, device="cuda")
    vw, rw = api.fh_hough_colmax(ctx, dpm, w.sky[1:2], w.grid, weights=wt)
    torch.cuda.synchronize()
    ctx.check()
    m = oracle.hough_map(w.pm, w.grid, w.sky[1], weights=w.weights.astype(np.float64))
    top, _ = _colmax_ref(m)
    vw, rw = vw.cpu().numpy()[0], rw.cpu().numpy()[0]
    tol = REL_TOL * np.maximum(top, float(np.mean(w.weights)))
    assert np.all(np.abs(vw.astype(np.float64) - top) <= tol)
    # the reported row holds a value within tolerance of the maximum
    assert np.all(m[rw, np.arange(w.grid.nf)] >= top - 2 * tol)
    dpm.release()


def test_weighted_candidates_batch_256hz(ctx):
    import torch
    api = _api()
    w = synth.workload("batch-256hz", n_sky=4)
    dpm = ctx.upload(w.pm)
    wt = torch.as_tensor(w.weights, device="cuda")
    raw_p = api.fh_hough_candidates(ctx, dpm, w.sky, w.grid, w.sel, weights=wt, schedule=1)
    raw_0 = api.fh_hough_candidates(ctx, dpm, w.sky, w.grid, w.sel, weights=wt, schedule=0)
    torch.cuda.synchronize()
    ctx.check()
    assert torch.equal(raw_p, raw_0)
    dec = api.decode_candidates(raw_p)
    for s in (0, 3):
        m, idx, val = _candidates_ref(w.pm, w.grid, w.sky[s], w.sel, weights=w.weights)
        _check_candidates(dec, s, idx, val, w.pm.n_fft, w.sel.theta, weighted_map=m, weights=w.weights)
    dpm.release()


def test_tile_width_does_not_change_results(ctx):
    import torch
    api = _api()
    w = synth.workload("sky-100hz", n_fft=800, n_sky=3)
    dpm = ctx.upload(w.pm)
    outs = [api.fh_hough_candidates(ctx, dpm, w.sky, w.grid, w.sel, tile_bins=tb)
            for tb in (64, 640, 0)]
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    dpm.release()


def test_graph_replays_match_eager(ctx):
    """A captured search replayed several times, with eager work and new sky
    vectors between replays, matches the eager result every time."""
    import torch
    api = _api()
    w = synth.workload("sky-100hz", n_fft=600, n_sky=6)
    dpm = ctx.upload(w.pm)
    st = torch.cuda.Stream()
    rng = synth.rng_for(9)
    wt = torch.as_tensor(w.weights, device="cuda")
    n_sb = api.n_subbands(w.grid, w.sel)
    out_g = torch.empty((6, n_sb, 2, 8), dtype=torch.int32, device="cuda")
    for rep in range(4):
        sky = synth.sky_uniform(6, rng)
        with torch.cuda.stream(st):
            api.fh_hough_candidates(ctx, dpm, sky, w.grid, w.sel, weights=wt, use_graph=1,
                                    out=out_g, stream=st)
            ref = api.fh_hough_candidates(ctx, dpm, sky, w.grid, w.sel, weights=wt, use_graph=0,
                                          stream=st)
        st.synchronize()
        assert torch.equal(out_g, ref), rep
        # eager work on the default stream between replays
        api.fh_hough_map_i32(ctx, dpm, sky[0], w.grid)
        torch.cuda.synchronize()
    dpm.release()


def test_window_methods_agree(ctx):
    """Binary-search, sweep and fused-front peak windows give identical
    candidates."""
    import torch
    api = _api()
    w = synth.workload("batch-256hz", n_fft=1500, n_sky=5)
    dpm = ctx.upload(w.pm)
    outs = []
    for m in (0, 1, 2):
        ctx.set_option("window_method", m)
        outs.append(api.fh_hough_candidates(ctx, dpm, w.sky, w.grid, w.sel, tile_bins=512))
    ctx.set_option("window_method", 2)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
    assert torch.equal(outs[0], outs[2])
    dpm.release()


def test_long_fft_falls_back_to_the_unfused_front(ctx):
    """An FFT with 7000 peaks does not fit the fused front's LDS (48 KB holds
    the edges of at most 6128): the library falls back to separate edge and
    window kernels on 64-bit edges; the map is still bit-exact, weighted and
    unweighted, and the front serves shorter peakmaps again afterwards."""
    rng = synth.rng_for(61)
    t_fft, n = 1024.0, 12
    k_lo = 300_000
    pm = synth.random_peakmap(n, t_fft, k_lo, k_lo + 2000, 0.1, rng)
    dense = np.arange(k_lo, k_lo + 14000, 2, dtype=np.int32)  # 7000 peaks, 2 bins apart
    segs = [pm.bins[pm.offsets[i]:pm.offsets[i + 1]] for i in range(n)]
    segs[5] = dense
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(x) for x in segs])
    big = synth.Peakmap(t_fft, pm.t, pm.v, off, np.concatenate(segs).astype(np.int32))
    assert int(np.diff(off).max()) == 7000
    grid = synth.make_grid(big, (k_lo + 3000) / t_fft, (k_lo + 3400) / t_fft, -3e-8, 2e-9)
    nhat = synth.sky_uniform(1, rng)[0]
    got = _gpu_map(ctx, big, grid, nhat)
    ref = oracle.hough_map(big, grid, nhat)
    np.testing.assert_array_equal(got, ref.astype(np.int32))
    wts = rng.uniform(0.5, 1.5, n).astype(np.float32)
    _assert_weighted_close(_gpu_map(ctx, big, grid, nhat, weights=wts),
                           oracle.hough_map(big, grid, nhat, weights=wts.astype(np.float64)), wts)
    small = pm.subset_ffts(range(n))
    g2 = synth.make_grid(small, (k_lo + 300) / t_fft, (k_lo + 700) / t_fft, -3e-8, 2e-9)
    np.testing.assert_array_equal(_gpu_map(ctx, small, g2, nhat), oracle.hough_map(small, g2, nhat).astype(np.int32))


@pytest.mark.parametrize("n_fft,nf,ns,kf", [(1, 1, 1, 10), (1, 7, 1, 1), (3, 1, 17, 10), (2, 64, 33, 64),
                                           (40, 2497, 1, 10), (25, 5000, 16, 3)])
def test_degenerate_grids(ctx, n_fft, nf, ns, kf):
    """One FFT, one fine bin, one row, row counts just past a tile, a map one
    bin wider than the widest tile: maps and candidates equal the oracle's."""
    api = _api()
    rng = synth.rng_for(7000 + n_fft * 31 + nf + ns + kf)
    t_fft = 2048.0
    k_lo = 123_456
    pm = synth.random_peakmap(n_fft, t_fft, k_lo, k_lo + 800, 0.1, rng)
    dfd = (1.0 / t_fft) / (max(n_fft, 2) * t_fft * 0.5)
    grid = synth.Grid(kf=kf, b0=kf * (k_lo + 100), nf=nf, ns=ns, fdot0=-(ns // 2) * dfd, dfdot=dfd,
                      t0=float(pm.t[0]))
    nhat = synth.sky_uniform(1, rng)[0]
    got = _gpu_map(ctx, pm, grid, nhat)
    ref = oracle.hough_map(pm, grid, nhat)
    np.testing.assert_array_equal(got, ref.astype(np.int32))
    sel = synth.Selection(width=max(1, nf // 3))
    dpm = ctx.upload(pm)
    dec = api.decode_candidates(api.fh_hough_candidates(ctx, dpm, nhat[None, :], grid, sel))
    idx, val = oracle.candidates(ref, sel.width, sel.excl, sel.sep)
    _check_candidates(dec, 0, idx, val, pm.n_fft, sel.theta)
    dpm.release()
