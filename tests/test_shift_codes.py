"""Host check of the tiles' compact spin-down shift encoding on the real grids.

The tiles rebuild the row term G_{i,s0} - G_{i,s0+j} of a row block from a
per-FFT linear step floor(j q_i / 2^16), q_i = rint(((dfdot tau_i) S) 2^16),
and a 2-bit residual c in {-1, 0, 1, 2} (the kernel flags any other value).
This evaluates, in binary64 with the library's operation order, every
(FFT, row) of the 256 Hz batch grid, the large band and the four serving
T_FFT classes with both spin-down ranges, and checks the residual range."""
import numpy as np
import pytest

from paper_1407_8333_amd import synth


def _shifts(t, t0, t_fft, kf, fdot0, dfdot, rows):
    tau = t - t0
    S = (float(kf) * t_fft) * 65536.0
    fs = fdot0 + rows.astype(np.float64)[:, None] * dfdot        # [rows, 1]
    return np.rint((fs * tau[None, :]) * S).astype(np.int64)       # [rows, N]


def _residuals(t, t0, t_fft, kf, fdot0, dfdot, ns):
    nrb = (ns + 15) // 16
    rows = np.arange(nrb * 16)
    G = _shifts(t, t0, t_fft, kf, fdot0, dfdot, rows)               # [nsp, N]
    tau = t - t0
    sig = (dfdot * tau) * ((float(kf) * t_fft) * 65536.0)
    q = np.rint(sig * 65536.0).astype(np.int64)
    j = np.arange(16)[:, None]
    lin = (j * q[None, :]) >> 16                                    # floor
    c = []
    for rb in range(nrb):
        blk = G[rb * 16:(rb + 1) * 16]
        c.append(blk - blk[0:1] - lin)
    return np.concatenate(c)


CASES = [("batch-256hz", 4096.0, 6300, 256.0, (-1e-8, 1e-9)),
         ("large-1024hz", 1024.0, 25000, 1024.0, (-1e-8, 1e-9))]
for t_fft, f in ((8192.0, 40.0), (4096.0, 200.0), (2048.0, 400.0), (1024.0, 900.0)):
    n = int(round(149.0 * 86400.0 / (0.5 * t_fft)))
    for rg in ((-1e-9, 1e-10), (-1e-8, 1e-9)):
        CASES.append(("serving", t_fft, n, f, rg))


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-%d-%g" % (c[0], c[1], c[4][0]))
def test_row_residuals_fit_two_bits(case):
    _, t_fft, n_fft, f_lo, (lo, hi) = case
    t = synth.fft_times(n_fft, t_fft)
    shape = synth.Peakmap(t_fft, t, np.zeros((n_fft, 3)), np.zeros(n_fft + 1, np.int64), np.zeros(0, np.int32))
    g = synth.make_grid(shape, f_lo, f_lo + 1.0, lo, hi)
    c = _residuals(t, g.t0, t_fft, g.kf, g.fdot0, g.dfdot, g.ns)
    assert c.min() >= -1 and c.max() <= 2, (c.min(), c.max())
    # the residual really varies (the linear step alone would be wrong)
    assert c.max() > c.min()
