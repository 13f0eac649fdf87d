"""The per-voxel FP32 sum of squared residuals: its rounding against the
FP32 forward model's own error (3-pool GRE likelihood, recurrence form).

Emulated on the CPU in float32 (numpy; separate multiplies and adds, so
slightly pessimistic against the GPU's fused multiply-adds).  The claim
checked: compensating the 48-term per-voxel sum could not change the
log-likelihood visibly, because the residuals' own FP32 error, from the
forward model, is two orders of magnitude larger than the sum's rounding."""
import numpy as np

F = np.float32


def _problem(n, seed=7):
    rng = np.random.default_rng(seed)
    te = 2.0 + 2.0 * np.arange(24)
    A = rng.dirichlet([2, 5, 3], n)
    T2 = np.stack([rng.uniform(5, 15, n), rng.uniform(40, 70, n), rng.uniform(20, 40, n)], 1)
    df = rng.normal(0, 5, (n, 3))

    def s64(A, T2, df):
        z = A[:, :, None] * np.exp(-te / T2[:, :, None] + 2j * np.pi * df[:, :, None] * te * 1e-3)
        return z.sum(1)

    y = s64(A, T2, df) + 0.01 * (rng.standard_normal((n, 24)) + 1j * rng.standard_normal((n, 24)))
    y = y.real.astype(F) + 1j * y.imag.astype(F)
    # a proposal near the truth, as in a chain
    A2 = A + 0.01 * rng.standard_normal(A.shape)
    T22 = T2 * (1 + 0.02 * rng.standard_normal(T2.shape))
    df2 = df + 0.3 * rng.standard_normal(df.shape)
    ref = (np.abs(y.astype(np.complex128) - s64(A2, T22, df2)) ** 2).sum(1)
    return y, (A2, T22, df2), ref


def test_sse_rounding_is_dominated_by_the_forward_model():
    n = 4000
    y, (A, T2, df), ref = _problem(n)
    yr, yi = y.real.astype(F), y.imag.astype(F)
    d = F(2.0)
    mag = np.exp((-F(1) / T2.astype(F)) * d).astype(F)
    ang = (F(2 * np.pi) * (df.astype(F) * F(1e-3)) * d).astype(F)
    qr, qi = (mag * np.cos(ang)).astype(F), (mag * np.sin(ang)).astype(F)
    zr, zi = (A.astype(F) * qr).astype(F), (A.astype(F) * qi).astype(F)
    accr, acci = np.zeros(n, F), np.zeros(n, F)
    exact = np.zeros(n)
    for m in range(24):
        rr = (yr[:, m] - (zr[:, 0] + zr[:, 1] + zr[:, 2]).astype(F)).astype(F)
        ri = (yi[:, m] - (zi[:, 0] + zi[:, 1] + zi[:, 2]).astype(F)).astype(F)
        accr = (accr + rr * rr).astype(F)
        acci = (acci + ri * ri).astype(F)
        exact += rr.astype(np.float64) ** 2 + ri.astype(np.float64) ** 2
        zr, zi = (zr * qr - zi * qi).astype(F), (zr * qi + zi * qr).astype(F)
    two_sums = (accr + acci).astype(np.float64)
    sum_err = np.abs(two_sums - exact) / exact          # rounding of the sum alone
    fwd_err = np.abs(exact - ref) / ref                  # FP32 residuals vs FP64
    assert np.percentile(sum_err, 99) < 1e-6
    assert np.median(fwd_err) > 30 * np.median(sum_err)
    assert np.percentile(fwd_err, 99) > 30 * np.percentile(sum_err, 99)
