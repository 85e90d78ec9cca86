"""Growth rate of the numerical Cherenkov instability from a magnetic-energy
history (oracle side). TEST INFRASTRUCTURE ONLY.

The paper plots growth rates (Fig. 4b, Fig. 6c; Sec. 3.2-3.3) without saying
how they were measured. Reading taken: the amplitude growth rate is half the
least-squares slope of ln W_B(t) over the exponential phase, which starts at
the first sample above 10x the median of the first 51 samples and ends at the
first sample above 0.1 x max W_B; at least 20 samples and R^2 >= 0.95 are
required, otherwise there is no exponential phase (None).
"""
import numpy as np


def growth_rate(t, wb, n_floor=51, min_samples=20, min_r2=0.95):
    t = np.asarray(t, dtype=np.float64)
    wb = np.asarray(wb, dtype=np.float64)
    if wb.size < max(n_floor, min_samples):
        return None
    floor = np.median(wb[:n_floor])
    top = wb.max()
    above = np.nonzero(wb > 10.0 * floor)[0]
    if above.size == 0:
        return None
    i0 = int(above[0])
    end = np.nonzero(wb > 0.1 * top)[0]
    i1 = int(end[0]) if end.size else wb.size - 1
    if i1 - i0 + 1 < min_samples:
        return None
    tt = t[i0:i1 + 1]
    yy = np.log(wb[i0:i1 + 1])
    A = np.vstack([tt, np.ones_like(tt)]).T
    coef, *_ = np.linalg.lstsq(A, yy, rcond=None)
    fit = A @ coef
    ss_res = float(np.sum((yy - fit) ** 2))
    ss_tot = float(np.sum((yy - yy.mean()) ** 2))
    r2 = 1.0 - ss_res / ss_tot if ss_tot > 0 else 0.0
    if r2 < min_r2:
        return None
    return dict(rate=0.5 * float(coef[0]), t0=float(tt[0]), t1=float(tt[-1]), r2=r2,
                samples=int(tt.size))
