"""Finite-size-scaling estimate of the threshold from the largest cluster
(Sec. II.A.1, eqs. (5)-(6)).

For every L the GPU sums S_max(n) over samples on a window of n around the
threshold (`nz_smax_window`, the sweep run past n*); the window average divided
by N = L^5 is P_max at fixed n, and its binomial convolution
(`nz_convolve_window`) gives P_max(p; L).  At p = p_c the rescaled curves
P_max(p; L) * L^(beta/nu) do not depend on L, so the crossings of the curves of
successive L estimate p_c.  Exponents: beta_5 = 0.8457, nu_5 = 0.5746, the 5D
values quoted in Sec. II.A.1.

    python -m paper_2607_18991_amd.fss --mask 1 --L 8 12 16 --samples 4000 2000 1000
    python -m paper_2607_18991_amd.fss --mask 1 --df 0.14079633 --L 16 20 24 28 32 --samples 2000 2000 1000 1000 1000

The second form fits the fractal dimension of the incipient cluster,
<S_max(p_c)> ~ L^d_f, at a given threshold (the estimator of Sec. II.A.3,
eq. (9), whose results are Table II of Sec. III.C).
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import nz

BETA5 = 0.8457
NU5_FSS = 0.5746


def window_for(L: int, p_lo: float, p_hi: float, k: float = 6.0):
    """[n_lo, n_hi) holding the binomial mass of every p in [p_lo, p_hi] up to k
    standard deviations."""
    N = L**5
    lo = N * p_lo - k * math.sqrt(N * p_lo * (1 - p_lo))
    hi = N * p_hi + k * math.sqrt(N * p_hi * (1 - p_hi))
    return max(1, int(math.floor(lo))), min(N, int(math.ceil(hi)) + 1)


def pmax_curve(L: int, mask: int, seed: int, samples: int, p_grid, prefill: bool = True, boundary: int = nz.NZ_FREE):
    """P_max(p; L) on p_grid, the binomial mass the window covers at each p,
    and the GPU time of the window sweep."""
    p_grid = np.asarray(p_grid, dtype=np.float64)
    N = L**5
    lo, hi = window_for(L, float(p_grid.min()), float(p_grid.max()))
    # label the sites below the window in bulk (2% below it, far more than the
    # fluctuation of the count of keys under the threshold)
    n0 = int(lo * 0.98) if prefill and lo > 64 else -1
    t0 = time.perf_counter()
    sums = nz.nz_smax_window(L, mask, seed, 0, samples, lo, hi, n0=n0, boundary=boundary)
    secs = time.perf_counter() - t0
    Q = sums.astype(np.float64) / (samples * N)
    P, cover = nz.nz_convolve_window(Q, lo, N, p_grid)
    return P, cover, {"L": L, "n_lo": lo, "n_hi": hi, "n0": n0, "samples": samples, "seconds": secs,
                      "sequential_steps": samples * (hi - 1 - max(n0, 0))}


def crossing(p, ya, yb):
    """p where ya - yb changes sign (linear interpolation between grid points);
    None if it does not on the grid."""
    d = np.asarray(ya) - np.asarray(yb)
    idx = np.nonzero(np.sign(d[:-1]) * np.sign(d[1:]) < 0)[0]
    if len(idx) == 0:
        return None
    i = idx[len(idx) // 2]
    return float(p[i] - d[i] * (p[i + 1] - p[i]) / (d[i + 1] - d[i]))


def estimate(mask: int, Ls, samples, p_grid, seed: int = 0xF55, beta_over_nu: float = BETA5 / NU5_FSS,
             boundary: int = nz.NZ_FREE):
    """Rescaled curves for every L and the crossings of successive L."""
    p_grid = np.asarray(p_grid, dtype=np.float64)
    curves, runs = {}, []
    for L, S in zip(Ls, samples):
        P, cover, info = pmax_curve(L, mask, seed + L, S, p_grid, boundary=boundary)
        if cover.min() < 1 - 1e-6:
            raise RuntimeError(f"window of L={L} misses binomial mass {1 - cover.min():.2e}")
        curves[L] = P * L**beta_over_nu
        runs.append(info)
    pairs = []
    for a, b in zip(Ls, Ls[1:]):
        pairs.append({"L": [a, b], "p": crossing(p_grid, curves[a], curves[b])})
    found = [c["p"] for c in pairs if c["p"] is not None]
    return {"mask": mask, "boundary": boundary, "beta_over_nu": beta_over_nu, "crossings": pairs,
            "p_c": float(np.mean(found)) if found else None,
            "spread": float(np.std(found)) if len(found) > 1 else None,
            "runs": runs, "p_grid": p_grid.tolist(), "curves": {str(L): c.tolist() for L, c in curves.items()}}


def smax_at(L: int, mask: int, p: float, samples: int, seed: int, boundary: int = nz.NZ_FREE):
    """<S_max>(p; L): the window of n around p*N holding the binomial mass of p,
    convolved at p and multiplied by N."""
    P, cover, info = pmax_curve(L, mask, seed, samples, [p], boundary=boundary)
    if cover[0] < 1 - 1e-6:
        raise RuntimeError(f"window of L={L} misses binomial mass {1 - cover[0]:.2e}")
    return float(P[0]) * L**5, info


def df_estimate(mask: int, p_c: float, Ls, samples, seed: int = 0xDF5, boundary: int = nz.NZ_FREE):
    """Fractal dimension of the incipient cluster (Sec. II.A.3, eq. (9); Sec. III.C, Table II):
    the least-squares slope of ln <S_max(p_c)> against ln L, with its standard
    error from the fit residuals."""
    pts, runs = [], []
    for L, S in zip(Ls, samples):
        m, info = smax_at(L, mask, p_c, S, seed + L, boundary)
        pts.append((math.log(L), math.log(m)))
        runs.append(dict(info, smax=m))
    x = np.array([a for a, _ in pts])
    y = np.array([b for _, b in pts])
    A = np.vstack([x, np.ones_like(x)]).T
    coef, res, _, _ = np.linalg.lstsq(A, y, rcond=None)
    dof = max(1, len(x) - 2)
    sigma2 = float(res[0]) / dof if len(res) else 0.0
    se = math.sqrt(sigma2 / float(((x - x.mean()) ** 2).sum())) if len(x) > 2 else None
    return {"mask": mask, "boundary": boundary, "p_c": p_c, "d_f": float(coef[0]), "d_f_stderr": se, "runs": runs}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--mask", type=lambda s: int(s, 0), default=1)
    ap.add_argument("--L", type=int, nargs="+", default=[8, 12, 16])
    ap.add_argument("--samples", type=int, nargs="+", default=[4000, 2000, 1000])
    ap.add_argument("--p", type=float, nargs=3, default=[0.1375, 0.1440, 0.0001], metavar=("LO", "HI", "STEP"))
    ap.add_argument("--seed", type=lambda s: int(s, 0), default=0xF55)
    ap.add_argument("--df", type=float, default=None, metavar="P_C",
                    help="fit the fractal dimension at this threshold instead of locating the crossing")
    ap.add_argument("--periodic", action="store_true", help="periodic boundaries (default: free)")
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    bc = nz.NZ_PERIODIC if args.periodic else nz.NZ_FREE
    if args.df is not None:
        print(json.dumps(df_estimate(args.mask, args.df, args.L, args.samples, args.seed, bc)), flush=True)
        return
    p = np.arange(args.p[0], args.p[1] + args.p[2] / 2, args.p[2])
    res = estimate(args.mask, args.L, args.samples, p, args.seed, boundary=bc)
    res.pop("curves")
    res.pop("p_grid")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
