"""Write sampled columns of X_true for the full-size workloads.

X_true is the fixed point of the CPU oracle's double-double refinement
(Algorithm 1 without splitting) started from an FP64 eigensolve; it is the
eigenvector matrix of the stored matrix A. The full matrix is too large to
keep, so this script stores 64 columns: the 40 whose eigenvalue has the
smallest gap to its neighbours (where forward errors concentrate) and 24
spread evenly over the spectrum, plus every eigenvalue and the digest of A.

Usage: python tests/golden/make_xtrue.py CONFIG N   (e.g. 3 8192: about 30 min
on 8 cores). Calls only oracle/ and the input generator.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402


def main():
    cfg, n = int(sys.argv[1]), int(sys.argv[2])
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"xtrue_cfg{cfg}_n{n}.npz")
    t0 = time.time()
    p = workloads.make_problem(cfg, n, x0="eigh")
    print(f"problem + eigh: {time.time() - t0:.0f}s, digest {p.meta['digest'][:16]}", flush=True)
    Xh, Xl, lh, ll, hist = oracle.refine_dd(p.A, p.X0, max_iter=14, verbose=True)
    print(f"oracle refinement: {time.time() - t0:.0f}s, history {hist}", flush=True)
    order = np.argsort(lh)
    gaps = np.full(n, np.inf)
    d = np.diff(lh[order])
    gaps[order[:-1]] = np.minimum(gaps[order[:-1]], d)
    gaps[order[1:]] = np.minimum(gaps[order[1:]], d)
    small = np.argsort(gaps, kind="stable")[:40]
    spread = np.linspace(0, n - 1, 24).round().astype(int)
    cols = np.unique(np.concatenate([small, spread]))
    err0 = float(np.max(np.abs(p.X0 - oracle.sign_align(p.X0, Xh))))
    np.savez_compressed(out, digest=p.meta["digest"], config=cfg, n=n, cols=cols,
                        X_hi=Xh[:, cols], X_lo=Xl[:, cols], lam_hi=lh, lam_lo=ll,
                        history=np.array(hist), x0_err=err0)
    print(f"wrote {out}: {len(cols)} columns, X0 max-abs error {err0:.3e}", flush=True)


if __name__ == "__main__":
    main()
