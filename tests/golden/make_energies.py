"""Write reference energies of the synthetic workloads from the CPU oracle.

The lowest eigenvalues of H over a selected basis (Eq. 2) are computed by the
oracle's Davidson iteration (Sec. II-C) driven by the oracle's matrix-free
sigma (Eq. 4, generic Slater-Condon elements).  Only ``oracle`` and
``workload`` are used; nothing of the HIP library is imported.  The residual
tolerance is tighter than the workloads' 1e-6 so that the stored energies
are good to far below the 1e-8 Ha parity bar (the energy error of a Ritz
value is of order |r|^2 / gap).

Usage (from the repository root):
    python tests/golden/make_energies.py sel16
    python tests/golden/make_energies.py block20 --nstr 2500
Each run writes tests/golden/energies_<workload>[_<nstr>].json.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workload as wl  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--nstr", type=int, default=None, help="strings per spin (default: the workload's)")
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--max-space", type=int, default=20)
    args = ap.parse_args()
    W = wl.make_config(args.workload, nstr=args.nstr)
    S = oracle.OracleSystem.from_workload(W)
    t0 = time.time()
    calls = [0]

    def apply_h(X):
        calls[0] += X.shape[0]
        t = time.time()
        Y = S.sigma(X)
        print(f"  sigma of {X.shape[0]} vector(s): {time.time() - t:.1f} s", flush=True)
        return Y

    res = oracle.davidson(apply_h, S.diag(), nroots=W.nroots, tol=args.tol,
                          max_space=args.max_space, max_iter=400)
    if not res.converged:
        raise SystemExit("oracle Davidson did not converge")
    suffix = "" if args.nstr is None else f"_{args.nstr}"
    out = dict(
        what=("lowest eigenvalues (hartree, including the core energy) of H over the selected basis "
              "(Eq. 2), from the oracle's Davidson on the oracle's sigma"),
        command=" ".join(["python", "tests/golden/make_energies.py"] + sys.argv[1:]),
        workload=W.name, norb=W.norb, n_alpha=W.n_alpha, n_beta=W.n_beta,
        strings_per_spin=int(W.alpha.size), determinants=int(S.N), nroots=int(W.nroots),
        seeds=list(W.meta["seeds"]), tol_residual=args.tol, max_space=args.max_space,
        energies=[float(e) for e in res.energies],
        residuals=[float(r) for r in res.residuals],
        iterations=int(res.iterations), sigma_vectors=int(calls[0]),
        oracle_threads=oracle.num_threads(), seconds=round(time.time() - t0, 1),
    )
    path = os.path.join(HERE, f"energies_{W.name}{suffix}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["energies"], out["iterations"], "iterations")


if __name__ == "__main__":
    np.set_printoptions(precision=12)
    main()
