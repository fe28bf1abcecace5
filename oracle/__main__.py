"""Command line for the CPU oracle (test infrastructure, like the package).

    python -m oracle build --X X.npy --ell ELL.npy --out PREFIX
        lattice keys, idx, w and nbr in canonical order -> PREFIX_{keys,idx,w,nbr}.npy
    python -m oracle mvm --X X.npy --ell ELL.npy --values V.npy --out Y.npy
        outputscale * W B W^T V (eq. ski_to_bf)
    python -m oracle cg --X X.npy --ell ELL.npy --values B.npy --noise S --tol T --out X.npy
        per-column CG on outputscale * K_lat + noise * I (Section 2); iterations and
        relative residuals are printed
    python -m oracle grad --X X.npy --ell ELL.npy --values V.npy --g G.npy --out PREFIX
        gradient of sum(G * K_lat V) in X and log-lengthscales (Section 4.2)

Inputs are .npy files (X n x d, ELL d, V n x C; loaded without pickles);
options: --order r, --kernel rbf|matern32, --blur symmetric|forward|reverse,
--outputscale.
"""
import argparse
import sys

import numpy as np

import oracle

_BLUR = {"symmetric": oracle.SYMMETRIC, "forward": oracle.FORWARD, "reverse": oracle.REVERSE}
_KERNEL = {"rbf": oracle.RBF, "matern32": oracle.MATERN32}


def _load(path):
    return np.load(path, allow_pickle=False)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m oracle", description="Simplex-GP CPU oracle (fp64)")
    ap.add_argument("op", choices=["build", "mvm", "cg", "grad"])
    ap.add_argument("--X", required=True)
    ap.add_argument("--ell", required=True)
    ap.add_argument("--values")
    ap.add_argument("--g")
    ap.add_argument("--out", required=True)
    ap.add_argument("--order", type=int, default=1)
    ap.add_argument("--kernel", choices=sorted(_KERNEL), default="rbf")
    ap.add_argument("--blur", choices=sorted(_BLUR), default="symmetric")
    ap.add_argument("--outputscale", type=float, default=1.0)
    ap.add_argument("--noise", type=float, default=0.0)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--max-iter", type=int, default=500)
    a = ap.parse_args(argv)

    X = _load(a.X)
    ell = np.atleast_1d(_load(a.ell)).astype(np.float64)
    if a.op == "grad":
        if a.values is None or a.g is None:
            ap.error("grad needs --values and --g")
        if a.kernel != "rbf":
            ap.error("grad is defined for the rbf kernel")
        dX, dl = oracle.mvm_grad(X, ell, _load(a.values), _load(a.g), r=a.order, mode=_BLUR[a.blur])
        np.save(a.out + "_dX.npy", dX)
        np.save(a.out + "_dlogell.npy", dl)
        return 0
    lat = oracle.Lattice(X, ell, r=a.order, kernel=_KERNEL[a.kernel])
    if a.op == "build":
        for name, arr in zip(("keys", "idx", "w", "nbr"), lat.export()):
            np.save(f"{a.out}_{name}.npy", arr)
        print(f"n={lat.n} d={lat.d} m={lat.m}")
        return 0
    if a.values is None:
        ap.error(f"{a.op} needs --values")
    V = _load(a.values)
    if a.op == "mvm":
        np.save(a.out, lat.mvm(V, mode=_BLUR[a.blur], outputscale=a.outputscale))
        return 0
    x, iters, rel, rel_true = lat.cg(V, a.noise, a.tol, a.max_iter, mode=_BLUR[a.blur],
                                     outputscale=a.outputscale)
    np.save(a.out, x)
    for c in range(x.shape[1]):
        print(f"column {c}: iterations {int(iters[c])}, relative residual {rel[c]:.3e} "
              f"(true {rel_true[c]:.3e})")
    return 0


if __name__ == "__main__":
    sys.exit(main())
