"""GP-level compositions of the lattice calls: the marginal-likelihood
gradient step and the predictive mean.

Every solve, MVM and adjoint runs in the library's kernels; torch only
concatenates and scales columns of device tensors between the calls.
"""
from __future__ import annotations

import numpy as np

from . import cg_solve, lattice_build, lattice_mvm, lattice_mvm_grad


def mll_gradient(X, lengthscales, Y, noise: float, tol: float = 1e-2, max_iter: int = 500,
                 outputscale: float = 1.0, **build_opts):
    """Gradient of the log marginal likelihood (Section 2, eq. gp_mll) with
    respect to the log-lengthscales and the inputs, by BBMM-style stochastic
    estimation: column 0 of Y is the target y, columns 1..P are probe vectors
    z_p (e.g. Rademacher). With a = K^-1 y and u_p = K^-1 z_p (one batched CG
    solve), K = outputscale*K_lat + noise*I,

        dMLL/dtheta = 1/2 a^T dK a - 1/(2P) sum_p u_p^T dK z_p,

    which is the gradient of sum_c G_c^T K V_c with V = [a, z_1..z_P] and
    G = [a/2, -u_1/(2P), .., -u_P/(2P)]: one adjoint call (Section 4.2).
    Returns dict(dlogell=(d,), dX=(n, d) tensor, alpha, iters, rel)."""
    import torch
    lat = lattice_build(X, lengthscales, outputscale=outputscale, **build_opts)
    sol, iters, rel = cg_solve(lat, Y, noise, tol, max_iter=max_iter)
    P = Y.shape[1] - 1
    V = torch.cat([sol[:, :1], Y[:, 1:]], dim=1).contiguous()
    G = torch.cat([0.5 * sol[:, :1], (-0.5 / max(P, 1)) * sol[:, 1:]], dim=1).contiguous()
    dX, dl = lattice_mvm_grad(lat, X, V, G)
    lat.free()
    return {"dlogell": dl, "dX": dX, "alpha": sol[:, 0], "iters": iters, "rel": rel}


def predictive_mean(lat_joint, n_train: int, alpha):
    """Predictive mean at the points after the first n_train of a lattice
    built on [X; X*] (Section 2, eq. gp_pred_mean, zero prior mean): one MVM of
    [alpha; 0], restricted to the test rows. alpha: (n_train,) or
    (n_train, C) device tensor."""
    import torch
    a = alpha if alpha.dim() == 2 else alpha[:, None]
    full = torch.zeros((lat_joint.n, a.shape[1]), device=a.device, dtype=torch.float32)
    full[:n_train] = a
    out = lattice_mvm(lat_joint, full)
    mu = out[n_train:]
    return mu if alpha.dim() == 2 else mu[:, 0]
