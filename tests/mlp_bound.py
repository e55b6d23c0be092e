"""Elementwise bound on what the BF16 rounding of the pre-activation
gradients (layers 2-4) can change in the network's parameter gradient.

Forward error analysis of the backward pass, run beside it in FP64 with
absolute values.  Both gradients share the forward pass; the rounded one
replaces dz_k by bf16(dz_k) for k = 2..4 before dW_k = dz_k x_k^T and before
the propagation g_{k-1} = W_k^T dz_k.  With u = 2^-8 (round-to-nearest-even
to 8 significant bits, after an FP32 step of 2^-24) and E_k a bound on the
difference of the two runs' dz_k:

    Q_k      = E_k + u |dz_k|          (layers 2-4; E_k elsewhere)
    |d dW_k| <= Q_k |x_k|^T,    |d db_k| <= sum over samples of E_k
    E_{k-1}  = |s'(z_{k-1})| * (|W_k|^T Q_k),    E_top = 0.

Returned in the flat parameter order of ``oracle.mlp.param_shapes``.
"""
import numpy as np

from oracle import mlp as om

U_BF16 = 2.0 ** -8 * (1.0 + 2.0 ** -15)


def grad_rounding_bound(params, F, T):
    out, cache = om.forward(params, F, bf16=True)
    T = np.asarray(T, dtype=np.float64)
    diff = out - T
    g = 2.0 * diff / diff.size
    E = np.zeros_like(g)
    parts = []
    for k in range(om.DEPTH, -1, -1):
        x_in, Wq, z = cache[k]
        dz = g if k == om.DEPTH else g * om.silu_grad(z)
        rounded = 1 <= k <= om.DEPTH - 1
        Q = E + U_BF16 * np.abs(dz) if rounded else E
        parts.append((Q @ np.abs(x_in).T, E.sum(axis=1)))
        dzq = om.bf16_round(dz) if rounded else dz
        g = Wq.T @ dzq
        if k > 0:
            E = np.abs(om.silu_grad(cache[k - 1][2])) * (np.abs(Wq).T @ Q)
    parts.reverse()
    return np.concatenate([np.concatenate([bw.ravel(), bb.ravel()]) for bw, bb in parts])
