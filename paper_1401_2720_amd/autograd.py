"""Differentiable Jacobi SVD: a torch.autograd.Function over the C ABI.

Forward: jsvd_gesvd for one matrix, jsvd_gesvd_batched for a batch of equally
sized matrices with n <= 256 (else one jsvd_gesvd per matrix).  Backward:
jsvd_svd_backward (the SVD adjoint on FP64 MFMA products).  With
recompute=True only A is kept for the backward and the forward is run again
there (less memory, one more forward).
"""
import torch

from . import _binding as B


def _forward(A, max_sweeps=30):
    """(U, S, V) of A (m, n) or (b, m, n), float64 CUDA."""
    if A.dim() == 2:
        # every non-zero status raises, as for the batched form: a result
        # that did not converge must not flow into the backward
        U, S, V, _ = B.gesvd(A, max_sweeps=max_sweeps, allow=())
        return U, S, V
    b, m, n = A.shape
    if n <= 256:
        batch = B.Batch.from_uniform(A)
        B.gesvd_batched(batch, max_sweeps=max_sweeps, restore=False)
        Ub = batch.A.view(b, n, m).transpose(-1, -2)
        Sb = batch.S.view(b, n)
        Vb = batch.V.view(b, n, n).transpose(-1, -2)
        if int(batch.status.abs().sum()) != 0:
            raise B.JsvdError(1, "jsvd_gesvd_batched")
        return Ub, Sb, Vb
    outs = [B.gesvd(A[i], max_sweeps=max_sweeps, allow=())[:3] for i in range(b)]
    return tuple(torch.stack([o[k] for o in outs]) for k in range(3))


class JacobiSVD(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, recompute=False, max_sweeps=30):
        U, S, V = _forward(A, max_sweeps)
        ctx.recompute = recompute
        ctx.max_sweeps = max_sweeps
        if recompute:
            ctx.save_for_backward(A)
        else:
            ctx.save_for_backward(U, S, V)
        ctx.set_materialize_grads(False)
        return U, S, V

    @staticmethod
    def backward(ctx, gU, gS, gV):
        if ctx.recompute:
            (A,) = ctx.saved_tensors
            U, S, V = _forward(A.detach(), ctx.max_sweeps)
        else:
            U, S, V = ctx.saved_tensors
        dA = B.svd_backward(U, S, V, gU, gS, gV)
        return dA, None, None


def svd(A, recompute=False, max_sweeps=30):
    """U, S, V with A = U diag(S) V^T (economy), differentiable.  Raises
    JsvdError when the forward does not converge within max_sweeps."""
    return JacobiSVD.apply(A, recompute, max_sweeps)
