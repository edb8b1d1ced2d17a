"""torch.autograd integration of the multiprecision determinant.

det(A) is affine in every entry, and d det / d a_ij is the cofactor C_ij
(Sec. 3: by Baur-Strassen all (N-1)x(N-1) minors are partial derivatives of
the determinant), so the gradient is adj(A)^T.  Multiprecision integers cannot
carry autograd state and float64 determinants overflow (2^1024) long before
N = 384, so the Function works on a float64 *proxy* leaf of shape (n, n):

    mant, e = MpDet.apply(proxy, A, "auto", holder)    # det(A) = mant * 2^e
    mant.backward()                                    # proxy.grad = adj(A)^T * 2^-e

`mant` is the determinant's mantissa in +-[0.5, 1) (differentiable), `e` its
exponent (not differentiable).  The backward runs mp_det_adjugate on the
stored factors; the exact multiprecision adj(A)^T is kept on `holder.adjT`
(a DeviceMp) when a holder is given.  Everything runs in libmpdet.so.

Elimination without pivoting stops at an exactly zero pivot.  The forward
reads the factorisation's info (one device-to-host copy) and raises
ZeroPivotError when a pivot before the last one is zero: det(A) itself may be
nonzero there, and the method cannot give it.  When only the last pivot u_nn
is zero the factors are complete, det(A) = 0 is exact (mant = 0, e = 0) and
the backward still returns adj(A)^T, which never divides by u_nn.
"""
from __future__ import annotations

import torch

from . import binding


class GradHolder:
    """Receives the exact multiprecision adj(A)^T from the backward pass."""

    def __init__(self):
        self.adjT = None
        self.D = None
        self.info = None


class ZeroPivotError(ArithmeticError):
    """Elimination without pivoting met an exactly zero pivot before step n
    (info = k) or an exponent overflow (info = -1)."""

    def __init__(self, info: int, n: int):
        what = "an exponent overflow" if info < 0 else f"an exactly zero pivot at step {info} of {n}"
        super().__init__(f"mp_det: the factorisation stopped at {what}; the determinant is not defined "
                         "by elimination without pivoting")
        self.info = info


class MpDet(torch.autograd.Function):
    @staticmethod
    def forward(ctx, proxy, A, path="auto", holder=None):
        n = A.rows
        LU = binding.DeviceMp(A.limbs.clone(), A.exp.clone(), A.sign.clone(), A.rows, A.cols)
        D, info = binding.factor(LU, path)
        code = int(info.item())
        if holder is not None:
            holder.info = info
        if code != 0 and code != n:
            raise ZeroPivotError(code, n)
        mant, e = binding.to_f64(D)
        dm = mant[0, n - 1].clone()
        de = e[0, n - 1].clone()
        ctx.LU, ctx.D, ctx.info, ctx.holder = LU, D, info, holder
        ctx.save_for_backward(de)
        if holder is not None:
            holder.D, holder.info = D, info
        ctx.mark_non_differentiable(de)
        return dm, de

    @staticmethod
    def backward(ctx, g_mant, g_e):
        (de,) = ctx.saved_tensors
        adjT = binding.adjugate(ctx.LU, ctx.D, ctx.info)
        if ctx.holder is not None:
            ctx.holder.adjT = adjT
        # d mant / d a_ij = C_ij 2^-e_det, converted in one kernel
        grad = binding.to_f64_scaled(adjT, de)
        return g_mant * grad, None, None, None


class MpDetBatch(torch.autograd.Function):
    """det of every matrix of a batch (mp_det_batched), with the backward of
    all of them at once (mp_det_adjugate_batched).  Inputs: one float64 proxy
    leaf per matrix (its gradient is that matrix's adj(A)^T * 2^-e_det), then
    the list of DeviceMp matrices, the path, the batched backward's schedule
    and an optional list of GradHolders.  Outputs: (mantissas [B], exponents
    [B]); a matrix whose elimination stopped before its last step raises
    ZeroPivotError."""

    @staticmethod
    def forward(ctx, mats, path, schedule, holders, *proxies):
        LUs = [binding.DeviceMp(A.limbs.clone(), A.exp.clone(), A.sign.clone(), A.rows, A.cols) for A in mats]
        Ds, _, info = binding.batched(LUs, path, minors=False)
        codes = info.cpu().tolist()
        for A, code in zip(mats, codes):
            if code != 0 and code != A.rows:
                raise ZeroPivotError(code, A.rows)
        mants, exps = [], []
        for A, D in zip(mats, Ds):
            mant, e = binding.to_f64(D)
            mants.append(mant[0, A.rows - 1])
            exps.append(e[0, A.rows - 1])
        dm, de = torch.stack(mants), torch.stack(exps)
        ctx.LUs, ctx.Ds, ctx.info, ctx.holders, ctx.schedule = LUs, Ds, info, holders, schedule
        ctx.save_for_backward(de)
        if holders is not None:
            for hd, D in zip(holders, Ds):
                hd.D, hd.info = D, info
        ctx.mark_non_differentiable(de)
        return dm, de

    @staticmethod
    def backward(ctx, g_mant, g_e):
        (de,) = ctx.saved_tensors
        adjTs, _ = binding.adjugate_batched(ctx.LUs, ctx.Ds, ctx.info, schedule=ctx.schedule)
        grads = []
        for b, adjT in enumerate(adjTs):
            if ctx.holders is not None:
                ctx.holders[b].adjT = adjT
            grads.append(g_mant[b] * binding.to_f64_scaled(adjT, de[b:b + 1]))
        return (None, None, None, None, *grads)


def mp_det_batch(mats, proxies=None, path: str = "auto", schedule: str = "persistent", holders=None):
    """Differentiable determinants of a list of DeviceMp matrices: returns
    (mantissas [B], exponents [B]); backward gives every proxy adj(A)^T 2^-e."""
    if proxies is None:
        proxies = [torch.zeros((A.rows, A.cols), dtype=torch.float64, device=A.limbs.device, requires_grad=True)
                   for A in mats]
    return MpDetBatch.apply(mats, path, schedule, holders, *proxies)


def mp_det(A, proxy=None, path: str = "auto", holder: GradHolder | None = None):
    """Differentiable determinant of a DeviceMp A: returns (mantissa, exponent)."""
    if proxy is None:
        proxy = torch.zeros((A.rows, A.cols), dtype=torch.float64, device=A.limbs.device,
                            requires_grad=True)
    return MpDet.apply(proxy, A, path, holder)
