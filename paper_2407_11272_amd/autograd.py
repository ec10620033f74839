"""Differentiable voxelization: ``torch.autograd.Function`` wrappers whose forward
and backward both run in the HIP library (Section 2.4 of arXiv 2407.11272 uses the
gradient of the voxelization with respect to the mesh vertices)."""
from __future__ import annotations

import torch

from . import api


class WindingNumber(torch.autograd.Function):
    """W = winding number of (V, F) at the centres of ``grid`` (or the rows of ``Q``);
    differentiable in V.  Backward recomputes solid angles per tile (no stored
    point x face matrix) and returns dL/dV.  Optional device ``strips`` (from
    ``wn_build_strips``) select the strip-order forward, and ``pairs`` (from
    ``wn_build_face_pairs``) the adjoint with two faces per lane and shared vertex sums;
    both depend only on F, so a loop over vertex positions builds them once."""

    @staticmethod
    def forward(ctx, V, F, grid=None, Q=None, strips=None, pairs=None):
        ctx.save_for_backward(V, F, Q, pairs)
        ctx.grid = grid
        if strips is not None:
            return api.wn_voxelize_strips(V, F, strips, grid=grid, Q=Q)
        return api.wn_voxelize(V, F, grid=grid, Q=Q)

    @staticmethod
    def backward(ctx, gW):
        V, F, Q, pairs = ctx.saved_tensors
        g = gW.contiguous().reshape(-1).to(torch.float32)
        dLdV = api.wn_backward(V, F, g, grid=ctx.grid, Q=Q, pairs=pairs)
        return dLdV, None, None, None, None, None


class NaiveWindingNumber(torch.autograd.Function):
    """The naive flux sum of Eq. 4 (centroid samples), differentiable in V; the surrogate
    the paper uses for morphing because its vertex gradients do not vanish."""

    @staticmethod
    def forward(ctx, V, F, grid=None, Q=None):
        ctx.save_for_backward(V, F, Q)
        ctx.grid = grid
        return api.wn_voxelize_naive(V, F, grid=grid, Q=Q)

    @staticmethod
    def backward(ctx, gW):
        V, F, Q = ctx.saved_tensors
        g = gW.contiguous().reshape(-1).to(torch.float32)
        return api.wn_backward_naive(V, F, g, grid=ctx.grid, Q=Q), None, None, None


class SigmoidOccupancy(torch.autograd.Function):
    """occ = sigmoid(k (W - tau)); forward and backward (g k occ (1 - occ)) both in the
    HIP library (wn_occupancy, wn_occupancy_backward)."""

    @staticmethod
    def forward(ctx, W, tau: float = 0.5, k: float = 50.0):
        W = W.contiguous()
        occ = api.wn_occupancy(W, "sigmoid", tau, k)
        ctx.save_for_backward(W)
        ctx.tau, ctx.k = tau, k
        return occ

    @staticmethod
    def backward(ctx, g):
        (W,) = ctx.saved_tensors
        g = g.contiguous().to(torch.float32)
        return api.wn_occupancy_backward(W, g, ctx.tau, ctx.k), None, None


def winding_number(V, F, grid=None, Q=None, strips=None, pairs=None):
    return WindingNumber.apply(V, F, grid, Q, strips, pairs)


def naive_winding_number(V, F, grid=None, Q=None):
    return NaiveWindingNumber.apply(V, F, grid, Q)


def soft_occupancy(V, F, grid=None, Q=None, tau: float = 0.5, k: float = 50.0, strips=None, pairs=None):
    return SigmoidOccupancy.apply(WindingNumber.apply(V, F, grid, Q, strips, pairs), tau, k)
