"""Differentiable persistence diagrams on the GPU.

The forward is the library's barcode (bit-exact with the CPU oracle); the
backward is rips_backward_device: every finite bar endpoint is the length of
its simplex's critical edge (largest float32 length, ties to the smallest CNS
edge index), so its gradient flows to the two points of that edge. Births of
vertices and infinite deaths carry no gradient. The combinatorics (which bars
exist, which simplices pair) are piecewise constant in the input, so the
gradient is that of the active pairing.
"""

from __future__ import annotations

from typing import NamedTuple

import torch


class Bars(NamedTuple):
    birth: torch.Tensor          # float32, differentiable
    death: torch.Tensor          # float32 (inf = essential), differentiable
    birth_simplex: torch.Tensor  # int64 CNS index
    death_simplex: torch.Tensor  # int64 CNS index, -1 for essential classes


def _lib():
    from . import barcode_device, barcode_batched, backward_scatter
    return barcode_device, barcode_batched, backward_scatter


class _DiagramFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, max_dim, threshold, p, is_distance):
        barcode_device, _, _ = _lib()
        bars, info = barcode_device(x.detach(), max_dim=max_dim, threshold=threshold, p=p,
                                    is_distance=is_distance)
        outs = []
        simp = []
        for b, d, bs, ds in bars:
            outs += [b.clone(), d.clone()]
            simp += [bs.clone(), ds.clone()]
        ctx.save_for_backward(x, *simp)
        ctx.max_dim, ctx.is_distance = max_dim, is_distance
        ctx.mark_non_differentiable(*simp)
        ctx.info = info
        return tuple(outs + simp)

    @staticmethod
    def backward(ctx, *grads):
        _, _, backward_scatter = _lib()
        x, *simp = ctx.saved_tensors
        D1 = ctx.max_dim + 1
        g = torch.zeros_like(x, dtype=torch.float32)
        n = x.shape[0]
        m = 0 if ctx.is_distance else x.shape[1]
        for d in range(D1):
            gb, gd = grads[2 * d], grads[2 * d + 1]
            bs, ds = simp[2 * d], simp[2 * d + 1]
            if bs.shape[0] == 0 or (gb is None and gd is None):
                continue
            gb = torch.zeros(bs.shape[0], device=x.device) if gb is None else gb.float()
            gd = torch.zeros(bs.shape[0], device=x.device) if gd is None else gd.float()
            # infinite deaths carry no gradient
            gd = torch.where(ds >= 0, gd, torch.zeros_like(gd)).contiguous()
            backward_scatter(x.detach(), n, m, d, bs, ds, gb.contiguous(), gd, g)
        return g.to(x.dtype), None, None, None, None


def diagram(x: torch.Tensor, *, max_dim: int = 1, threshold: float = float("inf"), p: int = 2,
            is_distance: bool = False) -> list[Bars]:
    """Per-dimension bars of a device point cloud (n, m) float32 (or an n x n
    distance matrix with is_distance=True), differentiable in x."""
    if not x.is_cuda or x.dtype != torch.float32:
        raise ValueError("x must be a float32 CUDA tensor")
    out = _DiagramFn.apply(x.contiguous(), max_dim, threshold, p, is_distance)
    D1 = max_dim + 1
    vals, simp = out[:2 * D1], out[2 * D1:]
    return [Bars(vals[2 * d], vals[2 * d + 1], simp[2 * d], simp[2 * d + 1]) for d in range(D1)]


class _BatchedFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, offsets, n_max, max_dim, threshold, p):
        _, barcode_batched, _ = _lib()
        bb = barcode_batched(x.detach(), offsets, n_max, max_dim=max_dim, threshold=threshold,
                             p=p)
        total = int(bb.offsets_host[-1])
        birth, death = bb.birth[:total].clone(), bb.death[:total].clone()
        bs, ds = bb.birth_simplex[:total].clone(), bb.death_simplex[:total].clone()
        seg = bb.offsets.clone()
        ctx.save_for_backward(x, offsets, bs, ds, seg)
        ctx.n_max, ctx.max_dim = n_max, max_dim
        ctx.mark_non_differentiable(bs, ds, seg)
        return birth, death, bs, ds, seg

    @staticmethod
    def backward(ctx, gb, gd, *_):
        _, _, backward_scatter = _lib()
        x, offsets, bs, ds, seg = ctx.saved_tensors
        D1 = ctx.max_dim + 1
        g = torch.zeros_like(x, dtype=torch.float32)
        total = bs.shape[0]
        if total == 0:
            return g, None, None, None, None, None
        gb = torch.zeros(total, device=x.device) if gb is None else gb.float()
        gd = torch.zeros(total, device=x.device) if gd is None else gd.float()
        gd = torch.where(ds >= 0, gd, torch.zeros_like(gd))
        B = offsets.shape[0] - 1
        lens = seg[1:] - seg[:-1]                          # bars per (cloud, dim) segment
        segid = torch.repeat_interleave(torch.arange(B * D1, device=x.device), lens)
        cloud, dim = segid // D1, segid % D1
        row0 = offsets[:-1][cloud]
        for d in range(D1):
            sel = torch.nonzero(dim == d).flatten()
            if sel.numel() == 0:
                continue
            backward_scatter(x.detach(), ctx.n_max, x.shape[1], d, bs[sel].contiguous(),
                             ds[sel].contiguous(), gb[sel].contiguous(), gd[sel].contiguous(),
                             g, row0=row0[sel].contiguous())
        return g.to(x.dtype), None, None, None, None, None


def batched_diagram(x: torch.Tensor, offsets: torch.Tensor, n_max: int, *, max_dim: int = 1,
                    threshold: float = float("inf"), p: int = 2):
    """Bars of a batch of clouds in one persistent launch, differentiable in
    x. Returns (birth, death, birth_simplex, death_simplex, segment_offsets):
    flat tensors; the bars of cloud b in dimension d are
    [segment_offsets[b*(max_dim+1)+d], segment_offsets[b*(max_dim+1)+d+1])."""
    return _BatchedFn.apply(x.contiguous(), offsets, n_max, max_dim, threshold, p)


def top_persistence_loss(birth: torch.Tensor, death: torch.Tensor,
                         birth_simplex: torch.Tensor, top: int = 5) -> torch.Tensor:
    """Sum of (death - birth)^2 over the `top` finite bars of largest float32
    persistence (ties: smaller birth, then larger birth simplex index)."""
    fin = torch.isfinite(death)
    idx = torch.nonzero(fin).flatten()
    if idx.numel() == 0:
        return (birth.sum() * 0.0).to(torch.float64)
    b, d, s = birth[idx], death[idx], birth_simplex[idx]
    pers = (d.detach() - b.detach())
    # stable sorts from the last key to the first
    o = torch.argsort(-s, stable=True)
    o = o[torch.argsort(b.detach()[o], stable=True)]
    o = o[torch.argsort(-pers[o], stable=True)]
    sel = o[:top]
    diff = d[sel].to(torch.float64) - b[sel].to(torch.float64)
    return (diff * diff).sum()
