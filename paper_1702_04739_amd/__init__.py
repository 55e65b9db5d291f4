"""isoclust -- MI355X (gfx950) implementation of the data-parallel hot path of
"An Efficient Parallel Data Clustering Algorithm Using Isoperimetric Number of
Trees" (Javadi & Ashkboos, arXiv 1702.04739).

    parent, length, info = mst(points)                      # Sec. 2.2 step 2, Sec. 3.5
    labels, i_k, info = isoperimetric_subpartition(parent, length, k)   # Algorithms 1, 2, 4
    labels, i_k, info = cluster(points, k)                  # both

Tensors live on the GPU (torch is used for device memory and streams only);
all computation runs in the HIP library libisoclust.so through its C ABI.
"""
from __future__ import annotations

import ctypes

from . import _lib

__all__ = ["mst", "isoperimetric_subpartition", "cluster", "adjoint", "MSTIsoCost", "version"]


def _torch():
    import torch
    return torch


def _stream_ptr(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require_cuda(t, name, dtype=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))


def version() -> str:
    return _lib.load().iso_version().decode()


def mst(points, precision: str = "fp32", recheck: str = "fp32", lists: bool = True, final_round: bool = True,
        escalate: bool = True, pair_bounds: bool = False, prune: bool = True):
    """Euclidean minimum spanning tree of the rows of ``points`` (n x d, float32, GPU).

    Returns (parent int32[n] rooted at 0 with parent[0] = -1, length float64[n]
    with length[0] = 0, info dict).  ``precision`` selects the Gram screen
    ("fp32", "bf16", "fp8", or "int8" for 8-bit data); ``recheck`` the exact arithmetic that orders the edges
    ("fp32", or "fp64" for parity with the FP64 oracle).  ``lists`` and
    ``final_round`` allow the rounds that skip the full screen (neighbour lists
    from the second round, one final round for the last <= 64 components); the
    tree is the same either way.  ``escalate`` lets a low-precision screen
    whose error bound is too loose for the data hand over to the FP32 screen
    (``info["screen_precision"]`` tells which one built the tree).
    ``pair_bounds`` makes a BF16 screen use each pair's own error bound in its
    capture thresholds (it does so by itself when the norms are heavy tailed).
    ``prune`` lets a round skip the tile pairs whose bounding balls are too far
    apart to hold a needed pair (``info["tile_pairs"]`` of
    ``info["tile_pairs_full"]`` are screened); the tree is the same either way."""
    torch = _torch()
    _require_cuda(points, "points", torch.float32)
    if points.dim() != 2:
        raise ValueError("points must be 2-D")
    if points.stride(1) != 1:
        points = points.contiguous()
    n, d = points.shape
    ld = points.stride(0)
    lib = _lib.load()
    need = ctypes.c_size_t(0)
    _lib.check(lib.iso_mst_workspace_size(n, d, _lib.PRECISION[precision], ctypes.byref(need)), "iso_mst_workspace_size")
    dev = points.device
    ws = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=dev)
    parent = torch.empty(n, dtype=torch.int32, device=dev)
    length = torch.empty(n, dtype=torch.float64, device=dev)
    info = _lib.MstInfo()
    flags = ((0 if lists else _lib.MST_NO_LISTS) | (0 if final_round else _lib.MST_NO_FINAL)
             | (0 if escalate else _lib.MST_NO_ESCALATE) | (_lib.MST_PAIR_BOUNDS if pair_bounds else 0)
             | (0 if prune else _lib.MST_NO_PRUNE))
    rc = lib.iso_mst(ctypes.c_void_p(points.data_ptr()), n, d, ld, _lib.PRECISION[precision], _lib.RECHECK[recheck],
                     flags,
                     ctypes.c_void_p(parent.data_ptr()), ctypes.c_void_p(length.data_ptr()), ctypes.byref(info),
                     ctypes.c_void_p(ws.data_ptr()), int(need.value), _stream_ptr(dev))
    _lib.check(rc, "iso_mst")
    return parent, length, {"rounds": info.rounds, "list_rounds": info.list_rounds, "candidates": info.candidates,
                            "rescanned_rows": info.rescanned_rows, "mst_weight": info.mst_weight,
                            "final_components": info.final_components,
                            "screen_precision": {v: k for k, v in _lib.PRECISION.items()}[info.screen_precision],
                            "pair_bounds": bool(info.pair_bounds), "tile_pairs": info.tile_pairs,
                            "tile_pairs_full": info.tile_pairs_full}


def mst_prim(points, return_order: bool = False):
    """The paper's MST construction (Algorithm 3: Prim from vertex 0 with one
    min-reduction per step) in exact FP64: (parent, length[, order]).  For
    comparison with mst(); n sequential steps."""
    torch = _torch()
    _require_cuda(points, "points", torch.float32)
    if points.stride(1) != 1:
        points = points.contiguous()
    n, d = points.shape
    lib = _lib.load()
    need = ctypes.c_size_t(0)
    _lib.check(lib.iso_mst_prim_workspace_size(n, ctypes.byref(need)), "iso_mst_prim_workspace_size")
    dev = points.device
    ws = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=dev)
    parent = torch.empty(n, dtype=torch.int32, device=dev)
    length = torch.empty(n, dtype=torch.float64, device=dev)
    order = torch.empty(n, dtype=torch.int32, device=dev) if return_order else None
    rc = lib.iso_mst_prim(ctypes.c_void_p(points.data_ptr()), n, d, points.stride(0), ctypes.c_void_p(parent.data_ptr()),
                          ctypes.c_void_p(length.data_ptr()), ctypes.c_void_p(order.data_ptr() if order is not None else 0),
                          ctypes.c_void_p(ws.data_ptr()), int(need.value), _stream_ptr(dev))
    _lib.check(rc, "iso_mst_prim")
    return (parent, length, order) if return_order else (parent, length)


def graph_weights(points, sigma: float, phi: str = "exp", alpha: float = 0.0, omega: bool = True, potential=None):
    """Full-graph vertex weights (eq. 2.2) and potential (eq. 2.3) of the
    points: (omega0 float64[n] or None, p0 float64[n] or None).  ``potential``
    None computes p0 only when alpha > 0."""
    torch = _torch()
    _require_cuda(points, "points", torch.float32)
    if points.dim() != 2:
        raise ValueError("points must be n x d")
    if points.stride(1) != 1:
        points = points.contiguous()
    n, d = points.shape
    want_p = (alpha > 0.0) if potential is None else bool(potential)
    om = torch.empty(n, dtype=torch.float64, device=points.device) if omega else None
    p0 = torch.empty(n, dtype=torch.float64, device=points.device) if want_p else None
    rc = _lib.load().iso_graph_weights(ctypes.c_void_p(points.data_ptr()), n, d, points.stride(0), float(sigma),
                                       _lib.PHI[phi], float(alpha),
                                       ctypes.c_void_p(om.data_ptr() if om is not None else 0),
                                       ctypes.c_void_p(p0.data_ptr() if p0 is not None else 0),
                                       _stream_ptr(points.device))
    _lib.check(rc, "iso_graph_weights")
    return om, p0


def sigma_median(parent, length) -> float:
    """The lower median of the tree's n-1 edge lengths (sigma of eq. 2.1)."""
    torch = _torch()
    _require_cuda(parent, "parent", torch.int32)
    _require_cuda(length, "length", torch.float64)
    out = ctypes.c_double(0.0)
    rc = _lib.load().iso_sigma_median(ctypes.c_void_p(parent.contiguous().data_ptr()),
                                      ctypes.c_void_p(length.contiguous().data_ptr()), parent.shape[0],
                                      ctypes.byref(out), _stream_ptr(parent.device))
    _lib.check(rc, "iso_sigma_median")
    return float(out.value)


def isoperimetric_subpartition(parent, length, k: int, sigma: float | None = None, root: int = 0, phi: str = "exp",
                               bracket: str = "pow2", max_iters: int = 2000, return_clusters: bool = False,
                               omega0=None, p0=None, noalloc: bool = False):
    """Optimal k-subpartition of the weighted tree and MISO_k (eqs. 2.4, 2.6).

    ``sigma`` None (or 0) selects the lower median edge length.  ``omega0``
    (float64[n], from graph_weights with the same sigma and phi) selects the
    full-graph omega of eq. 2.2 instead of the tree degree; ``p0`` adds the
    potential of eq. 2.3.  Returns (labels int32[n] with -1 for residual
    vertices, i_k, info dict); with ``return_clusters`` the info also holds
    per-cluster num, den and size.  ``noalloc`` runs the allocation-free entry
    point (workspace in the library's fixed device array, n <= 32768)."""
    torch = _torch()
    _require_cuda(parent, "parent", torch.int32)
    _require_cuda(length, "length", torch.float64)
    parent = parent.contiguous()
    length = length.contiguous()
    n = parent.shape[0]
    if length.shape[0] != n:
        raise ValueError("parent and length differ in size")
    lib = _lib.load()
    dev = parent.device
    need = ctypes.c_size_t(0)
    ws = None
    if not noalloc:
        _lib.check(lib.iso_sub_workspace_size(n, int(k), ctypes.byref(need)), "iso_sub_workspace_size")
        ws = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    cnum = torch.empty(k, dtype=torch.float64, device=dev)
    cden = torch.empty(k, dtype=torch.float64, device=dev)
    csize = torch.empty(k, dtype=torch.int32, device=dev)
    for name, arr in (("omega0", omega0), ("p0", p0)):
        if arr is not None:
            _require_cuda(arr, name, torch.float64)
            if arr.shape[0] != n or not arr.is_contiguous():
                raise ValueError("%s must be a contiguous float64[n]" % name)
    opts = _lib.SubOpts(_lib.OMEGA["full" if omega0 is not None else "tree"], _lib.PHI[phi], _lib.BRACKET[bracket],
                        int(max_iters), omega0.data_ptr() if omega0 is not None else None,
                        p0.data_ptr() if p0 is not None else None)
    info = _lib.SubInfo()
    ik = ctypes.c_double(0.0)
    args = (ctypes.c_void_p(parent.data_ptr()), ctypes.c_void_p(length.data_ptr()), n, int(root), int(k),
            float(sigma or 0.0), ctypes.byref(opts), ctypes.c_void_p(labels.data_ptr()), ctypes.byref(ik),
            ctypes.c_void_p(cnum.data_ptr()), ctypes.c_void_p(cden.data_ptr()), ctypes.c_void_p(csize.data_ptr()),
            ctypes.byref(info))
    if noalloc:
        _lib.check(lib.iso_subpartition_noalloc(*args, _stream_ptr(dev)), "iso_subpartition_noalloc")
    else:
        _lib.check(lib.iso_subpartition(*args, ctypes.c_void_p(ws.data_ptr()), int(need.value), _stream_ptr(dev)),
                   "iso_subpartition")
    out = {f: getattr(info, f) for f, _ in _lib.SubInfo._fields_ if f != "reserved0"}
    if return_clusters:
        out.update(cluster_num=cnum, cluster_den=cden, cluster_size=csize)
    return labels, float(ik.value), out


def subpartition_all_k(parent, length, kmax: int, sigma: float | None = None, root: int = 0, phi: str = "exp",
                       bracket: str = "pow2", max_iters: int = 2000, omega0=None, p0=None, labels: bool = True):
    """The optimal k-subpartition for every k = 2 .. kmax of one tree: (i_k
    float64 numpy array indexed by k - 2, labels int32[kmax - 1, n] or None,
    passes).  Equal, k by k, to isoperimetric_subpartition."""
    torch = _torch()
    _require_cuda(parent, "parent", torch.int32)
    _require_cuda(length, "length", torch.float64)
    parent = parent.contiguous()
    length = length.contiguous()
    n = parent.shape[0]
    lib = _lib.load()
    need = ctypes.c_size_t(0)
    _lib.check(lib.iso_sub_workspace_size(n, int(kmax), ctypes.byref(need)), "iso_sub_workspace_size")
    dev = parent.device
    ws = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=dev)
    lab = torch.empty((kmax - 1, n), dtype=torch.int32, device=dev) if labels else None
    ik = (ctypes.c_double * max(kmax - 1, 1))()
    passes = ctypes.c_int32(0)
    opts = _lib.SubOpts(_lib.OMEGA["full" if omega0 is not None else "tree"], _lib.PHI[phi], _lib.BRACKET[bracket],
                        int(max_iters), omega0.data_ptr() if omega0 is not None else None,
                        p0.data_ptr() if p0 is not None else None)
    rc = lib.iso_subpartition_all_k(ctypes.c_void_p(parent.data_ptr()), ctypes.c_void_p(length.data_ptr()), n,
                                    int(root), int(kmax), float(sigma or 0.0), ctypes.byref(opts), ik,
                                    ctypes.c_void_p(lab.data_ptr() if lab is not None else 0), ctypes.byref(passes),
                                    ctypes.c_void_p(ws.data_ptr()), int(need.value), _stream_ptr(dev))
    _lib.check(rc, "iso_subpartition_all_k")
    import numpy as np
    return np.array(ik[:kmax - 1], dtype=np.float64), lab, int(passes.value)


def cluster(points, k: int, sigma: float | None = None, precision: str = "fp32", recheck: str = "fp32",
            omega: str = "tree", alpha: float = 0.0, prune: bool = True, **kw):
    """MST followed by the optimal k-subpartition (the paper's full hot path).
    ``omega="full"`` and/or ``alpha > 0`` use the full-graph weights of
    eqs. 2.2 and 2.3 (O(n^2 d) extra work); ``prune`` as in ``mst``."""
    parent, length, minfo = mst(points, precision=precision, recheck=recheck, prune=prune)
    om0 = p0 = None
    if omega == "full" or alpha > 0.0:
        if not sigma:
            sigma = sigma_median(parent, length)
        om0, p0 = graph_weights(points, sigma, phi=kw.get("phi", "exp"), alpha=alpha, omega=(omega == "full"))
    elif omega != "tree":
        raise ValueError("omega must be 'tree' or 'full'")
    labels, ik, sinfo = isoperimetric_subpartition(parent, length, k, sigma=sigma, omega0=om0, p0=p0, **kw)
    return labels, ik, {"mst": minfo, "sub": sinfo, "parent": parent, "length": length}


def adjoint(points, parent, labels, jstar: int, sigma: float, gW: float = 1.0, gI: float = 1.0, phi: str = "exp"):
    """Gradient of gW * W + gI * I with respect to the points and sigma, where W
    is the total length of the tree (parent) and I the cost (eq. 2.4) of
    cluster ``jstar`` of ``labels``, tree and subpartition held fixed.

    Returns (grad_points float32[n, d], grad_sigma float, I float)."""
    torch = _torch()
    _require_cuda(points, "points", torch.float32)
    _require_cuda(parent, "parent", torch.int32)
    _require_cuda(labels, "labels", torch.int32)
    if points.stride(1) != 1:
        points = points.contiguous()
    parent = parent.contiguous()
    labels = labels.contiguous()
    n, d = points.shape
    lib = _lib.load()
    need = ctypes.c_size_t(0)
    _lib.check(lib.iso_backward_workspace_size(n, ctypes.byref(need)), "iso_backward_workspace_size")
    dev = points.device
    ws = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=dev)
    gX = torch.empty((n, d), dtype=torch.float32, device=dev)
    gs = ctypes.c_double(0.0)
    I = ctypes.c_double(0.0)
    rc = lib.iso_backward(ctypes.c_void_p(points.data_ptr()), n, d, points.stride(0),
                          ctypes.c_void_p(parent.data_ptr()), ctypes.c_void_p(labels.data_ptr()),
                          int(jstar), float(sigma), _lib.PHI[phi], float(gW), float(gI), ctypes.c_void_p(gX.data_ptr()),
                          d, ctypes.byref(gs), ctypes.byref(I), ctypes.c_void_p(ws.data_ptr()), int(need.value),
                          _stream_ptr(dev))
    _lib.check(rc, "iso_backward")
    return gX, float(gs.value), float(I.value)


def _make_autograd():
    torch = _torch()

    class MSTIsoCost(torch.autograd.Function):
        """(W, i_k, labels) = MSTIsoCost.apply(points, sigma, k, precision, recheck, phi).

        W is the total MST length and i_k = MISO_k of the tree with phi at scale
        ``sigma`` (a 0-d tensor or float; None or 0 selects the lower median
        MST edge length, which is then a constant with no gradient).  The
        backward pass holds the tree and the optimal subpartition fixed and
        differentiates W and the cost of the cluster attaining i_k with respect
        to the points and (when given) sigma."""

        @staticmethod
        def forward(ctx, points, sigma, k, precision="fp32", recheck="fp32", phi="exp"):
            sig = 0.0 if sigma is None else float(sigma)
            parent, length, minfo = mst(points.detach(), precision=precision, recheck=recheck)
            labels, ik, sinfo = isoperimetric_subpartition(parent, length, int(k), sigma=sig, phi=phi)
            ctx.save_for_backward(points.detach(), parent, labels)
            ctx.jstar = sinfo["jstar"]
            ctx.sigma = sinfo["sigma"]  # the scale actually used (the median when sig == 0)
            ctx.phi = phi
            ctx.sigma_grad = isinstance(sigma, torch.Tensor) and sig != 0.0
            ctx.mark_non_differentiable(labels)
            W = torch.tensor(minfo["mst_weight"], dtype=torch.float64, device=points.device)
            I = torch.tensor(ik, dtype=torch.float64, device=points.device)
            return W, I, labels

        @staticmethod
        def backward(ctx, gW, gI, _glabels):
            points, parent, labels = ctx.saved_tensors
            gw = float(gW) if gW is not None else 0.0
            gi = float(gI) if gI is not None else 0.0
            gX, gs, _ = adjoint(points, parent, labels, ctx.jstar, ctx.sigma, gw, gi, ctx.phi)
            gsig = torch.tensor(gs, dtype=torch.float64, device=points.device) if ctx.sigma_grad else None
            return gX, gsig, None, None, None, None

    return MSTIsoCost


class _LazyAutograd:
    _cls = None

    def __getattr__(self, name):
        if _LazyAutograd._cls is None:
            _LazyAutograd._cls = _make_autograd()
        return getattr(_LazyAutograd._cls, name)


MSTIsoCost = _LazyAutograd()
