"""MI355X (gfx950) long-range P3T tree force of PeTar, as a C-ABI library.

The functions below carry the names of the C entry points of
``include/petar.h`` and only marshal arguments: every step of the tree
build, walk and force runs in the HIP kernels of ``libpetar.so``. PyTorch
provides device memory and the stream. Importing this package fails loudly
when the HIP library has not been built.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

from . import _capi
from ._capi import (PETAR_E_INTERNAL, PETAR_E_INVALID, PETAR_E_NB_OVERFLOW, PETAR_E_NODEVICE,
                    PETAR_E_NOMEM, PETAR_E_STATE, PETAR_FP64, PETAR_MIXED, PETAR_NO_DEVICE,
                    PETAR_OK)

_lib = _capi.load()

__all__ = [
    "PetarError", "Context", "petar_create", "petar_destroy", "petar_set_params",
    "petar_get_params", "petar_changeover_radii", "petar_tree_build", "petar_batch_build",
    "petar_force_long", "petar_set_targets", "petar_step_graph", "petar_nb_filter",
    "petar_clusters", "petar_clusters_noalloc",
    "petar_force_long_kick", "petar_groups", "petar_kick", "petar_artificial_make",
    "petar_tidal_fit", "petar_tidal_eval",
    "art_points",
    "petar_copy_counts", "petar_get_stats", "petar_autotune", "petar_autotune_lookup",
    "petar_autotune_batch", "petar_autotune_lookup_batch", "launch_config", "TUNED_CACHE", "petar_last_error", "PETAR_MIXED", "PETAR_FP64",
    "PETAR_NO_DEVICE", "lib_path",
]


def lib_path() -> str:
    return _capi.LIB_PATH


class PetarError(RuntimeError):
    def __init__(self, status: int, message: str, required: Optional[int] = None):
        self.status = status
        self.required = required
        super().__init__("%s: %s" % (_capi.STATUS_NAMES.get(status, str(status)), message))


class Context:
    """Owns a petar_ctx handle (destroyed with the object)."""

    def __init__(self, handle: ctypes.c_void_p, device: int, stream):
        self.handle = handle
        self.device = device
        self.stream = stream
        # held by the object: module globals may already be gone when a
        # context is collected at interpreter exit
        self._destroy = _lib.petar_destroy

    def __del__(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._destroy(self.handle)
            self.handle = None


def petar_last_error(ctx: Optional[Context] = None) -> str:
    msg = _lib.petar_last_error(ctx.handle if ctx else None)
    return msg.decode() if msg else ""


def _check(status: int, ctx: Optional[Context], required: Optional[int] = None) -> None:
    if status != PETAR_OK:
        raise PetarError(status, petar_last_error(ctx), required)


def _dptr(t: Optional[torch.Tensor], dtype: torch.dtype, shape, name: str, device: int):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if t.device.type != "cuda" or t.device.index != device:
        raise ValueError("%s must live on cuda:%d" % (name, device))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


def petar_create(device: int = 0, stream: Optional[torch.cuda.Stream] = None) -> Context:
    """Context on `device` whose work goes to `stream` (torch's current by default).
    device = PETAR_NO_DEVICE gives a validation-only context."""
    h = ctypes.c_void_p()
    sp = None
    if device != PETAR_NO_DEVICE:
        if stream is None:
            stream = torch.cuda.current_stream(device)
        sp = ctypes.c_void_p(stream.cuda_stream)
    _check(_lib.petar_create(ctypes.byref(h), device, sp), None)
    return Context(h, device, stream)


def petar_destroy(ctx: Context) -> None:
    if ctx.handle is not None and ctx.handle.value:
        _check(_lib.petar_destroy(ctx.handle), None)
        ctx.handle = None


def petar_set_params(ctx: Context, **kw) -> None:
    p = _capi.petar_params()
    _check(_lib.petar_get_params(ctx.handle, ctypes.byref(p)), ctx)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    _check(_lib.petar_set_params(ctx.handle, ctypes.byref(p)), ctx)


def petar_get_params(ctx: Context) -> dict:
    p = _capi.petar_params()
    _check(_lib.petar_get_params(ctx.handle, ctypes.byref(p)), ctx)
    return {name: getattr(p, name) for name, _ in p._fields_}


def petar_changeover_radii(ctx: Context, mass: torch.Tensor, r_in_ref: float, r_out_ref: float,
                           search_factor: float = 1.2, vel: Optional[torch.Tensor] = None,
                           cr_dt: float = 0.0, out=None):
    """(r_in, r_out, r_search) per particle (eq. rcut; eq. rnb if vel is given)."""
    n = mass.shape[0]
    dev = ctx.device
    if out is None:
        out = tuple(torch.empty(n, dtype=torch.float64, device="cuda:%d" % dev) for _ in range(3))
    args = [_dptr(mass, torch.float64, (n,), "mass", dev),
            _dptr(vel, torch.float64, (3, n), "vel", dev)]
    outs = [_dptr(o, torch.float64, (n,), nm, dev) for o, nm in zip(out, ("r_in", "r_out", "r_search"))]
    _check(_lib.petar_changeover_radii(ctx.handle, args[0], args[1], n, float(r_in_ref),
                                       float(r_out_ref), float(search_factor), float(cr_dt), *outs),
           ctx)
    return out


def petar_tree_build(ctx: Context, pos: torch.Tensor, mass: torch.Tensor, theta: float,
                     leaf_size: int) -> None:
    """Octree of the particles pos (3, N), mass (N,)."""
    n = mass.shape[0] if mass.dim() == 1 else -1
    _check(_lib.petar_tree_build(ctx.handle, _dptr(pos, torch.float64, (3, n), "pos", ctx.device),
                                 _dptr(mass, torch.float64, (n,), "mass", ctx.device), n,
                                 float(theta), int(leaf_size)), ctx)


def petar_batch_build(ctx: Context, sys_offsets, pos: torch.Tensor, mass: torch.Tensor,
                      theta: float, leaf_size: int) -> None:
    """One octree per system; system s owns particles sys_offsets[s]:sys_offsets[s+1]."""
    offs = [int(v) for v in sys_offsets]
    n_sys = len(offs) - 1
    n = mass.shape[0] if mass.dim() == 1 else -1
    arr = (ctypes.c_int64 * len(offs))(*offs)
    _check(_lib.petar_batch_build(ctx.handle, n_sys, arr,
                                  _dptr(pos, torch.float64, (3, n), "pos", ctx.device),
                                  _dptr(mass, torch.float64, (n,), "mass", ctx.device),
                                  float(theta), int(leaf_size)), ctx)


def petar_set_targets(ctx: Context, target: Optional[torch.Tensor]) -> None:
    """Restrict the next force calls on the current tree to the particles
    with target[i] != 0 (uint8 (N,)); None: every particle. The tensor must
    stay alive until those calls return. See petar.h."""
    if target is not None and target.dim() != 1:
        raise ValueError("target must be one-dimensional (N,)")
    _check(_lib.petar_set_targets(ctx.handle, _dptr(target, torch.uint8, None, "target",
                                                    ctx.device)), ctx)
    ctx._target = target  # kept alive with the context


def petar_force_long(ctx: Context, group_size: int, r_in: torch.Tensor, r_out: torch.Tensor,
                     r_search: torch.Tensor, acc: Optional[torch.Tensor] = None,
                     pot: Optional[torch.Tensor] = None, nb_capacity: Optional[int] = None,
                     kick: Optional[tuple] = None):
    """Long-range acceleration (3, N) and potential (N,) in input order.

    With nb_capacity (int), also returns the neighbour lists as
    (offsets int64 [N+1], idx int32 [total]). If the capacity is too small a
    PetarError with status PETAR_E_NB_OVERFLOW and `.required` is raised;
    acc and pot are complete in that case. With kick = (vel, dt), vel
    (3, N) is kicked in place by dt * acc in the same launch
    (petar_force_long_kick).
    """
    n = r_in.shape[0]
    dev = ctx.device
    d = "cuda:%d" % dev
    if acc is None:
        acc = torch.empty((3, n), dtype=torch.float64, device=d)
    if pot is None:
        pot = torch.empty(n, dtype=torch.float64, device=d)
    nb = None
    offsets = idx = None
    if nb_capacity is not None:
        offsets = torch.empty(n + 1, dtype=torch.int64, device=d)
        idx = torch.empty(max(int(nb_capacity), 1), dtype=torch.int32, device=d)
        nb = _capi.petar_nblist(offsets.data_ptr(), idx.data_ptr(), int(nb_capacity), 0)
    args = (ctx.handle, int(group_size), _dptr(r_in, torch.float64, (n,), "r_in", dev),
            _dptr(r_out, torch.float64, (n,), "r_out", dev),
            _dptr(r_search, torch.float64, (n,), "r_search", dev),
            _dptr(acc, torch.float64, (3, n), "acc", dev),
            _dptr(pot, torch.float64, (n,), "pot", dev),
            ctypes.byref(nb) if nb is not None else None)
    if kick is None:
        st = _lib.petar_force_long(*args)
    else:
        vel, dt = kick
        st = _lib.petar_force_long_kick(*args, _dptr(vel, torch.float64, (3, n), "vel", dev),
                                        float(dt))
    _check(st, ctx, nb.required if nb is not None else None)
    if nb is None:
        return acc, pot
    return acc, pot, (offsets, idx[: nb.required])


def petar_step_graph(ctx: Context, pos: torch.Tensor, mass: torch.Tensor, theta: float,
                     leaf_size: int, group_size: int, r_in: torch.Tensor, r_out: torch.Tensor,
                     r_search: torch.Tensor, acc: torch.Tensor, pot: torch.Tensor,
                     sys_offsets=None, nb=None):
    """Tree build + long-range force as a captured, replayed hipGraph.

    The output tensors (and nb = (offsets, idx) if given) must be the same
    objects on every call for the graph to be replayed. Returns the number of
    neighbour entries (or None).
    """
    n = mass.shape[0]
    dev = ctx.device
    n_sys, arr = 0, None
    if sys_offsets is not None:
        offs = [int(v) for v in sys_offsets]
        n_sys = len(offs) - 1
        arr = (ctypes.c_int64 * len(offs))(*offs)
    nbs = None
    if nb is not None:
        off_t, idx_t = nb
        nbs = _capi.petar_nblist(off_t.data_ptr(), idx_t.data_ptr(), idx_t.numel(), 0)
    st = _lib.petar_step_graph(ctx.handle, n_sys, arr,
                               _dptr(pos, torch.float64, (3, n), "pos", dev),
                               _dptr(mass, torch.float64, (n,), "mass", dev), n, float(theta),
                               int(leaf_size), int(group_size),
                               _dptr(r_in, torch.float64, (n,), "r_in", dev),
                               _dptr(r_out, torch.float64, (n,), "r_out", dev),
                               _dptr(r_search, torch.float64, (n,), "r_search", dev),
                               _dptr(acc, torch.float64, (3, n), "acc", dev),
                               _dptr(pot, torch.float64, (n,), "pot", dev),
                               ctypes.byref(nbs) if nbs is not None else None)
    _check(st, ctx, nbs.required if nbs is not None else None)
    return nbs.required if nbs is not None else None


def _nonempty(idx: torch.Tensor, d: str) -> torch.Tensor:
    # an empty list still needs a valid device pointer
    return idx if idx.numel() > 0 else torch.zeros(1, dtype=torch.int32, device=d)


def petar_nb_filter(ctx: Context, pos: torch.Tensor, vel: torch.Tensor, mass: torch.Tensor,
                    r_nb: torch.Tensor, c_v: float, offsets: torch.Tensor, idx: torch.Tensor,
                    capacity: Optional[int] = None):
    """Second-stage neighbour filter (Kepler pericentre < c_v * r_nb,i) of
    the candidate CSR (offsets int64 [N+1], idx int32). Returns the kept CSR
    (offsets int64 [N+1], idx int32 [kept]); with a capacity below the kept
    count a PetarError PETAR_E_NB_OVERFLOW with ``.required`` is raised."""
    n = mass.shape[0]
    dev = ctx.device
    d = "cuda:%d" % dev
    cap = int(idx.numel()) if capacity is None else int(capacity)
    out_off = torch.empty(n + 1, dtype=torch.int64, device=d)
    out_idx = torch.empty(max(cap, 1), dtype=torch.int32, device=d)
    nbs = _capi.petar_nblist(out_off.data_ptr(), out_idx.data_ptr(), cap, 0)
    st = _lib.petar_nb_filter(ctx.handle, n, _dptr(pos, torch.float64, (3, n), "pos", dev),
                              _dptr(vel, torch.float64, (3, n), "vel", dev),
                              _dptr(mass, torch.float64, (n,), "mass", dev),
                              _dptr(r_nb, torch.float64, (n,), "r_nb", dev), float(c_v),
                              _dptr(offsets, torch.int64, (n + 1,), "offsets", dev),
                              _dptr(_nonempty(idx, d), torch.int32, None, "idx", dev),
                              ctypes.byref(nbs))
    _check(st, ctx, nbs.required)
    return out_off, out_idx[: nbs.required]


def petar_clusters(ctx: Context, offsets: torch.Tensor, idx: torch.Tensor):
    """Clusters of the neighbour CSR: (label int32 [N], cluster offsets
    int64 [n_clusters + 1], members int32 [N]); see petar.h."""
    return _clusters(_lib.petar_clusters, ctx, offsets, idx)


def petar_clusters_noalloc(ctx: Context, offsets: torch.Tensor, idx: torch.Tensor, out=None):
    """petar_clusters with the library's fixed scratch (N <= 2^20, no device
    allocation inside the call). `out` = (label, cl_offsets, members) of
    sizes N, N + 1, N may be passed in to allocate nothing here either."""
    return _clusters(_lib.petar_clusters_noalloc, ctx, offsets, idx, out)


def _clusters(fn, ctx: Context, offsets: torch.Tensor, idx: torch.Tensor, out=None):
    n = offsets.shape[0] - 1
    dev = ctx.device
    d = "cuda:%d" % dev
    if out is None:
        out = (torch.empty(n, dtype=torch.int32, device=d),
               torch.empty(n + 1, dtype=torch.int64, device=d),
               torch.empty(n, dtype=torch.int32, device=d))
    label, cl, members = out
    nc = ctypes.c_int64(0)
    st = fn(ctx.handle, n, _dptr(offsets, torch.int64, (n + 1,), "offsets", dev),
            _dptr(_nonempty(idx, d), torch.int32, None, "idx", dev),
            _dptr(label, torch.int32, (n,), "label", dev),
            _dptr(cl, torch.int64, (n + 1,), "cl_offsets", dev),
            _dptr(members, torch.int32, (n,), "members", dev), ctypes.byref(nc))
    _check(st, ctx)
    return label, cl[: nc.value + 1], members



def petar_groups(ctx: Context, pos: torch.Tensor, vel: torch.Tensor, mass: torch.Tensor,
                 r_in: torch.Tensor, theta: float, offsets: torch.Tensor, idx: torch.Tensor):
    """SDAR groups (r_ij < theta max(r_in,i, r_in,j)) among the candidate
    CSR: (label int32 [N], group offsets int64 [n_groups + 1], members int32
    [N], pairs int32 [2, n_pairs]: the bound two-member groups); see
    petar.h."""
    n = offsets.shape[0] - 1
    dev = ctx.device
    d = "cuda:%d" % dev
    label = torch.empty(n, dtype=torch.int32, device=d)
    go = torch.empty(n + 1, dtype=torch.int64, device=d)
    members = torch.empty(n, dtype=torch.int32, device=d)
    cap = max(n // 2, 1)
    pairs = torch.empty((2, cap), dtype=torch.int32, device=d)
    ng, npair = ctypes.c_int64(0), ctypes.c_int64(0)
    st = _lib.petar_groups(ctx.handle, n, _dptr(pos, torch.float64, (3, n), "pos", dev),
                           _dptr(vel, torch.float64, (3, n), "vel", dev),
                           _dptr(mass, torch.float64, (n,), "mass", dev),
                           _dptr(r_in, torch.float64, (n,), "r_in", dev), float(theta),
                           _dptr(offsets, torch.int64, (n + 1,), "offsets", dev),
                           _dptr(_nonempty(idx, d), torch.int32, None, "idx", dev),
                           ctypes.c_void_p(label.data_ptr()), ctypes.c_void_p(go.data_ptr()),
                           ctypes.c_void_p(members.data_ptr()), ctypes.byref(ng),
                           ctypes.c_void_p(pairs.data_ptr()), cap, ctypes.byref(npair))
    _check(st, ctx)
    return label, go[: ng.value + 1], members, pairs[:, : npair.value].contiguous()


def petar_kick(ctx: Context, vel: torch.Tensor, acc: torch.Tensor, dt: float) -> torch.Tensor:
    """vel += dt * acc in place ([3, N] FP64); returns vel."""
    n = vel.shape[1]
    dev = ctx.device
    st = _lib.petar_kick(ctx.handle, n, _dptr(vel, torch.float64, (3, n), "vel", dev),
                         _dptr(acc, torch.float64, (3, n), "acc", dev), float(dt))
    _check(st, ctx)
    return vel

def art_points(order: int) -> int:
    """Measure points of the order-2 (4) or order-3 (8) tidal tensor."""
    if order not in (2, 3):
        raise ValueError("order must be 2 or 3")
    return 4 if order == 2 else 8


def petar_artificial_make(ctx: Context, pos: torch.Tensor, vel: torch.Tensor, mass: torch.Tensor,
                          r_in: torch.Tensor, r_out: torch.Tensor, r_search: torch.Tensor,
                          pairs: torch.Tensor, order: int = 3, c_d: float = 1.0) -> dict:
    """Set of the long-range force with artificial particles for the bound
    pairs pairs[2, n_pair] (int32): dict(pos (3, n_out), mass, r_in, r_out,
    r_search, src (int32), target (uint8: 0 for the pseudoparticles, which
    are sources only; for petar_set_targets), frame (4, n_pair), pair_of (N,)
    int32, n_single); see petar.h."""
    n = mass.shape[0]
    dev = ctx.device
    d = "cuda:%d" % dev
    if pairs.dim() != 2 or pairs.shape[0] != 2:
        raise ValueError("pairs must have shape (2, n_pair)")
    n_pair = pairs.shape[1]
    n_out = n + n_pair * (art_points(order) + 2)
    out = dict(pos=torch.empty((3, n_out), dtype=torch.float64, device=d),
               mass=torch.empty(n_out, dtype=torch.float64, device=d),
               r_in=torch.empty(n_out, dtype=torch.float64, device=d),
               r_out=torch.empty(n_out, dtype=torch.float64, device=d),
               r_search=torch.empty(n_out, dtype=torch.float64, device=d),
               src=torch.empty(n_out, dtype=torch.int32, device=d),
               target=torch.empty(n_out, dtype=torch.uint8, device=d),
               frame=torch.empty((4, n_pair), dtype=torch.float64, device=d),
               pair_of=torch.empty(n, dtype=torch.int32, device=d),
               n_single=n - 2 * n_pair, order=order)
    st_ = _capi.petar_art_set(out["pos"].data_ptr(), out["mass"].data_ptr(),
                              out["r_in"].data_ptr(), out["r_out"].data_ptr(),
                              out["r_search"].data_ptr(), out["src"].data_ptr(), n_out,
                              out["target"].data_ptr())
    frame = out["frame"]
    st = _lib.petar_artificial_make(
        ctx.handle, n, _dptr(pos, torch.float64, (3, n), "pos", dev),
        _dptr(vel, torch.float64, (3, n), "vel", dev), _dptr(mass, torch.float64, (n,), "mass", dev),
        _dptr(r_in, torch.float64, (n,), "r_in", dev), _dptr(r_out, torch.float64, (n,), "r_out", dev),
        _dptr(r_search, torch.float64, (n,), "r_search", dev), n_pair,
        _dptr(pairs, torch.int32, (2, n_pair), "pairs", dev) if n_pair else None, int(order),
        float(c_d), ctypes.byref(st_), ctypes.c_void_p(frame.data_ptr()) if n_pair else None,
        ctypes.c_void_p(out["pair_of"].data_ptr()))
    _check(st, ctx)
    return out


def petar_tidal_fit(ctx: Context, art: dict, pairs: torch.Tensor, acc_set: torch.Tensor,
                    pot_set: Optional[torch.Tensor], pos: Optional[torch.Tensor] = None):
    """Post-fit of the long-range force on an artificial set: returns
    (tensor (4 + K, n_pair), acc (3, N) or None, pot (N,) or None); acc and
    pot are computed when pos (3, N) is given. See petar.h."""
    order = art["order"]
    dev = ctx.device
    d = "cuda:%d" % dev
    n_out = art["mass"].shape[0]
    n_pair = art["frame"].shape[1]
    K = 6 if order == 2 else 16
    tensor = torch.empty((4 + K, n_pair), dtype=torch.float64, device=d)
    acc = pot = None
    n = 0
    if pos is not None:
        n = pos.shape[1]
        acc = torch.empty((3, n), dtype=torch.float64, device=d)
        if pot_set is not None:
            pot = torch.empty(n, dtype=torch.float64, device=d)
    st = _lib.petar_tidal_fit(
        ctx.handle, int(order), n, _dptr(pos, torch.float64, (3, n), "pos", dev), n_pair,
        _dptr(pairs, torch.int32, (2, n_pair), "pairs", dev) if n_pair else None,
        _dptr(art["frame"], torch.float64, (4, n_pair), "frame", dev) if n_pair else None, n_out,
        _dptr(art["src"], torch.int32, (n_out,), "src", dev),
        _dptr(acc_set, torch.float64, (3, n_out), "acc_set", dev),
        _dptr(pot_set, torch.float64, (n_out,), "pot_set", dev),
        ctypes.c_void_p(tensor.data_ptr()) if n_pair else None,
        ctypes.c_void_p(acc.data_ptr()) if acc is not None else None,
        ctypes.c_void_p(pot.data_ptr()) if pot is not None else None)
    _check(st, ctx)
    return tensor, acc, pot


def petar_tidal_eval(ctx: Context, order: int, tensor: torch.Tensor, frame: torch.Tensor,
                     pair_of: torch.Tensor, pos: torch.Tensor, acc: Optional[torch.Tensor] = None,
                     pot: Optional[torch.Tensor] = None):
    """Fitted field (3, n_pt) and potential (n_pt,) at pos (3, n_pt); points
    with pair_of < 0 keep the values already in acc / pot (zeros when those
    are not given)."""
    dev = ctx.device
    d = "cuda:%d" % dev
    n_pt = pos.shape[1]
    n_pair = frame.shape[1]
    K = 6 if order == 2 else 16
    if acc is None:
        acc = torch.zeros((3, n_pt), dtype=torch.float64, device=d)
    if pot is None:
        pot = torch.zeros(n_pt, dtype=torch.float64, device=d)
    if n_pt == 0:
        return acc, pot
    st = _lib.petar_tidal_eval(
        ctx.handle, int(order), n_pair,
        _dptr(tensor, torch.float64, (4 + K, n_pair), "tensor", dev) if n_pair else None,
        _dptr(frame, torch.float64, (4, n_pair), "frame", dev) if n_pair else None, n_pt,
        _dptr(pair_of, torch.int32, (n_pt,), "pair_of", dev),
        _dptr(pos, torch.float64, (3, n_pt), "pos", dev),
        _dptr(acc, torch.float64, (3, n_pt), "acc", dev),
        _dptr(pot, torch.float64, (n_pt,), "pot", dev))
    _check(st, ctx)
    return acc, pot


def petar_copy_counts(ctx: Context) -> torch.Tensor:
    """Per-particle interaction counts (4, N) int32 of the last force call."""
    n = petar_get_stats(ctx)["n"]
    out = torch.empty((4, n), dtype=torch.int32, device="cuda:%d" % ctx.device)
    _check(_lib.petar_copy_counts(ctx.handle, ctypes.c_void_p(out.data_ptr())), ctx)
    return out


def petar_get_stats(ctx: Context) -> dict:
    s = _capi.petar_stats()
    _check(_lib.petar_get_stats(ctx.handle, ctypes.byref(s)), ctx)
    return s.as_dict()


def petar_autotune(ctx: Context, pos: torch.Tensor, mass: torch.Tensor, theta: float,
                   r_in: torch.Tensor, r_out: torch.Tensor, r_search: torch.Tensor,
                   cache_path: Optional[str] = None) -> dict:
    """Fastest (leaf_size, group_size, i_per_lane) for these particles; see petar.h."""
    n = mass.shape[0]
    dev = ctx.device
    out = _capi.petar_tuned()
    st = _lib.petar_autotune(ctx.handle, _dptr(pos, torch.float64, (3, n), "pos", dev),
                             _dptr(mass, torch.float64, (n,), "mass", dev), n, float(theta),
                             _dptr(r_in, torch.float64, (n,), "r_in", dev),
                             _dptr(r_out, torch.float64, (n,), "r_out", dev),
                             _dptr(r_search, torch.float64, (n,), "r_search", dev),
                             cache_path.encode() if cache_path else None, ctypes.byref(out))
    _check(st, ctx)
    return {name: getattr(out, name) for name, _ in out._fields_}


def petar_autotune_batch(ctx: Context, sys_offsets, pos: torch.Tensor, mass: torch.Tensor,
                         theta: float, r_in: torch.Tensor, r_out: torch.Tensor,
                         r_search: torch.Tensor, cache_path: Optional[str] = None) -> dict:
    """Fastest (leaf_size, group_size, i_per_lane) for the batched step of
    these systems (system s owns particles sys_offsets[s]:sys_offsets[s+1]);
    see petar.h."""
    offs = [int(v) for v in sys_offsets]
    n = mass.shape[0] if mass.dim() == 1 else -1
    dev = ctx.device
    arr = (ctypes.c_int64 * len(offs))(*offs)
    out = _capi.petar_tuned()
    st = _lib.petar_autotune_batch(ctx.handle, len(offs) - 1, arr,
                                   _dptr(pos, torch.float64, (3, n), "pos", dev),
                                   _dptr(mass, torch.float64, (n,), "mass", dev), float(theta),
                                   _dptr(r_in, torch.float64, (n,), "r_in", dev),
                                   _dptr(r_out, torch.float64, (n,), "r_out", dev),
                                   _dptr(r_search, torch.float64, (n,), "r_search", dev),
                                   cache_path.encode() if cache_path else None,
                                   ctypes.byref(out))
    _check(st, ctx)
    return {name: getattr(out, name) for name, _ in out._fields_}


# Parameters petar_autotune chose on an MI355X for the particle sets of the
# benchmark (JSON lines, written by the autotuner itself).
TUNED_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.jsonl")


def petar_autotune_lookup(ctx: Context, n: int, theta: float,
                          cache_path: Optional[str] = None) -> Optional[dict]:
    """The stored autotuner choice for (N, theta, the context's precision),
    or None when the cache holds none; launches nothing. See petar.h."""
    out = _capi.petar_tuned()
    path = TUNED_CACHE if cache_path is None else cache_path
    st = _lib.petar_autotune_lookup(ctx.handle, int(n), float(theta), path.encode(),
                                    ctypes.byref(out))
    if st == PETAR_E_STATE:
        return None
    _check(st, ctx)
    return {name: getattr(out, name) for name, _ in out._fields_}


def petar_autotune_lookup_batch(ctx: Context, n: int, n_sys: int, theta: float,
                                cache_path: Optional[str] = None) -> Optional[dict]:
    """The stored autotuner choice for a batch of n_sys systems holding n
    particles in total, or None; launches nothing. See petar.h."""
    out = _capi.petar_tuned()
    path = TUNED_CACHE if cache_path is None else cache_path
    st = _lib.petar_autotune_lookup_batch(ctx.handle, int(n), int(n_sys), float(theta),
                                          path.encode(), ctypes.byref(out))
    if st == PETAR_E_STATE:
        return None
    _check(st, ctx)
    return {name: getattr(out, name) for name, _ in out._fields_}


def launch_config(ctx: Context, n: int, theta: float, leaf_default: int = 8,
                  group_default: int = 64, ipl_default: int = 2, n_sys: int = 1) -> dict:
    """Leaf size, group size and targets per lane for a force at (N, theta)
    on one system or a batch of n_sys: the autotuner's stored choice when
    the package cache holds one (source "autotune"), else the defaults
    (source "default")."""
    t = petar_autotune_lookup(ctx, n, theta) if n_sys == 1 else \
        petar_autotune_lookup_batch(ctx, n, n_sys, theta)
    if t is None:
        return {"leaf_size": leaf_default, "group_size": group_default,
                "i_per_lane": ipl_default, "source": "default"}
    return {"leaf_size": t["leaf_size"], "group_size": t["group_size"],
            "i_per_lane": t["i_per_lane"], "source": "autotune", "tuned_ms": t["ms"]}


def force_long_with_retry(ctx: Context, group_size: int, r_in, r_out, r_search,
                          nb_capacity: int = 0):
    """petar_force_long with neighbour lists, retrying once with the required
    capacity if the first guess was too small."""
    try:
        return petar_force_long(ctx, group_size, r_in, r_out, r_search, nb_capacity=nb_capacity)
    except PetarError as e:
        if e.status != PETAR_E_NB_OVERFLOW:
            raise
        return petar_force_long(ctx, group_size, r_in, r_out, r_search, nb_capacity=e.required)
