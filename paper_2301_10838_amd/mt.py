"""Python binding of libmt.so (ctypes): argument marshalling only.

Every step of the merge-tree path runs in the library's HIP kernels; this
module allocates torch tensors for outputs and workspaces, passes raw device
pointers and the current HIP stream, and turns status codes into exceptions.
It never falls back to another implementation: without the built library, or
without a GPU, every call raises.

Functions keep the C names: ``mt_build``, ``mt_persistence_pairs``,
``mt_build_pairs``, ``mt_batch_build``, ``mt_pairs_backward``; ``MergeTreePairs`` wraps the batch
build and the backward scatter as a ``torch.autograd.Function``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmt.so")

MT_OK = 0
STATUS_NAMES = {
    0: "MT_OK", -1: "MT_ERR_INVALID_ARG", -2: "MT_ERR_TOO_LARGE", -3: "MT_ERR_NAN", -4: "MT_ERR_CAPACITY",
    -5: "MT_ERR_LIVELOCK", -6: "MT_ERR_WORKSPACE", -7: "MT_ERR_HIP", -8: "MT_ERR_INTERNAL",
}
EXPORTS = [
    "mt_status_string", "mt_workspace_bytes", "mt_batch_workspace_bytes", "mt_build", "mt_persistence_pairs",
    "mt_batch_build", "mt_sync_status", "mt_build_stats", "mt_pairs_backward", "mt_release_caches",
    "mt_profile_begin",
    "mt_profile_end", "mt_profile_count", "mt_profile_get", "mt_tile_shape_count", "mt_tile_shape_info",
    "mt_set_tile_shape", "mt_get_tile_shape", "mt_autotune_workspace_bytes", "mt_autotune", "mt_build_tree",
    "mt_batch_build_tree", "mt_build_pairs", "mt_vertex_ranks", "mt_rank_workspace_bytes",
    "mt_set_max_steps", "mt_get_max_steps", "mt_set_table_probes", "mt_get_table_probes", "mt_workspace_reset",
    "mt_set_counting", "mt_get_counting", "mt_read_counters", "mt_build_pairs64",
    "mt_build_pairs_noalloc", "mt_noalloc_scratch_bytes", "mt_set_schedule", "mt_get_schedule",
    "mt_autotune_schedule",
]

COUNTER_NAMES = [
    "gm_facts", "gm_steps", "gm_descents", "gm_cas", "gm_cas_fail", "gm_remerge", "gm_max_steps",
    "lds_merges", "lds_steps", "lds_cas", "lds_cas_fail", "lds_max_steps",
    "table_inserts", "table_probes", "table_direct", "output_chase_steps", "gm_compress", "min_chase_steps",
    "cyc_load", "cyc_descent", "cyc_number", "cyc_basin", "cyc_clear", "cyc_insert", "cyc_compact", "cyc_merge",
    "cyc_repair", "cyc_label", "table_overflow_tiles",
    "output_chase_rounds",
]

# tree kinds (include/mt.h)
MT_TREE_MERGE, MT_TREE_SPLIT = 0, 1
_KINDS = {"merge": MT_TREE_MERGE, "split": MT_TREE_SPLIT}


def _kind(kind) -> int:
    if isinstance(kind, str):
        if kind not in _KINDS:
            raise ValueError(f"tree kind must be one of {sorted(_KINDS)}")
        return _KINDS[kind]
    return int(kind)


class MTError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}")
        self.status = status


_lib = None


def load_library():
    """Load libmt.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    lib.mt_status_string.argtypes = [ctypes.c_int]
    lib.mt_status_string.restype = ctypes.c_char_p
    lib.mt_workspace_bytes.argtypes = [I64, I64, I64]
    lib.mt_workspace_bytes.restype = SZ
    lib.mt_batch_workspace_bytes.argtypes = [P, I32]
    lib.mt_batch_workspace_bytes.restype = SZ
    lib.mt_build.argtypes = [P, I64, I64, I64, P, P, SZ, P]
    lib.mt_build.restype = ctypes.c_int
    lib.mt_build_tree.argtypes = [P, I64, I64, I64, ctypes.c_int, P, P, SZ, P]
    lib.mt_build_tree.restype = ctypes.c_int
    lib.mt_persistence_pairs.argtypes = [P, P, I64, I64, I64, P, P, P, P, I64, P, P, P, SZ, P]
    lib.mt_persistence_pairs.restype = ctypes.c_int
    lib.mt_build_pairs.argtypes = [P, I64, I64, I64, ctypes.c_int, P, P, P, P, P, I64, P, P, P, SZ, P]
    lib.mt_build_pairs.restype = ctypes.c_int
    lib.mt_build_pairs64.argtypes = [P, I64, I64, I64, ctypes.c_int, P, P, P, P, P, I64, P, P, P, SZ, P]
    lib.mt_build_pairs64.restype = ctypes.c_int
    lib.mt_build_pairs_noalloc.argtypes = [P, I64, I64, I64, ctypes.c_int, P, P, P, P, P, I64, P, P, P]
    lib.mt_build_pairs_noalloc.restype = ctypes.c_int
    lib.mt_noalloc_scratch_bytes.argtypes = []
    lib.mt_noalloc_scratch_bytes.restype = SZ
    lib.mt_vertex_ranks.argtypes = [P, I64, I64, I64, ctypes.c_int, P, P, SZ, P]
    lib.mt_vertex_ranks.restype = ctypes.c_int
    lib.mt_rank_workspace_bytes.argtypes = [I64, I64, I64]
    lib.mt_rank_workspace_bytes.restype = SZ
    lib.mt_batch_build.argtypes = [P, P, I32, P, P, P, P, P, I64, P, P, SZ, P]
    lib.mt_batch_build.restype = ctypes.c_int
    lib.mt_batch_build_tree.argtypes = [P, P, I32, ctypes.c_int, P, P, P, P, P, I64, P, P, SZ, P]
    lib.mt_batch_build_tree.restype = ctypes.c_int
    lib.mt_sync_status.argtypes = [P, P, P, P]
    lib.mt_sync_status.restype = ctypes.c_int
    lib.mt_build_stats.argtypes = [P, P, P, P]
    lib.mt_build_stats.restype = ctypes.c_int
    lib.mt_pairs_backward.argtypes = [P, I32, P, I64, P, P, P, P, P, ctypes.c_int, P]
    lib.mt_pairs_backward.restype = ctypes.c_int
    lib.mt_release_caches.argtypes = []
    lib.mt_release_caches.restype = None
    lib.mt_profile_begin.argtypes = []
    lib.mt_profile_begin.restype = ctypes.c_int
    lib.mt_profile_end.argtypes = []
    lib.mt_profile_end.restype = ctypes.c_int
    lib.mt_profile_count.argtypes = []
    lib.mt_profile_count.restype = ctypes.c_int
    lib.mt_profile_get.argtypes = [ctypes.c_int, ctypes.c_char_p, SZ, P, P]
    lib.mt_profile_get.restype = ctypes.c_int
    lib.mt_tile_shape_count.argtypes = []
    lib.mt_tile_shape_count.restype = ctypes.c_int
    lib.mt_tile_shape_info.argtypes = [ctypes.c_int, P, P, P, P, P]
    lib.mt_tile_shape_info.restype = ctypes.c_int
    lib.mt_set_tile_shape.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.mt_set_tile_shape.restype = ctypes.c_int
    lib.mt_get_tile_shape.argtypes = [ctypes.c_int]
    lib.mt_get_tile_shape.restype = ctypes.c_int
    lib.mt_autotune_workspace_bytes.argtypes = [P, I32]
    lib.mt_autotune_workspace_bytes.restype = SZ
    lib.mt_autotune.argtypes = [P, P, I32, P, P, P, SZ, ctypes.c_int, P, P]
    lib.mt_autotune.restype = ctypes.c_int
    lib.mt_autotune_schedule.argtypes = [P, P, I32, P, P, P, SZ, ctypes.c_int, P, P]
    lib.mt_autotune_schedule.restype = ctypes.c_int
    lib.mt_set_schedule.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.mt_set_schedule.restype = ctypes.c_int
    lib.mt_get_schedule.argtypes = [P, P]
    lib.mt_get_schedule.restype = ctypes.c_int
    lib.mt_set_max_steps.argtypes = [I64]
    lib.mt_set_max_steps.restype = ctypes.c_int
    lib.mt_get_max_steps.argtypes = []
    lib.mt_get_max_steps.restype = I64
    lib.mt_set_table_probes.argtypes = [ctypes.c_int]
    lib.mt_set_table_probes.restype = ctypes.c_int
    lib.mt_get_table_probes.argtypes = []
    lib.mt_get_table_probes.restype = ctypes.c_int
    lib.mt_workspace_reset.argtypes = [P, SZ, P]
    lib.mt_workspace_reset.restype = ctypes.c_int
    lib.mt_set_counting.argtypes = [ctypes.c_int]
    lib.mt_set_counting.restype = ctypes.c_int
    lib.mt_get_counting.argtypes = []
    lib.mt_get_counting.restype = ctypes.c_int
    lib.mt_read_counters.argtypes = [P, P, P, ctypes.c_int]
    lib.mt_read_counters.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != MT_OK:
        raise MTError(rc, what)


def grid_dims(shape: Sequence[int]):
    """(nx, ny, nz) of a C-order [nz][ny][nx] (or lower-rank) shape."""
    shape = tuple(int(s) for s in shape)
    if len(shape) == 1:
        return shape[0], 1, 1
    if len(shape) == 2:
        return shape[1], shape[0], 1
    if len(shape) == 3:
        return shape[2], shape[1], shape[0]
    raise ValueError("fields must be 1-D, 2-D or 3-D")


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream_ptr(device: torch.device) -> int:
    """The current stream of `device` as a raw handle.  (The raw accessor
    builds no Stream object: a few microseconds less per call, which the
    autograd backward pays once per step.)"""
    if _raw_stream is not None:
        idx = device.index if device.index is not None else torch.cuda.current_device()
        return int(_raw_stream(idx))
    return torch.cuda.current_stream(device).cuda_stream


def _field(field: torch.Tensor) -> torch.Tensor:
    if not isinstance(field, torch.Tensor) or field.device.type != "cuda":
        raise TypeError("field must be a torch tensor on a HIP device")
    if field.dtype != torch.float32:
        raise TypeError("field must be float32")
    return field.contiguous()


def workspace_bytes(shape) -> int:
    nx, ny, nz = grid_dims(shape)
    return int(load_library().mt_workspace_bytes(nx, ny, nz))


def alloc_workspace(nbytes: int, device) -> torch.Tensor:
    """Device workspace of at least `nbytes` bytes with its status head
    cleared (mt_workspace_reset), so that no leftover byte reads as an error."""
    ws = torch.empty(max(int(nbytes), 4096), dtype=torch.uint8, device=device)
    workspace_reset(ws)
    return ws


def workspace_reset(workspace: torch.Tensor):
    _check(load_library().mt_workspace_reset(workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                             _stream_ptr(workspace.device)), "mt_workspace_reset")


def mt_build(field: torch.Tensor, triplets: torch.Tensor | None = None,
             workspace: torch.Tensor | None = None, kind="merge", check: bool = True) -> torch.Tensor:
    """Triplets T[u] = (s, v) of the merge tree (kind "merge") or split tree
    (kind "split": the merge tree of -f) of `field` (int32 [N, 2], uint32 bit
    patterns).

    The C call is asynchronous and latches device-side errors (a NaN in the
    field, a loop that hit the step cap) in the workspace.  With check=True
    (the default) this waits for the build and raises MTError on such a
    status; with check=False it returns at once and the status is read later
    (sync_status, or mt_persistence_pairs on the same workspace)."""
    lib = load_library()
    f = _field(field)
    nx, ny, nz = grid_dims(f.shape)
    N = nx * ny * nz
    if triplets is None:
        triplets = torch.empty((N, 2), dtype=torch.int32, device=f.device)
    if workspace is None:
        workspace = alloc_workspace(lib.mt_workspace_bytes(nx, ny, nz), f.device)
    rc = lib.mt_build_tree(f.data_ptr(), nx, ny, nz, _kind(kind), triplets.data_ptr(), workspace.data_ptr(),
                           workspace.numel(), _stream_ptr(f.device))
    _check(rc, "mt_build_tree")
    if check:
        sync_status(workspace)
    return triplets


def mt_persistence_pairs(field: torch.Tensor, triplets: torch.Tensor, capacity: int | None = None,
                         workspace: torch.Tensor | None = None):
    """(birth, death, birth_val, death_val, n_roots); ids int32, ascending birth id."""
    lib = load_library()
    f = _field(field)
    nx, ny, nz = grid_dims(f.shape)
    N = nx * ny * nz
    if capacity is None:
        capacity = N // 2 + 1
    dev = f.device
    birth = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    death = torch.empty_like(birth)
    bval = torch.empty(max(capacity, 1), dtype=torch.float32, device=dev)
    dval = torch.empty_like(bval)
    if workspace is None:
        workspace = alloc_workspace(lib.mt_workspace_bytes(nx, ny, nz), dev)
    n_pairs = ctypes.c_int64(0)
    n_roots = ctypes.c_int64(0)
    rc = lib.mt_persistence_pairs(f.data_ptr(), triplets.data_ptr(), nx, ny, nz, birth.data_ptr(),
                                  death.data_ptr(), bval.data_ptr(), dval.data_ptr(), capacity,
                                  ctypes.byref(n_pairs), ctypes.byref(n_roots), workspace.data_ptr(),
                                  workspace.numel(), _stream_ptr(dev))
    _check(rc, "mt_persistence_pairs")
    P = n_pairs.value
    return birth[:P], death[:P], bval[:P], dval[:P], n_roots.value


def mt_build_pairs(field: torch.Tensor, kind="merge", capacity: int | None = None,
                   triplets: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """Tree and pairs in one call: (triplets, birth, death, birth_val,
    death_val, n_roots), the results of mt_build then mt_persistence_pairs."""
    lib = load_library()
    f = _field(field)
    nx, ny, nz = grid_dims(f.shape)
    N = nx * ny * nz
    if capacity is None:
        capacity = N // 2 + 1
    dev = f.device
    if triplets is None:
        triplets = torch.empty((N, 2), dtype=torch.int32, device=dev)
    birth = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    death = torch.empty_like(birth)
    bval = torch.empty(max(capacity, 1), dtype=torch.float32, device=dev)
    dval = torch.empty_like(bval)
    if workspace is None:
        workspace = alloc_workspace(lib.mt_workspace_bytes(nx, ny, nz), dev)
    n_pairs = ctypes.c_int64(0)
    n_roots = ctypes.c_int64(0)
    rc = lib.mt_build_pairs(f.data_ptr(), nx, ny, nz, _kind(kind), triplets.data_ptr(), birth.data_ptr(),
                            death.data_ptr(), bval.data_ptr(), dval.data_ptr(), capacity, ctypes.byref(n_pairs),
                            ctypes.byref(n_roots), workspace.data_ptr(), workspace.numel(), _stream_ptr(dev))
    _check(rc, "mt_build_pairs")
    P = n_pairs.value
    return triplets, birth[:P], death[:P], bval[:P], dval[:P], n_roots.value


def mt_build_pairs64(field: torch.Tensor, kind="merge", capacity: int | None = None,
                     triplets: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """mt_build_pairs with 64-bit ids: (triplets int64 [N, 2], birth, death
    (int64), birth_val, death_val, n_roots)."""
    lib = load_library()
    f = _field(field)
    nx, ny, nz = grid_dims(f.shape)
    N = nx * ny * nz
    if capacity is None:
        capacity = N // 2 + 1
    dev = f.device
    if triplets is None:
        triplets = torch.empty((N, 2), dtype=torch.int64, device=dev)
    birth = torch.empty(max(capacity, 1), dtype=torch.int64, device=dev)
    death = torch.empty_like(birth)
    bval = torch.empty(max(capacity, 1), dtype=torch.float32, device=dev)
    dval = torch.empty_like(bval)
    if workspace is None:
        workspace = alloc_workspace(lib.mt_workspace_bytes(nx, ny, nz), dev)
    n_pairs = ctypes.c_int64(0)
    n_roots = ctypes.c_int64(0)
    rc = lib.mt_build_pairs64(f.data_ptr(), nx, ny, nz, _kind(kind), triplets.data_ptr(), birth.data_ptr(),
                              death.data_ptr(), bval.data_ptr(), dval.data_ptr(), capacity, ctypes.byref(n_pairs),
                              ctypes.byref(n_roots), workspace.data_ptr(), workspace.numel(), _stream_ptr(dev))
    _check(rc, "mt_build_pairs64")
    P = n_pairs.value
    return triplets, birth[:P], death[:P], bval[:P], dval[:P], n_roots.value


def mt_vertex_ranks(field: torch.Tensor, kind="merge", ranks: torch.Tensor | None = None,
                    workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Position of every vertex in the (value, id) order (of -f for kind
    "split"): int32 [N] holding uint32 ranks.  Asynchronous; a NaN is reported
    by mt_sync_status on the workspace."""
    lib = load_library()
    f = _field(field)
    nx, ny, nz = grid_dims(f.shape)
    N = nx * ny * nz
    if ranks is None:
        ranks = torch.empty(N, dtype=torch.int32, device=f.device)
    if workspace is None:
        workspace = alloc_workspace(lib.mt_rank_workspace_bytes(nx, ny, nz), f.device)
    rc = lib.mt_vertex_ranks(f.data_ptr(), nx, ny, nz, _kind(kind), ranks.data_ptr(), workspace.data_ptr(),
                             workspace.numel(), _stream_ptr(f.device))
    _check(rc, "mt_vertex_ranks")
    return ranks


def sync_status(workspace: torch.Tensor):
    """Status latched in a workspace by the work enqueued before: (n_pairs, n_roots); raises on error."""
    lib = load_library()
    n_pairs, n_roots = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = lib.mt_sync_status(workspace.data_ptr(), _stream_ptr(workspace.device), ctypes.byref(n_pairs),
                            ctypes.byref(n_roots))
    _check(rc, "mt_sync_status")
    return n_pairs.value, n_roots.value


class BatchPlan:
    """Buffers of one batch configuration (reused across calls, so the library's
    cached graph for these pointers is replayed)."""

    def __init__(self, shapes: Sequence[Sequence[int]], device, pair_capacity: int | None = None, kind="merge"):
        lib = load_library()
        self.kind = _kind(kind)
        self.shapes = [tuple(int(s) for s in shp) for shp in shapes]
        self.dims = [grid_dims(s) for s in self.shapes]
        self.sizes = [nx * ny * nz for nx, ny, nz in self.dims]
        self.n_total = sum(self.sizes)
        self.device = torch.device(device)
        self._dims_c = (ctypes.c_int64 * (3 * len(self.dims)))(*[v for d in self.dims for v in d])
        ws = lib.mt_batch_workspace_bytes(self._dims_c, len(self.dims))
        if ws == 0:
            raise MTError(-1, "mt_batch_workspace_bytes")
        if pair_capacity is None:
            pair_capacity = sum(n // 2 + 1 for n in self.sizes)
        self.pair_capacity = int(pair_capacity)
        dev = self.device
        self.fields = torch.empty(self.n_total, dtype=torch.float32, device=dev)
        self.triplets = torch.empty((self.n_total, 2), dtype=torch.int32, device=dev)
        cap = max(self.pair_capacity, 1)
        self.birth = torch.empty(cap, dtype=torch.int32, device=dev)
        self.death = torch.empty(cap, dtype=torch.int32, device=dev)
        self.bval = torch.empty(cap, dtype=torch.float32, device=dev)
        self.dval = torch.empty(cap, dtype=torch.float32, device=dev)
        self.pair_offsets = torch.empty(len(self.dims) + 1, dtype=torch.int64, device=dev)
        self.workspace = alloc_workspace(ws, dev)
        starts = [0]
        for n in self.sizes:
            starts.append(starts[-1] + n)
        self.vertex_offsets = starts

    def load(self, fields: Sequence[torch.Tensor]):
        for i, f in enumerate(fields):
            a, b = self.vertex_offsets[i], self.vertex_offsets[i + 1]
            self.fields[a:b].copy_(f.reshape(-1))

    def launch(self):
        rc = load_library().mt_batch_build_tree(
            self.fields.data_ptr(), self._dims_c, len(self.dims), self.kind, self.triplets.data_ptr(),
            self.birth.data_ptr(),
            self.death.data_ptr(), self.bval.data_ptr(), self.dval.data_ptr(), self.pair_capacity,
            self.pair_offsets.data_ptr(), self.workspace.data_ptr(), self.workspace.numel(),
            _stream_ptr(self.device))
        _check(rc, "mt_batch_build_tree")

    def sync_status(self):
        n_pairs = ctypes.c_int64(0)
        rc = load_library().mt_sync_status(self.workspace.data_ptr(), _stream_ptr(self.device),
                                           ctypes.byref(n_pairs), None)
        _check(rc, "mt_batch_build (device status)")
        return n_pairs.value

    def backward(self, grad_birth: torch.Tensor, grad_death: torch.Tensor, grad_field: torch.Tensor | None = None,
                 accumulate: bool = False) -> torch.Tensor:
        if grad_field is None:
            grad_field = torch.empty(self.n_total, dtype=torch.float32, device=self.device)
        return mt_pairs_backward(self._dims_c, len(self.dims), self.pair_offsets, self.pair_capacity, self.birth,
                                 self.death, grad_birth, grad_death, grad_field, accumulate)


def mt_batch_build(fields: Sequence[torch.Tensor], plan: BatchPlan | None = None, sync: bool = True,
                   kind="merge"):
    """Merge (or split) trees + pairs of many fields in one graph launch; returns the plan holding the outputs."""
    if plan is None:
        plan = BatchPlan([f.shape for f in fields], fields[0].device, kind=kind)
    plan.load(fields)
    plan.launch()
    if sync:
        plan.sync_status()
    return plan


def mt_pairs_backward(dims_c, n_fields: int, pair_offsets: torch.Tensor, pair_capacity: int, birth: torch.Tensor,
                      death: torch.Tensor, grad_birth: torch.Tensor, grad_death: torch.Tensor,
                      grad_field: torch.Tensor, accumulate: bool = False) -> torch.Tensor:
    """grad_field[birth] += grad_birth; grad_field[death] += grad_death (concatenated batch ids)."""
    if not isinstance(dims_c, ctypes.Array):
        flat = [int(v) for d in dims_c for v in d]
        dims_c = (ctypes.c_int64 * len(flat))(*flat)
    gb = grad_birth.contiguous()
    gd = grad_death.contiguous()
    if gb.dtype != torch.float32 or gd.dtype != torch.float32 or grad_field.dtype != torch.float32:
        raise TypeError("gradients must be float32")
    n = min(pair_capacity, gb.numel(), gd.numel(), birth.numel(), death.numel())
    rc = load_library().mt_pairs_backward(dims_c, n_fields, pair_offsets.data_ptr(), n, birth.data_ptr(),
                                          death.data_ptr(), gb.data_ptr(), gd.data_ptr(), grad_field.data_ptr(),
                                          1 if accumulate else 0, _stream_ptr(grad_field.device))
    _check(rc, "mt_pairs_backward")
    return grad_field


class MergeTreePairs(torch.autograd.Function):
    """Persistence pairs of a batch of fields as differentiable values.

    forward(flat_fields, plan) -> (birth_val, death_val) over all pairs of all
    fields (concatenated; ``plan.pair_offsets`` splits them per field).  The
    pairing is piecewise constant in the field, so the derivative of a birth
    value is 1 at its birth vertex and that of a death value 1 at its death
    vertex; backward scatters the upstream gradients there with the library's
    adjoint kernel.
    """

    @staticmethod
    def forward(ctx, flat_fields: torch.Tensor, plan: BatchPlan):
        plan.fields.copy_(flat_fields.detach().reshape(-1))
        plan.launch()
        P = plan.sync_status()
        if P > plan.pair_capacity:
            raise MTError(-4, "MergeTreePairs")
        ctx.plan = plan
        ctx.P = P
        # the plan's buffers are reused by the next forward: keep this pairing
        # (private copies, neither inputs nor outputs of the function, so they
        # are kept on ctx directly: save_for_backward's checks cost host time)
        ctx.pairing = (plan.birth[:P].clone(), plan.death[:P].clone(), plan.pair_offsets.clone())
        return plan.bval[:P].clone(), plan.dval[:P].clone()

    @staticmethod
    def backward(ctx, g_birth, g_death):
        # (one C call with the plan's prepared arguments: this runs once per
        # optimisation step, so its host time is part of the step)
        plan, P = ctx.plan, ctx.P
        dev = plan.device
        if g_birth is None:
            g_birth = torch.zeros(P, dtype=torch.float32, device=dev)
        if g_death is None:
            g_death = torch.zeros(P, dtype=torch.float32, device=dev)
        gb = g_birth.contiguous().float()
        gd = g_death.contiguous().float()
        birth, death, offsets = ctx.pairing
        grad = torch.empty(plan.n_total, dtype=torch.float32, device=dev)
        _check(load_library().mt_pairs_backward(plan._dims_c, len(plan.dims), offsets.data_ptr(), P,
                                                birth.data_ptr(), death.data_ptr(), gb.data_ptr(), gd.data_ptr(),
                                                grad.data_ptr(), 0, _stream_ptr(dev)),
               "mt_pairs_backward")
        return grad, None


def profile_begin():
    _check(load_library().mt_profile_begin(), "mt_profile_begin")


def profile_end():
    """Stop per-kernel timing; returns {kernel name: (total ms, launches)}."""
    lib = load_library()
    _check(lib.mt_profile_end(), "mt_profile_end")
    out = {}
    buf = ctypes.create_string_buffer(128)
    for i in range(lib.mt_profile_count()):
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        _check(lib.mt_profile_get(i, buf, 128, ctypes.byref(ms), ctypes.byref(n)), "mt_profile_get")
        out[buf.value.decode()] = (ms.value, n.value)
    return out


def build_stats(workspace: torch.Tensor):
    """(tile-local minima, cross-tile facts) of the last build on this
    workspace (synchronizes)."""
    n, q = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(load_library().mt_build_stats(workspace.data_ptr(), _stream_ptr(workspace.device), ctypes.byref(n),
                                         ctypes.byref(q)), "mt_build_stats")
    return n.value, q.value


def tile_shapes():
    """Compiled tile shapes: list of dicts (id, tx, ty, tz, threads, dims_class)."""
    lib = load_library()
    out = []
    for i in range(lib.mt_tile_shape_count()):
        v = [ctypes.c_int(0) for _ in range(5)]
        _check(lib.mt_tile_shape_info(i, *[ctypes.byref(x) for x in v]), "mt_tile_shape_info")
        out.append(dict(id=i, tx=v[0].value, ty=v[1].value, tz=v[2].value, threads=v[3].value,
                        dims_class=v[4].value))
    return out


def set_tile_shape(dims_class: int, shape_id: int):
    _check(load_library().mt_set_tile_shape(dims_class, shape_id), "mt_set_tile_shape")


def get_tile_shape(dims_class: int) -> int:
    return int(load_library().mt_get_tile_shape(dims_class))


def autotune(fields: Sequence[torch.Tensor], reps: int = 3):
    """Time every compiled tile shape on this batch (bit-identical output is
    checked by the library) and select the fastest per dims class.  Returns
    {dims_class: (shape id, best ms)} for the classes present."""
    lib = load_library()
    dev = fields[0].device
    dims = [grid_dims(f.shape) for f in fields]
    dims_c = (ctypes.c_int64 * (3 * len(dims)))(*[v for d in dims for v in d])
    flat = torch.cat([_field(f).reshape(-1) for f in fields])
    n = flat.numel()
    t1 = torch.empty((n, 2), dtype=torch.int32, device=dev)
    t2 = torch.empty_like(t1)
    ws = alloc_workspace(lib.mt_autotune_workspace_bytes(dims_c, len(dims)), dev)
    best = (ctypes.c_double * 3)()
    _check(lib.mt_autotune(flat.data_ptr(), dims_c, len(dims), t1.data_ptr(), t2.data_ptr(), ws.data_ptr(),
                           ws.numel(), reps, _stream_ptr(dev), best), "mt_autotune")
    return {c: (get_tile_shape(c), best[c]) for c in range(3) if best[c] >= 0}


def autotune_schedule(fields: Sequence[torch.Tensor], reps: int = 3):
    """Time the schedule candidates (XCD-aware tile order on/off, merge
    workgroups per XCD) on this batch with the current tile shapes (the
    library checks bit-identical output) and select the fastest.  Returns
    (xcd_remap, merge_groups, best ms)."""
    lib = load_library()
    dev = fields[0].device
    dims = [grid_dims(f.shape) for f in fields]
    dims_c = (ctypes.c_int64 * (3 * len(dims)))(*[v for d in dims for v in d])
    flat = torch.cat([_field(f).reshape(-1) for f in fields])
    n = flat.numel()
    t1 = torch.empty((n, 2), dtype=torch.int32, device=dev)
    t2 = torch.empty_like(t1)
    ws = alloc_workspace(lib.mt_batch_workspace_bytes(dims_c, len(dims)), dev)
    best = ctypes.c_double(-1.0)
    _check(lib.mt_autotune_schedule(flat.data_ptr(), dims_c, len(dims), t1.data_ptr(), t2.data_ptr(), ws.data_ptr(),
                                    ws.numel(), reps, _stream_ptr(dev), ctypes.byref(best)), "mt_autotune_schedule")
    r, g = get_schedule()
    return r, g, best.value


def set_schedule(xcd_remap: int = -1, merge_groups: int = 0):
    """XCD-aware tile order (1 on, 0 off, -1 default) and merge workgroups per XCD (0 default)."""
    _check(load_library().mt_set_schedule(int(xcd_remap), int(merge_groups)), "mt_set_schedule")


def get_schedule():
    r, g = ctypes.c_int(0), ctypes.c_int(0)
    _check(load_library().mt_get_schedule(ctypes.byref(r), ctypes.byref(g)), "mt_get_schedule")
    return r.value, g.value


def release_caches():
    load_library().mt_release_caches()


def set_max_steps(steps: int):
    """Step cap of every merge/descent/chase loop (0 restores the default)."""
    _check(load_library().mt_set_max_steps(int(steps)), "mt_set_max_steps")


def get_max_steps() -> int:
    return int(load_library().mt_get_max_steps())


def set_table_probes(probes: int):
    """Probes per edge in the LDS pair tables before the table-free path (-1 restores the default)."""
    _check(load_library().mt_set_table_probes(int(probes)), "mt_set_table_probes")


def get_table_probes() -> int:
    return int(load_library().mt_get_table_probes())


def set_counting(on):
    """Counting build: False/0 the timed kernels, True/1 event counters in the
    workspace, 2 phase clocks of the tile pass only."""
    _check(load_library().mt_set_counting(int(on)), "mt_set_counting")


def read_counters(workspace: torch.Tensor) -> dict:
    """Event counters of the last counting build on `workspace` (synchronizes)."""
    n = len(COUNTER_NAMES)
    buf = (ctypes.c_uint64 * n)()
    rc = load_library().mt_read_counters(workspace.data_ptr(), _stream_ptr(workspace.device), buf, n)
    if rc < 0:
        raise MTError(rc, "mt_read_counters")
    return {COUNTER_NAMES[i]: int(buf[i]) for i in range(n)}
