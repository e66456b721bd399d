"""mgrav: PKDGRAV3 gravity interaction lists on one AMD MI355X (gfx950).

Thin Python binding of the C ABI declared in ``include/mgrav.h``
(arXiv:1609.08621, Sec. 3.1-3.3).  This module only marshals arguments:
torch tensors provide device memory and the HIP stream, and every step of
the evaluation runs in the HIP kernels of ``libmgrav.so``.  There is no CPU
fallback: if the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MGRAV_LIBRARY may name another build of the same library (tuning variants).
LIB_PATH = os.environ.get("MGRAV_LIBRARY", os.path.join(_HERE, "libmgrav.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -m paper_1609_08621_amd.build` "
        "(the HIP extension is required, there is no fallback)")

# torch first: its HIP runtime is then the one the library binds to.  With
# the library loaded first, the process would hold two HIP runtimes (the
# system one and torch's), and device calls fail once torch has
# initialised its own.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_D = ctypes.c_double

OK, ERR_INVALID_ARG, ERR_BAD_TREE, ERR_BAD_LIST, ERR_DEVICE, ERR_NO_MEMORY, \
    ERR_TIMEOUT, ERR_STATE, ERR_NOT_TRAINED = range(9)
PART_PP, PART_PC, PART_EWALD, PART_ALL = 1, 2, 4, 7
EWALD_NONE, EWALD_EXACT, EWALD_SURROGATE, EWALD_SURROGATE_FALLBACK = 0, 1, 2, 3
LAUNCH_GRAPH, LAUNCH_DIRECT = 0, 1
QUEUE_AUTO, QUEUE_LPT, QUEUE_LOCAL = 0, 1, 2
MAX_BUCKET = 16
STATIC_WORKSPACE_BYTES = 64 << 20  # mgrav_bind_static's workspace per GPU


class Problem(ctypes.Structure):
    _fields_ = [
        ("n", _I64), ("pos", _P), ("mass", _P), ("eps", _D), ("theta", _D), ("box_L", _D),
        ("n_images", _I), ("n_cell", _I64), ("n_bucket", _I64), ("cell_first", _P),
        ("cell_count", _P), ("child", _P), ("com", _P), ("bbox", _P), ("mom", _P),
        ("bucket_cell", _P), ("pp_off", _P), ("pp_src", _P), ("pp_img", _P), ("pc_off", _P),
        ("pc_src", _P), ("pc_img", _P), ("n_pp", _I64), ("n_pc", _I64),
        ("pos_q", _P), ("q_origin", _D * 3), ("q_scale", _D), ("mass_uniform", _D),
        ("pp_sub", _P),
    ]


class Store(ctypes.Structure):
    """mgrav_store: device arrays q [n][3] uint32, vel [n][3] float32,
    aux [n] uint32 and the grid (x = origin + q * scale)."""
    _fields_ = [("q", _P), ("vel", _P), ("aux", _P), ("origin", _D * 3), ("scale", _D)]


class EwaldConfig(ctypes.Structure):
    _fields_ = [("mode", _I), ("alpha", _D), ("real_layers", _I), ("h2max", _I),
                ("order", _I), ("top_cells", _I), ("fallback_tol", _D),
                ("sample_stride", _I64)]


class Stats(ctypes.Structure):
    _fields_ = [("n_pp_interactions", _I64), ("n_pc_interactions", _I64),
                ("n_active_buckets", _I64), ("n_active_particles", _I64),
                ("ms_total", _D), ("ms_interact", _D), ("ms_ewald", _D),
                ("graph_replay", _I), ("interact_variant", _I), ("graph_error", _I),
                ("ewald_fallback", _I), ("ewald_samples", _I64), ("ewald_sample_err", _D),
                ("queue_local", _I), ("queue_pad", _I)]


class TreeDev(ctypes.Structure):
    _fields_ = [("perm", _P), ("pos", _P), ("mass", _P), ("cell_first", _P),
                ("cell_count", _P), ("child", _P), ("com", _P), ("bmax", _P), ("bbox", _P),
                ("mom", _P), ("bucket_cell", _P)]


class Walk(ctypes.Structure):
    _fields_ = [("n_cell", _I64), ("child", _P), ("com", _P), ("bmax", _P), ("bbox", _P),
                ("n_roots", _I), ("roots", ctypes.c_int32 * 2), ("theta", _D), ("eps", _D),
                ("L", _D), ("n_images", _I), ("n_sink", _I64), ("sink_cell", _P)]


class Fmm(ctypes.Structure):
    _fields_ = [("n", _I64), ("n_cell", _I64), ("n_bucket", _I64), ("child", _P), ("com", _P),
                ("mom", _P), ("cell_first", _P), ("cell_count", _P), ("bucket_cell", _P),
                ("pos", _P), ("mass", _P), ("mass_uniform", _D), ("eps", _D), ("box_L", _D),
                ("cc_off", _P), ("cc_src", _P), ("cc_img", _P), ("active", _P)]


class TrainConfig(ctypes.Structure):
    _fields_ = [("epochs", _I), ("batch", _I), ("lr", ctypes.c_float),
                ("lr_min", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("adam_eps", ctypes.c_float),
                ("loss_weight", ctypes.c_float * 4), ("psi0", _D)]


MLP_PARAMS = 34052


# int query(void *user): 0 = done, > 0 = not yet, < 0 = failed
WATCHDOG_QUERY = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p)


def _declare():
    L = _lib
    L.mgrav_version.restype = _I
    L.mgrav_status_string.restype = ctypes.c_char_p
    L.mgrav_status_string.argtypes = [_I]
    L.mgrav_last_error.restype = ctypes.c_char_p
    L.mgrav_last_error.argtypes = [_P]
    L.mgrav_create.restype = _I
    L.mgrav_create.argtypes = [_I, _P, ctypes.POINTER(_P)]
    L.mgrav_destroy.restype = None
    L.mgrav_destroy.argtypes = [_P]
    L.mgrav_tree_build_host.restype = _I
    L.mgrav_tree_build_host.argtypes = [_I64, _P, _P, _D, _I, _I64] + [_P] * 11
    L.mgrav_lists_count_host.restype = _I
    L.mgrav_lists_count_host.argtypes = [_I64, _P, _P, _P, _P, _P, _D, _D, _D, _I, _P, _P]
    L.mgrav_lists_fill_host.restype = _I
    L.mgrav_lists_fill_host.argtypes = [_I64, _P, _P, _P, _P, _P, _D, _D, _D, _I, _P, _P,
                                        _P, _P, _P, _P]
    L.mgrav_workspace_size.restype = _I
    L.mgrav_workspace_size.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_size_t)]
    L.mgrav_bind.restype = _I
    L.mgrav_bind.argtypes = [_P, ctypes.POINTER(Problem), _P, ctypes.c_size_t]
    L.mgrav_bind_static.restype = _I
    L.mgrav_bind_static.argtypes = [_P, ctypes.POINTER(Problem)]
    L.mgrav_set_ewald.restype = _I
    L.mgrav_set_ewald.argtypes = [_P, ctypes.POINTER(EwaldConfig)]
    L.mgrav_set_active.restype = _I
    L.mgrav_set_active.argtypes = [_P, _P]
    L.mgrav_compute.restype = _I
    L.mgrav_compute.argtypes = [_P, _P, _P]
    L.mgrav_compute_parts.restype = _I
    L.mgrav_compute_parts.argtypes = [_P, _I, _P, _P]
    L.mgrav_wait.restype = _I
    L.mgrav_wait.argtypes = [_P, _D, ctypes.POINTER(Stats)]
    L.mgrav_ewald_psi.restype = _I
    L.mgrav_ewald_psi.argtypes = [_P, _P, _I64, _D, _I, _I, _P]
    L.mgrav_mlp_workspace_size.restype = _I
    L.mgrav_mlp_workspace_size.argtypes = [_I64, ctypes.POINTER(ctypes.c_size_t)]
    L.mgrav_mlp_attach.restype = _I
    L.mgrav_mlp_attach.argtypes = [_P, _P, ctypes.c_size_t, _I64]
    L.mgrav_mlp_set_weights.restype = _I
    L.mgrav_mlp_set_weights.argtypes = [_P, _P, _I64, _D]
    L.mgrav_mlp_get_weights.restype = _I
    L.mgrav_mlp_get_weights.argtypes = [_P, _P, _I64]
    L.mgrav_mlp_forward.restype = _I
    L.mgrav_mlp_forward.argtypes = [_P, _P, _I64, _P]
    L.mgrav_mlp_backward.restype = _I
    L.mgrav_mlp_backward.argtypes = [_P, _P, _P, _I64, _P]
    L.mgrav_mlp_train.restype = _I
    L.mgrav_mlp_train.argtypes = [_P, _P, _P, _I64, ctypes.POINTER(TrainConfig), _P]
    L.mgrav_interact_variants.restype = _I
    L.mgrav_interact_variants.argtypes = [ctypes.POINTER(_I)]
    L.mgrav_interact_variant_info.restype = _I
    L.mgrav_interact_variant_info.argtypes = [_I, ctypes.POINTER(_I), ctypes.POINTER(_I),
                                              ctypes.POINTER(_I)]
    L.mgrav_set_interact_variant.restype = _I
    L.mgrav_set_interact_variant.argtypes = [_P, _I]
    L.mgrav_autotune.restype = _I
    L.mgrav_autotune.argtypes = [_P, _P, _P, ctypes.c_char_p, _D, ctypes.POINTER(_I), _P]
    L.mgrav_set_launch_mode.restype = _I
    L.mgrav_set_launch_mode.argtypes = [_P, _I]
    L.mgrav_set_queue_order.restype = _I
    L.mgrav_set_queue_order.argtypes = [_P, _I]
    L.mgrav_tree_workspace_size.restype = _I
    L.mgrav_tree_workspace_size.argtypes = [_I64, _I, _I64, ctypes.POINTER(ctypes.c_size_t)]
    L.mgrav_tree_build.restype = _I
    L.mgrav_tree_build.argtypes = [_P, _I64, _P, _P, _P, _D, _I, _P, ctypes.c_size_t, _I64,
                                   ctypes.POINTER(TreeDev), ctypes.POINTER(_I64),
                                   ctypes.POINTER(_I64), ctypes.POINTER(_I64)]
    L.mgrav_lists_workspace_size.restype = _I
    L.mgrav_lists_workspace_size.argtypes = [_I64, _I64, ctypes.POINTER(ctypes.c_size_t)]
    L.mgrav_tree_offset.restype = _I
    L.mgrav_tree_offset.argtypes = [_P, ctypes.POINTER(TreeDev), _I64, _I64, _I64, _I64, _I64,
                                    _P, _I64]
    L.mgrav_lists_count.restype = _I
    L.mgrav_lists_count.argtypes = [_P, ctypes.POINTER(Walk), _P, ctypes.c_size_t, _P, _P,
                                    ctypes.POINTER(_I64), ctypes.POINTER(_I64)]
    L.mgrav_lists_fill.restype = _I
    L.mgrav_lists_fill.argtypes = [_P, ctypes.POINTER(Walk), _P, ctypes.c_size_t, _P, _P, _P,
                                   _P, _P, _P]
    SP = ctypes.POINTER(Store)
    L.mgrav_store_encode.restype = _I
    L.mgrav_store_encode.argtypes = [_P, _I64, _P, _P, _I, SP]
    L.mgrav_store_decode.restype = _I
    L.mgrav_store_decode.argtypes = [_P, _I64, SP, _P, _P]
    L.mgrav_store_permute.restype = _I
    L.mgrav_store_permute.argtypes = [_P, _I64, SP, _P, SP]
    L.mgrav_store_drift.restype = _I
    L.mgrav_store_drift.argtypes = [_P, _I64, SP, _D, _I]
    L.mgrav_store_drift_rungs.restype = _I
    L.mgrav_store_drift_rungs.argtypes = [_P, _I64, SP, _D, _I, _I, _I]
    L.mgrav_store_kick.restype = _I
    L.mgrav_store_kick.argtypes = [_P, _I64, SP, _P, _D, _I]
    L.mgrav_store_rungs.restype = _I
    L.mgrav_store_rungs.argtypes = [_P, _I64, SP, _P, _D, _D, _D, _I, _I, _I]
    L.mgrav_store_active.restype = _I
    L.mgrav_store_active.argtypes = [_P, _I64, SP, _I, _P]
    L.mgrav_fmm_lists_count_host.restype = _I
    L.mgrav_fmm_lists_count_host.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _D, _D, _D, _I,
                                             _P, _P, _P]
    L.mgrav_fmm_lists_fill_host.restype = _I
    L.mgrav_fmm_lists_fill_host.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _D, _D, _D, _I,
                                            _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.mgrav_fmm_workspace_size.restype = _I
    L.mgrav_fmm_workspace_size.argtypes = [_I64, ctypes.POINTER(ctypes.c_size_t)]
    L.mgrav_fmm_apply.restype = _I
    L.mgrav_fmm_apply.argtypes = [_P, ctypes.POINTER(Fmm), _P, ctypes.c_size_t, _P, _P, _P]
    L.mgrav_watchdog_poll.restype = _I
    L.mgrav_watchdog_poll.argtypes = [WATCHDOG_QUERY, _P, _D]


_declare()

# Every symbol include/mgrav.h declares (checked by the CPU tests).
EXPORTS = (
    "mgrav_version", "mgrav_status_string", "mgrav_last_error", "mgrav_create",
    "mgrav_destroy", "mgrav_tree_build_host", "mgrav_lists_count_host",
    "mgrav_lists_fill_host", "mgrav_workspace_size", "mgrav_bind", "mgrav_bind_static", "mgrav_set_ewald",
    "mgrav_set_active", "mgrav_compute", "mgrav_compute_parts", "mgrav_wait",
    "mgrav_ewald_psi", "mgrav_mlp_workspace_size", "mgrav_mlp_attach", "mgrav_mlp_set_weights",
    "mgrav_mlp_get_weights", "mgrav_mlp_forward", "mgrav_mlp_backward", "mgrav_mlp_train",
    "mgrav_interact_variants", "mgrav_interact_variant_info", "mgrav_set_interact_variant",
    "mgrav_autotune", "mgrav_set_launch_mode", "mgrav_set_queue_order", "mgrav_watchdog_poll",
    "mgrav_tree_workspace_size", "mgrav_tree_build", "mgrav_tree_offset",
    "mgrav_lists_workspace_size",
    "mgrav_lists_count", "mgrav_lists_fill", "mgrav_store_encode", "mgrav_store_decode",
    "mgrav_store_permute", "mgrav_store_drift", "mgrav_store_drift_rungs", "mgrav_store_kick",
    "mgrav_store_rungs",
    "mgrav_store_active", "mgrav_fmm_lists_count_host", "mgrav_fmm_lists_fill_host",
    "mgrav_fmm_workspace_size", "mgrav_fmm_apply",
)


class MgravError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        name = _lib.mgrav_status_string(status).decode()
        super().__init__(f"mgrav: {name} ({status}): {msg}")


def _check(status: int, ctx=None):
    if status != OK:
        msg = _lib.mgrav_last_error(ctx).decode(errors="replace")
        raise MgravError(status, msg)


def watchdog_poll(query, timeout_s: float) -> int:
    """The library's watchdog loop on a Python completion query (a callable
    returning 0 when done, > 0 while pending, < 0 on failure); returns the
    status code (OK, TIMEOUT or DEVICE) without raising."""
    cb = WATCHDOG_QUERY(lambda _user: int(query()))
    return int(_lib.mgrav_watchdog_poll(cb, None, float(timeout_s)))


def version() -> int:
    return _lib.mgrav_version()


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Host-side input preparation (tree build and checklist walk on the CPU)
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Tree:
    """Host arrays of a tree, layout as in include/mgrav.h."""

    perm: np.ndarray
    cell_first: np.ndarray
    cell_count: np.ndarray
    child: np.ndarray
    com: np.ndarray
    bmax: np.ndarray
    bbox: np.ndarray
    mom: np.ndarray
    bucket_cell: np.ndarray
    box_L: float

    @property
    def n_cell(self):
        return int(self.cell_first.shape[0])

    @property
    def n_bucket(self):
        return int(self.bucket_cell.shape[0])


@dataclasses.dataclass
class Lists:
    pp_off: np.ndarray
    pp_src: np.ndarray
    pp_img: np.ndarray
    pc_off: np.ndarray
    pc_src: np.ndarray
    pc_img: np.ndarray
    n_images: int


@dataclasses.dataclass
class ParticleStore:
    """Device arrays of the 28-byte particle store (mgrav_store): q [n, 3]
    (uint32 bits held in int32), vel [n, 3] float32, aux [n] (rung in bits
    0..7, group id above); x = origin + q * scale."""

    q: object
    vel: object
    aux: object
    origin: tuple
    scale: float

    @property
    def n(self) -> int:
        return int(self.q.shape[0])

    def c(self) -> "Store":
        s = Store()
        s.q, s.vel, s.aux = self.q.data_ptr(), self.vel.data_ptr(), self.aux.data_ptr()
        for k in range(3):
            s.origin[k] = self.origin[k]
        s.scale = self.scale
        return s

    @property
    def rung(self):
        return self.aux & 0xff


@dataclasses.dataclass
class KeptForest:
    """A fixed tree kept for a forest (Sec. 3.2): the forest's arrays with
    the first tree in place and room for the second (``Context.forest_keep``,
    ``Context.forest_rebuild``)."""

    arrays: dict
    n_cell_first: int
    n_bucket_first: int
    n_first: int
    ids_second: object
    cap_second: int
    box_L: float
    bucket: int


@dataclasses.dataclass
class DeviceTree:
    """Tree (or two-tree forest) built on the device: torch tensors in the
    layout of include/mgrav.h, plus the particles in tree order."""

    perm: object
    pos: object
    mass: object
    cell_first: object
    cell_count: object
    child: object
    com: object
    bmax: object
    bbox: object
    mom: object
    bucket_cell: object
    box_L: float
    n_cell_first: int  # cells of the first tree (all cells for one tree)
    grouped: bool

    @property
    def roots(self):
        return (0, self.n_cell_first) if self.grouped else (0,)

    @property
    def n_bucket_first(self) -> int:
        return (self.n_cell_first + 1) // 2

    def to_host(self) -> "Tree":
        f = {k: getattr(self, k).cpu().numpy() for k in
             ("perm", "cell_first", "cell_count", "child", "com", "bmax", "bbox", "mom",
              "bucket_cell")}
        return Tree(**f, box_L=self.box_L)


@dataclasses.dataclass
class DeviceLists:
    pp_off: object
    pp_src: object
    pp_img: object
    pc_off: object
    pc_src: object
    pc_img: object
    n_images: int
    first_sink: int  # buckets before it have empty lists

    def to_host(self) -> "Lists":
        return Lists(*[getattr(self, k).cpu().numpy() for k in
                       ("pp_off", "pp_src", "pp_img", "pc_off", "pc_src", "pc_img")],
                     self.n_images)


def tree_build(pos: np.ndarray, mass: np.ndarray, box_L: float, bucket: int = 16) -> Tree:
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[0]
    # A tree of buckets of b particles has about 2n/b cells; n/2 covers every
    # tree with average leaf occupancy of 4 or more.  Degenerate inputs that
    # need more (the bound is 2n) are built again with the full capacity.
    for cap in (n // 2 + 64, 2 * n + 2):
        perm = np.empty(n, np.int64)
        cf = np.empty(cap, np.int64)
        cc = np.empty(cap, np.int32)
        ch = np.empty(2 * cap, np.int32)
        com = np.empty(3 * cap)
        bmax = np.empty(cap)
        bbox = np.empty(6 * cap)
        mom = np.empty(32 * cap)
        bc = np.empty(cap, np.int32)
        nc = np.zeros(1, np.int64)
        nb = np.zeros(1, np.int64)
        st = _lib.mgrav_tree_build_host(n, _ptr(pos), _ptr(mass), float(box_L), int(bucket), cap,
                                        _ptr(perm), _ptr(cf), _ptr(cc), _ptr(ch), _ptr(com),
                                        _ptr(bmax), _ptr(bbox), _ptr(mom), _ptr(bc), _ptr(nc),
                                        _ptr(nb))
        if st == OK:
            break
        msg = _lib.mgrav_last_error(None)
        if st != ERR_INVALID_ARG or b"capacity" not in (msg or b"") or cap >= 2 * n + 2:
            _check(st)
    c, b = int(nc[0]), int(nb[0])
    # views of the first c cells (no copy: at 512^3 the moment array alone
    # is several GB)
    return Tree(perm, cf[:c], cc[:c], ch[:2 * c].reshape(c, 2), com[:3 * c].reshape(c, 3),
                bmax[:c], bbox[:6 * c].reshape(c, 6), mom[:32 * c].reshape(c, 32), bc[:b],
                float(box_L))


def lists_build(tree: Tree, theta: float, eps: float, n_images: Optional[int] = None) -> Lists:
    if n_images is None:
        n_images = 27 if tree.box_L > 0 else 1
    nb = tree.n_bucket
    pp_off = np.zeros(nb + 1, np.int64)
    pc_off = np.zeros(nb + 1, np.int64)
    common = (nb, _ptr(tree.bucket_cell), _ptr(tree.child), _ptr(tree.com), _ptr(tree.bmax),
              _ptr(tree.bbox), float(theta), float(eps), float(tree.box_L), int(n_images))
    _check(_lib.mgrav_lists_count_host(*common, _ptr(pp_off), _ptr(pc_off)))
    pp_src = np.empty(max(1, int(pp_off[-1])), np.int32)
    pp_img = np.empty(max(1, int(pp_off[-1])), np.uint8)
    pc_src = np.empty(max(1, int(pc_off[-1])), np.int32)
    pc_img = np.empty(max(1, int(pc_off[-1])), np.uint8)
    _check(_lib.mgrav_lists_fill_host(*common, _ptr(pp_off), _ptr(pc_off), _ptr(pp_src),
                                      _ptr(pp_img), _ptr(pc_src), _ptr(pc_img)))
    npp, npc = int(pp_off[-1]), int(pc_off[-1])
    return Lists(pp_off, pp_src[:npp], pp_img[:npp], pc_off, pc_src[:npc], pc_img[:npc],
                 int(n_images))


@dataclasses.dataclass
class FmmLists:
    """Lists of the fast-multipole walk (include/mgrav.h): per bucket PP
    (with pp_sub) and PC entries, per cell CC / CP entries."""
    pp_off: np.ndarray
    pp_src: np.ndarray
    pp_img: np.ndarray
    pp_sub: np.ndarray
    pc_off: np.ndarray
    pc_src: np.ndarray
    pc_img: np.ndarray
    cc_off: np.ndarray
    cc_src: np.ndarray
    cc_img: np.ndarray
    n_images: int


def fmm_lists_build(tree: Tree, pos_tree: np.ndarray, theta: float, eps: float,
                    n_images: Optional[int] = None) -> FmmLists:
    """The fast-multipole walk on the host (C++/OpenMP)."""
    if n_images is None:
        n_images = 27 if tree.box_L > 0 else 1
    pos_tree = np.ascontiguousarray(pos_tree, dtype=np.float64)
    nb, nc = tree.n_bucket, tree.n_cell
    pp_off = np.zeros(nb + 1, np.int64)
    pc_off = np.zeros(nb + 1, np.int64)
    cc_off = np.zeros(nc + 1, np.int64)
    head = (nc, _ptr(tree.cell_first), _ptr(tree.cell_count), _ptr(tree.child), _ptr(tree.com),
            _ptr(tree.bmax), _ptr(tree.bbox), _ptr(pos_tree), float(theta), float(eps),
            float(tree.box_L), int(n_images))
    _check(_lib.mgrav_fmm_lists_count_host(*head, _ptr(pp_off), _ptr(pc_off), _ptr(cc_off)))
    o = dict(pp_src=np.empty(max(1, pp_off[-1]), np.int32),
             pp_img=np.empty(max(1, pp_off[-1]), np.uint8),
             pp_sub=np.empty(max(1, pp_off[-1]), np.uint8),
             pc_src=np.empty(max(1, pc_off[-1]), np.int32),
             pc_img=np.empty(max(1, pc_off[-1]), np.uint8),
             cc_src=np.empty(max(1, cc_off[-1]), np.int32),
             cc_img=np.empty(max(1, cc_off[-1]), np.uint8))
    _check(_lib.mgrav_fmm_lists_fill_host(*head, _ptr(pp_off), _ptr(pc_off), _ptr(cc_off),
                                          *[_ptr(o[k]) for k in ("pp_src", "pp_img", "pp_sub",
                                                                 "pc_src", "pc_img", "cc_src",
                                                                 "cc_img")]))
    npp, npc, ncc = int(pp_off[-1]), int(pc_off[-1]), int(cc_off[-1])
    return FmmLists(pp_off, o["pp_src"][:npp], o["pp_img"][:npp], o["pp_sub"][:npp], pc_off,
                    o["pc_src"][:npc], o["pc_img"][:npc], cc_off, o["cc_src"][:ncc],
                    o["cc_img"][:ncc], int(n_images))


# --------------------------------------------------------------------------
# Device side
# --------------------------------------------------------------------------
def interact_variants():
    """[(pp_chunk, waves_per_simd, pc_prefetch), ...] of the compiled PP + PC
    kernel variants, by index."""
    n = _I(0)
    _check(_lib.mgrav_interact_variants(ctypes.byref(n)))
    out = []
    for v in range(n.value):
        ch, wv, pf = _I(0), _I(0), _I(0)
        _check(_lib.mgrav_interact_variant_info(v, ctypes.byref(ch), ctypes.byref(wv),
                                                ctypes.byref(pf)))
        out.append((ch.value, wv.value, pf.value))
    return out


class Context:
    """One mgrav context on a device and a (torch) HIP stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("mgrav needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        h = _P()
        _check(_lib.mgrav_create(int(device), _P(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None):
            _lib.mgrav_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------------
    def upload(self, pos_tree: np.ndarray, mass_tree: np.ndarray, tree, lists, eps: float,
               theta: float):
        """Copy particles (tree order), tree and lists to the device and
        return the device tensors plus a filled Problem (not yet bound)."""
        torch = self._torch
        dev = torch.device("cuda", self.device)

        def t(a, dtype=None):
            a = np.ascontiguousarray(a if dtype is None else a.astype(dtype))
            return torch.from_numpy(a).to(dev)

        keep = dict(
            pos=t(pos_tree, np.float64), mass=t(mass_tree, np.float64),
            cell_first=t(tree.cell_first, np.int64), cell_count=t(tree.cell_count, np.int32),
            child=t(tree.child, np.int32), com=t(tree.com, np.float64),
            bbox=t(tree.bbox, np.float64), mom=t(tree.mom, np.float64),
            bucket_cell=t(tree.bucket_cell, np.int32), pp_off=t(lists.pp_off, np.int64),
            pp_src=t(lists.pp_src if lists.pp_src.size else np.zeros(1, np.int32), np.int32),
            pp_img=t(lists.pp_img if lists.pp_img.size else np.zeros(1, np.uint8), np.uint8),
            pc_off=t(lists.pc_off, np.int64),
            pc_src=t(lists.pc_src if lists.pc_src.size else np.zeros(1, np.int32), np.int32),
            pc_img=t(lists.pc_img if lists.pc_img.size else np.zeros(1, np.uint8), np.uint8),
        )
        p = Problem()
        p.n = pos_tree.shape[0]
        p.eps = float(eps)
        p.theta = float(theta)
        p.box_L = float(tree.box_L)
        p.n_images = int(lists.n_images)
        p.n_cell = int(tree.cell_first.shape[0])
        p.n_bucket = int(tree.bucket_cell.shape[0])
        for name in ("pos", "mass", "cell_first", "cell_count", "child", "com", "bbox", "mom",
                     "bucket_cell", "pp_off", "pp_src", "pp_img", "pc_off", "pc_src",
                     "pc_img"):
            setattr(p, name, keep[name].data_ptr())
        p.n_pp = int(lists.pp_off[-1])
        p.n_pc = int(lists.pc_off[-1])
        sub = getattr(lists, "pp_sub", None)
        if sub is not None:
            keep["pp_sub"] = t(sub if sub.size else np.zeros(1, np.uint8), np.uint8)
            p.pp_sub = keep["pp_sub"].data_ptr()
        torch.cuda.synchronize(dev)
        return keep, p

    def _tree_build_into(self, pos_dev, mass_dev, box_L: float, bucket: int, group_dev,
                         cap: int, out: dict):
        """One mgrav_tree_build call writing into the tensors of ``out`` (room
        for ``cap`` cells).  Returns (cells, buckets, first tree's cells), or
        None when the tree needs more than ``cap`` cells."""
        torch = self._torch
        dev = torch.device("cuda", self.device)
        n = int(pos_dev.shape[0])
        sz = ctypes.c_size_t(0)
        _check(_lib.mgrav_tree_workspace_size(n, int(bucket), int(cap), ctypes.byref(sz)))
        ws = torch.empty(int(sz.value), dtype=torch.uint8, device=dev)
        td = TreeDev(*[out[f].data_ptr() for f, _ in TreeDev._fields_])
        nc, nb, nf = _I64(0), _I64(0), _I64(0)
        st = _lib.mgrav_tree_build(self._h, n, _P(pos_dev.data_ptr()), _P(mass_dev.data_ptr()),
                                   _P(group_dev.data_ptr()) if group_dev is not None else None,
                                   float(box_L), int(bucket), _P(ws.data_ptr()),
                                   ctypes.c_size_t(ws.numel()), int(cap), ctypes.byref(td),
                                   ctypes.byref(nc), ctypes.byref(nb), ctypes.byref(nf))
        del ws
        if st == OK:
            return int(nc.value), int(nb.value), int(nf.value)
        msg = _lib.mgrav_last_error(self._h) or b""
        if st == ERR_INVALID_ARG and b"capacity" in msg:
            return None
        _check(st, self._h)

    def _tree_out(self, n: int, cap: int) -> dict:
        torch = self._torch
        dev = torch.device("cuda", self.device)
        f64 = dict(dtype=torch.float64, device=dev)
        return dict(perm=torch.empty(n, dtype=torch.int64, device=dev),
                    pos=torch.empty((n, 3), **f64), mass=torch.empty(n, **f64),
                    cell_first=torch.empty(cap, dtype=torch.int64, device=dev),
                    cell_count=torch.empty(cap, dtype=torch.int32, device=dev),
                    child=torch.empty((cap, 2), dtype=torch.int32, device=dev),
                    com=torch.empty((cap, 3), **f64), bmax=torch.empty(cap, **f64),
                    bbox=torch.empty((cap, 6), **f64), mom=torch.empty((cap, 32), **f64),
                    bucket_cell=torch.empty(cap, dtype=torch.int32, device=dev))

    def tree_build(self, pos_dev, mass_dev, box_L: float, bucket: int = 16, group_dev=None,
                   cap: Optional[int] = None):
        """The tree (or, with ``group_dev``, the two-tree forest of Sec. 3.2)
        built on the device from positions [n, 3] and masses [n] (float64
        device tensors, input order).  Returns a DeviceTree of device
        tensors trimmed to the cell count."""
        torch = self._torch
        dev = torch.device("cuda", self.device)
        n = int(pos_dev.shape[0])
        pos_dev = pos_dev.contiguous()
        mass_dev = mass_dev.contiguous()
        caps = [cap] if cap else sorted({min(c, 2 * n + 2) for c in (max(64, n // 4), n // 2 + 64,
                                                                     2 * n + 2)})
        self.stream.wait_stream(torch.cuda.current_stream(dev))
        for k, cp in enumerate(caps):
            out = self._tree_out(n, cp)
            got = self._tree_build_into(pos_dev, mass_dev, box_L, bucket, group_dev, cp, out)
            if got is not None:
                break
            if k == len(caps) - 1:
                raise MgravError(ERR_INVALID_ARG, "tree: capacity")
        c, b, nf = got
        trim = {f: (v if f in ("perm", "pos", "mass") else v[:(b if f == "bucket_cell" else c)])
                for f, v in out.items()}
        return DeviceTree(**trim, box_L=float(box_L), n_cell_first=nf,
                          grouped=group_dev is not None)

    def _tree_offset(self, views: dict, n_cell: int, n_bucket: int, n_part: int,
                     cell_offset: int, particle_offset: int, ids):
        td = TreeDev(*[views[f].data_ptr() for f, _ in TreeDev._fields_])
        _check(_lib.mgrav_tree_offset(self._h, ctypes.byref(td), int(n_cell), int(n_bucket),
                                      int(n_part), int(cell_offset), int(particle_offset),
                                      _P(ids.data_ptr()) if ids is not None else None,
                                      int(ids.numel()) if ids is not None else 0), self._h)

    def forest_keep(self, pos_dev, mass_dev, box_L: float, group_dev, bucket: int = 16):
        """The fixed tree of Sec. 3.2 built once: the tree of the group-0
        particles alone (periodic box), renumbered as the first tree of the
        forest over all particles and stored with room for a second tree of
        the other particles (``forest_rebuild`` adds it)."""
        torch = self._torch
        if not box_L > 0:
            raise ValueError("forest_keep: a periodic box is needed (an open forest takes the "
                             "root box of all particles)")
        n = int(pos_dev.shape[0])
        g = group_dev.to(torch.bool)
        ids0 = torch.nonzero(~g).flatten()
        ids1 = torch.nonzero(g).flatten()
        n0, n1 = int(ids0.numel()), int(ids1.numel())
        if n0 == 0 or n1 == 0:
            raise ValueError("forest_keep: both groups must be non-empty")
        t0 = self.tree_build(pos_dev.index_select(0, ids0), mass_dev.index_select(0, ids0),
                             box_L, bucket)
        nc0, nb0 = int(t0.cell_first.shape[0]), int(t0.bucket_cell.shape[0])
        fields0 = {f.name: getattr(t0, f.name) for f in dataclasses.fields(t0)}
        self._tree_offset(fields0, nc0, nb0, n0, 0, 0, ids0)
        cap1 = 2 * n1 + 2
        arrays = self._tree_out(n, nc0 + cap1)
        for f, v in arrays.items():
            src = getattr(t0, f)
            v[:src.shape[0]].copy_(src)
        return KeptForest(arrays=arrays, n_cell_first=nc0, n_bucket_first=nb0, n_first=n0,
                          ids_second=ids1, cap_second=cap1, box_L=float(box_L), bucket=bucket)

    def forest_rebuild(self, kf, pos_dev, mass_dev):
        """The very active tree of Sec. 3.2 rebuilt alone from the group != 0
        particles of pos_dev / mass_dev (input order, current positions) and
        put behind the kept fixed tree.  Returns the forest as a DeviceTree
        (views of the kept arrays, valid until the next rebuild)."""
        torch = self._torch
        dev = torch.device("cuda", self.device)
        ids = kf.ids_second
        p1 = pos_dev.index_select(0, ids).contiguous()
        m1 = mass_dev.index_select(0, ids).contiguous()
        nc0, nb0, n0 = kf.n_cell_first, kf.n_bucket_first, kf.n_first
        A = kf.arrays
        views = {f: (v[n0:] if f in ("perm", "pos", "mass") else
                     v[(nb0 if f == "bucket_cell" else nc0):]) for f, v in A.items()}
        self.stream.wait_stream(torch.cuda.current_stream(dev))
        got = self._tree_build_into(p1, m1, kf.box_L, kf.bucket, None, kf.cap_second, views)
        if got is None:  # cannot happen with room for 2 n + 2 cells
            raise MgravError(ERR_INVALID_ARG, "forest_rebuild: capacity")
        nc1, nb1, _ = got
        self._tree_offset(views, nc1, nb1, int(ids.numel()), nc0, n0, ids)
        trim = {f: (v if f in ("perm", "pos", "mass") else
                    v[:(nb0 + nb1 if f == "bucket_cell" else nc0 + nc1)]) for f, v in A.items()}
        return DeviceTree(**trim, box_L=kf.box_L, n_cell_first=nc0, grouped=True)

    def lists_build(self, dtree, theta: float, eps: float, sinks: str = "all",
                    n_images: Optional[int] = None):
        """Checklist walk on the device for the buckets of a DeviceTree
        (``sinks='all'``) or of its second tree only (``'second'``, a forest);
        the checklist holds every root of the tree.  Returns DeviceLists
        whose offsets cover every bucket of the tree (buckets that are not
        sinks get empty lists)."""
        torch = self._torch
        dev = torch.device("cuda", self.device)
        L = dtree.box_L
        nimg = n_images if n_images is not None else (27 if L > 0 else 1)
        nb = int(dtree.bucket_cell.shape[0])
        first = 0
        if sinks == "second":
            if not dtree.grouped:
                raise ValueError("sinks='second' needs a forest")
            first = dtree.n_bucket_first
        w = Walk()
        w.n_cell = int(dtree.cell_first.shape[0])
        w.child, w.com = dtree.child.data_ptr(), dtree.com.data_ptr()
        w.bmax, w.bbox = dtree.bmax.data_ptr(), dtree.bbox.data_ptr()
        roots = dtree.roots
        w.n_roots = len(roots)
        w.roots[0] = roots[0]
        w.roots[1] = roots[1] if len(roots) > 1 else 0
        w.theta, w.eps, w.L, w.n_images = float(theta), float(eps), float(L), int(nimg)
        w.n_sink = nb - first
        sink = dtree.bucket_cell[first:]
        w.sink_cell = sink.data_ptr()
        sz = ctypes.c_size_t(0)
        _check(_lib.mgrav_lists_workspace_size(w.n_cell, w.n_sink, ctypes.byref(sz)))
        ws = torch.empty(int(sz.value), dtype=torch.uint8, device=dev)
        pp_off = torch.zeros(nb + 1, dtype=torch.int64, device=dev)
        pc_off = torch.zeros(nb + 1, dtype=torch.int64, device=dev)
        self.stream.wait_stream(torch.cuda.current_stream(dev))
        npp, npc = _I64(0), _I64(0)
        _check(_lib.mgrav_lists_count(self._h, ctypes.byref(w), _P(ws.data_ptr()),
                                      ctypes.c_size_t(ws.numel()), _P(pp_off[first:].data_ptr()),
                                      _P(pc_off[first:].data_ptr()), ctypes.byref(npp),
                                      ctypes.byref(npc)), self._h)
        pp_src = torch.empty(max(1, npp.value), dtype=torch.int32, device=dev)
        pp_img = torch.empty(max(1, npp.value), dtype=torch.uint8, device=dev)
        pc_src = torch.empty(max(1, npc.value), dtype=torch.int32, device=dev)
        pc_img = torch.empty(max(1, npc.value), dtype=torch.uint8, device=dev)
        _check(_lib.mgrav_lists_fill(self._h, ctypes.byref(w), _P(ws.data_ptr()),
                                     ctypes.c_size_t(ws.numel()), _P(pp_off[first:].data_ptr()),
                                     _P(pc_off[first:].data_ptr()), _P(pp_src.data_ptr()),
                                     _P(pp_img.data_ptr()), _P(pc_src.data_ptr()),
                                     _P(pc_img.data_ptr())), self._h)
        return DeviceLists(pp_off, pp_src[:npp.value], pp_img[:npp.value], pc_off,
                           pc_src[:npc.value], pc_img[:npc.value], int(nimg), first)

    def _sync_in(self):
        """Inputs produced on torch's current stream come before the
        context's own work."""
        torch = self._torch
        self.stream.wait_stream(torch.cuda.current_stream(torch.device("cuda", self.device)))

    # ---- particle store (Sec. 3.4) and integrator steps (Sec. 3.2) ----
    def store_alloc(self, n: int, origin, scale: float) -> "ParticleStore":
        torch = self._torch
        dev = torch.device("cuda", self.device)
        return ParticleStore(torch.zeros((n, 3), dtype=torch.int32, device=dev),
                             torch.zeros((n, 3), dtype=torch.float32, device=dev),
                             torch.zeros(n, dtype=torch.int32, device=dev),
                             tuple(float(o) for o in origin), float(scale))

    def store_encode(self, st: "ParticleStore", pos_dev, vel_dev=None, periodic: bool = True):
        self._sync_in()
        s = st.c()
        _check(_lib.mgrav_store_encode(self._h, st.n, _P(pos_dev.contiguous().data_ptr()),
                                       _P(vel_dev.contiguous().data_ptr()) if vel_dev is not None
                                       else None, int(bool(periodic)), ctypes.byref(s)), self._h)

    def store_decode(self, st: "ParticleStore", with_vel: bool = False):
        self._sync_in()
        torch = self._torch
        dev = torch.device("cuda", self.device)
        pos = torch.empty((st.n, 3), dtype=torch.float64, device=dev)
        vel = torch.empty((st.n, 3), dtype=torch.float32, device=dev) if with_vel else None
        s = st.c()
        _check(_lib.mgrav_store_decode(self._h, st.n, ctypes.byref(s), _P(pos.data_ptr()),
                                       _P(vel.data_ptr()) if vel is not None else None), self._h)
        return (pos, vel) if with_vel else pos

    def store_permute(self, st: "ParticleStore", perm_dev) -> "ParticleStore":
        out = self.store_alloc(st.n, st.origin, st.scale)
        self._sync_in()
        a, b = st.c(), out.c()
        _check(_lib.mgrav_store_permute(self._h, st.n, ctypes.byref(a), _P(perm_dev.data_ptr()),
                                        ctypes.byref(b)), self._h)
        return out

    def store_drift(self, st: "ParticleStore", dt: float, periodic: bool = True):
        self._sync_in()
        s = st.c()
        _check(_lib.mgrav_store_drift(self._h, st.n, ctypes.byref(s), float(dt),
                                      int(bool(periodic))), self._h)

    def store_drift_rungs(self, st: "ParticleStore", dt: float, periodic: bool, rung_lo: int,
                          rung_hi: int):
        """Drift of the particles on rungs rung_lo <= rung < rung_hi only."""
        self._sync_in()
        s = st.c()
        _check(_lib.mgrav_store_drift_rungs(self._h, st.n, ctypes.byref(s), float(dt),
                                            int(bool(periodic)), int(rung_lo), int(rung_hi)),
               self._h)

    def store_kick(self, st: "ParticleStore", acc_dev, dt_base: float, rung_lo: int):
        self._sync_in()
        s = st.c()
        _check(_lib.mgrav_store_kick(self._h, st.n, ctypes.byref(s), _P(acc_dev.data_ptr()),
                                     float(dt_base), int(rung_lo)), self._h)

    def store_rungs(self, st: "ParticleStore", acc_dev, eps: float, eta: float, dt_base: float,
                    rung_lo: int, rung_floor: int, rung_max: int):
        self._sync_in()
        s = st.c()
        _check(_lib.mgrav_store_rungs(self._h, st.n, ctypes.byref(s), _P(acc_dev.data_ptr()),
                                      float(eps), float(eta), float(dt_base), int(rung_lo),
                                      int(rung_floor), int(rung_max)), self._h)

    def store_active(self, st: "ParticleStore", rung_lo: int):
        self._sync_in()
        torch = self._torch
        act = torch.empty(st.n, dtype=torch.uint8, device=torch.device("cuda", self.device))
        s = st.c()
        _check(_lib.mgrav_store_active(self._h, st.n, ctypes.byref(s), int(rung_lo),
                                       _P(act.data_ptr())), self._h)
        return act

    def fmm_apply(self, pos_tree_dev, mass_tree_dev, keep: dict, fl_dev: dict, eps: float,
                  box_L: float, acc, pot, active_dev=None, want_local: bool = False):
        """The CC / CP part (local expansions) added to acc / pot after a
        compute: keep holds the bound problem's device tensors (tree), fl_dev
        the device CC lists (cc_off, cc_src, cc_img)."""
        torch = self._torch
        dev = torch.device("cuda", self.device)
        f = Fmm()
        f.n = int(pos_tree_dev.shape[0])
        f.n_cell = int(keep["cell_first"].shape[0])
        f.n_bucket = int(keep["bucket_cell"].shape[0])
        for k in ("child", "com", "mom", "cell_first", "cell_count", "bucket_cell"):
            setattr(f, k, keep[k].data_ptr())
        f.pos = pos_tree_dev.data_ptr()
        f.mass = mass_tree_dev.data_ptr()
        f.eps, f.box_L = float(eps), float(box_L)
        for k in ("cc_off", "cc_src", "cc_img"):
            setattr(f, k, fl_dev[k].data_ptr())
        f.active = active_dev.data_ptr() if active_dev is not None else None
        sz = ctypes.c_size_t(0)
        _check(_lib.mgrav_fmm_workspace_size(f.n_cell, ctypes.byref(sz)))
        ws = torch.empty(int(sz.value), dtype=torch.uint8, device=dev)
        local = torch.empty((f.n_bucket, 56), dtype=torch.float64, device=dev) if want_local \
            else None
        self._sync_in()
        _check(_lib.mgrav_fmm_apply(self._h, ctypes.byref(f), _P(ws.data_ptr()),
                                    ctypes.c_size_t(ws.numel()), _P(acc.data_ptr()),
                                    _P(pot.data_ptr()),
                                    _P(local.data_ptr()) if local is not None else None), self._h)
        return local

    def problem_device(self, dtree, dlists, eps: float, theta: float):
        """A Problem over a DeviceTree and DeviceLists (no host copies);
        returns (tensors to keep alive, Problem)."""
        keep = dict(pos=dtree.pos, mass=dtree.mass, cell_first=dtree.cell_first,
                    cell_count=dtree.cell_count, child=dtree.child, com=dtree.com,
                    bbox=dtree.bbox, mom=dtree.mom, bucket_cell=dtree.bucket_cell,
                    pp_off=dlists.pp_off, pp_src=dlists.pp_src, pp_img=dlists.pp_img,
                    pc_off=dlists.pc_off, pc_src=dlists.pc_src, pc_img=dlists.pc_img)
        torch = self._torch
        one32 = torch.zeros(1, dtype=torch.int32, device=dtree.pos.device)
        one8 = torch.zeros(1, dtype=torch.uint8, device=dtree.pos.device)
        for k, z in (("pp_src", one32), ("pc_src", one32), ("pp_img", one8), ("pc_img", one8)):
            if keep[k].numel() == 0:
                keep[k] = z
        p = Problem()
        p.n = int(dtree.pos.shape[0])
        p.eps, p.theta, p.box_L = float(eps), float(theta), float(dtree.box_L)
        p.n_images = int(dlists.n_images)
        p.n_cell = int(dtree.cell_first.shape[0])
        p.n_bucket = int(dtree.bucket_cell.shape[0])
        for name in ("pos", "mass", "cell_first", "cell_count", "child", "com", "bbox", "mom",
                     "bucket_cell", "pp_off", "pp_src", "pp_img", "pc_off", "pc_src",
                     "pc_img"):
            setattr(p, name, keep[name].data_ptr())
        p.n_pp = int(dlists.pp_src.numel())
        p.n_pc = int(dlists.pc_src.numel())
        return keep, p

    def workspace_size(self, p: Problem) -> int:
        sz = ctypes.c_size_t(0)
        _check(_lib.mgrav_workspace_size(ctypes.byref(p), ctypes.byref(sz)))
        return int(sz.value)

    def bind(self, p: Problem, tensors: dict, workspace=None):
        """Bind a problem; allocates the workspace as a torch uint8 tensor
        unless one is given.  Keeps references to the device tensors."""
        torch = self._torch
        nbytes = self.workspace_size(p)
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8,
                                    device=torch.device("cuda", self.device))
        self._keep = dict(tensors)
        self._keep["workspace"] = workspace
        self.problem = p
        self.n = int(p.n)
        # inputs were produced on torch's current stream
        self.stream.wait_stream(torch.cuda.current_stream(torch.device("cuda", self.device)))
        _check(_lib.mgrav_bind(self._h, ctypes.byref(p), _P(workspace.data_ptr()),
                               ctypes.c_size_t(workspace.numel())), self._h)

    def bind_static(self, p: Problem, tensors: dict):
        """Bind a problem to the library's static workspace (no device
        allocation; see mgrav_bind_static).  Keeps references to the device
        tensors."""
        torch = self._torch
        self._keep = dict(tensors)
        self.problem = p
        self.n = int(p.n)
        self.stream.wait_stream(torch.cuda.current_stream(torch.device("cuda", self.device)))
        _check(_lib.mgrav_bind_static(self._h, ctypes.byref(p)), self._h)

    def set_ewald(self, mode: int = EWALD_EXACT, alpha: float = 2.6, real_layers: int = 1,
                  h2max: int = 10, order: int = 4, top_cells: int = 1,
                  fallback_tol: float = 1e-4, sample_stride: int = 0):
        cfg = EwaldConfig(int(mode), float(alpha), int(real_layers), int(h2max), int(order),
                          int(top_cells), float(fallback_tol), int(sample_stride))
        _check(_lib.mgrav_set_ewald(self._h, ctypes.byref(cfg)), self._h)

    def set_launch_mode(self, mode: int):
        """LAUNCH_GRAPH (one HIP graph per compute) or LAUNCH_DIRECT."""
        _check(_lib.mgrav_set_launch_mode(self._h, int(mode)), self._h)

    def set_queue_order(self, order: int):
        """QUEUE_AUTO, QUEUE_LPT (most expensive buckets first) or QUEUE_LOCAL
        (expensive ones first, the rest in tree order per die)."""
        _check(_lib.mgrav_set_queue_order(self._h, int(order)), self._h)

    def set_interact_variant(self, variant: int):
        _check(_lib.mgrav_set_interact_variant(self._h, int(variant)), self._h)

    def autotune(self, acc, pot, cache_path: Optional[str] = None, budget_ms: float = 2000.0):
        """Time every PP + PC kernel variant on the bound problem and keep the
        fastest.  Returns (variant, [median ms per variant, -1 if untimed])."""
        torch = self._torch
        self.stream.wait_stream(torch.cuda.current_stream(torch.device("cuda", self.device)))
        nv = len(interact_variants())
        ms = (_D * nv)()
        chosen = _I(-1)
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(_lib.mgrav_autotune(self._h, _P(acc.data_ptr()), _P(pot.data_ptr()), path,
                                   float(budget_ms), ctypes.byref(chosen), ms), self._h)
        return chosen.value, list(ms)

    def set_active(self, active_dev=None):
        self._keep["active"] = active_dev
        ptr = None if active_dev is None else _P(active_dev.data_ptr())
        _check(_lib.mgrav_set_active(self._h, ptr), self._h)

    def compute(self, acc, pot, parts: int = PART_ALL):
        torch = self._torch
        self.stream.wait_stream(torch.cuda.current_stream(torch.device("cuda", self.device)))
        _check(_lib.mgrav_compute_parts(self._h, int(parts), _P(acc.data_ptr()),
                                        _P(pot.data_ptr())), self._h)

    def wait(self, timeout_s: float = 60.0) -> Stats:
        st = Stats()
        _check(_lib.mgrav_wait(self._h, float(timeout_s), ctypes.byref(st)), self._h)
        return st

    # ---------------------------------------------------------- surrogate
    def ewald_psi(self, r_dev, alpha: float = 2.6, real_layers: int = 1, h2max: int = 10):
        """psi and grad psi (unit box, unit mass) at device points r[n,3]
        (float64); returns a device tensor [n, 4]."""
        torch = self._torch
        out = torch.empty((r_dev.shape[0], 4), dtype=torch.float64, device=r_dev.device)
        self.stream.wait_stream(torch.cuda.current_stream(r_dev.device))
        _check(_lib.mgrav_ewald_psi(self._h, _P(r_dev.data_ptr()), int(r_dev.shape[0]),
                                    float(alpha), int(real_layers), int(h2max),
                                    _P(out.data_ptr())), self._h)
        torch.cuda.current_stream(r_dev.device).wait_stream(self.stream)
        return out

    def mlp_attach(self, max_batch: int = 8192):
        torch = self._torch
        sz = ctypes.c_size_t(0)
        _check(_lib.mgrav_mlp_workspace_size(int(max_batch), ctypes.byref(sz)))
        ws = torch.empty(sz.value, dtype=torch.uint8, device=torch.device("cuda", self.device))
        self._mlp_ws = ws
        _check(_lib.mgrav_mlp_attach(self._h, _P(ws.data_ptr()), ctypes.c_size_t(sz.value),
                                     int(max_batch)), self._h)

    def mlp_set_weights(self, params: np.ndarray, psi0: float = 0.0):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(_lib.mgrav_mlp_set_weights(self._h, _ptr(p), int(p.size), float(psi0)), self._h)

    def mlp_get_weights(self) -> np.ndarray:
        p = np.empty(MLP_PARAMS, np.float32)
        _check(_lib.mgrav_mlp_get_weights(self._h, _ptr(p), MLP_PARAMS), self._h)
        return p

    def mlp_forward(self, x_dev):
        torch = self._torch
        y = torch.empty((x_dev.shape[0], 4), dtype=torch.float32, device=x_dev.device)
        self.stream.wait_stream(torch.cuda.current_stream(x_dev.device))
        _check(_lib.mgrav_mlp_forward(self._h, _P(x_dev.data_ptr()), int(x_dev.shape[0]),
                                      _P(y.data_ptr())), self._h)
        torch.cuda.current_stream(x_dev.device).wait_stream(self.stream)
        return y

    def mlp_backward(self, x_dev, dy_dev):
        torch = self._torch
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x_dev.device)
        self.stream.wait_stream(torch.cuda.current_stream(x_dev.device))
        _check(_lib.mgrav_mlp_backward(self._h, _P(x_dev.data_ptr()), _P(dy_dev.data_ptr()),
                                       int(x_dev.shape[0]), _P(g.data_ptr())), self._h)
        torch.cuda.current_stream(x_dev.device).wait_stream(self.stream)
        return g

    def mlp_train(self, u_dev, psi_dev, epochs: int, batch: int, lr: float = 2e-3,
                  lr_min: float = 2e-5, loss_weight=(1.0, 1.0, 1.0, 1.0), psi0: float = 0.0,
                  beta1: float = 0.9, beta2: float = 0.999, adam_eps: float = 1e-8):
        torch = self._torch
        cfg = TrainConfig(int(epochs), int(batch), float(lr), float(lr_min), float(beta1),
                          float(beta2), float(adam_eps),
                          (ctypes.c_float * 4)(*[float(w) for w in loss_weight]), float(psi0))
        losses = np.zeros(int(epochs))
        self.stream.wait_stream(torch.cuda.current_stream(u_dev.device))
        _check(_lib.mgrav_mlp_train(self._h, _P(u_dev.data_ptr()), _P(psi_dev.data_ptr()),
                                    int(u_dev.shape[0]), ctypes.byref(cfg), _ptr(losses)),
               self._h)
        return losses

    def outputs(self):
        torch = self._torch
        dev = torch.device("cuda", self.device)
        acc = torch.zeros(3 * self.n, dtype=torch.float32, device=dev)
        pot = torch.zeros(self.n, dtype=torch.float32, device=dev)
        return acc, pot


def solve(ctx: Context, pos_tree, mass_tree, tree, lists, eps: float, theta: float,
          parts: int = PART_ALL, ewald: Optional[dict] = None, active: Optional[np.ndarray] = None,
          timeout_s: float = 120.0):
    """Upload, bind, compute once and return (acc [n,3], pot [n], stats) as
    numpy arrays in tree order."""
    torch = ctx._torch
    tensors, p = ctx.upload(pos_tree, mass_tree, tree, lists, eps, theta)
    ctx.bind(p, tensors)
    if ewald is not None:
        ctx.set_ewald(**ewald)
    if active is not None:
        act = torch.from_numpy(np.ascontiguousarray(active, dtype=np.uint8)).to(
            torch.device("cuda", ctx.device))
        ctx.set_active(act)
    acc, pot = ctx.outputs()
    ctx.compute(acc, pot, parts)
    st = ctx.wait(timeout_s)
    a = acc.cpu().numpy().reshape(3, -1).T.copy()
    return a, pot.cpu().numpy().copy(), st
