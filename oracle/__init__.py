"""FP64 CPU oracle for the gravity hot path (arXiv:1609.08621, Sec. 3.1).

TEST INFRASTRUCTURE ONLY: the plain, slow reference the GPU library is
checked against.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import it.  It shares no code with the GPU library
(``paper_1609_08621_amd``) and imports nothing from it.

The arithmetic lives in ``mgrav_oracle.c`` (plain C99, double precision,
built with gcc); this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mgrav_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Ewald parameters of the "exact" configuration (unit box): Gaussian split
# alpha = 2.6 / L, only the 27 near images in real space, k-space terms
# with |h|^2 <= 10.
EXACT_EWALD = dict(alpha=2.6, rmax=1, h2max=10)
# Converged Ewald kernel used as the reference for truncation errors.
CONVERGED_EWALD = dict(alpha=2.0, rmax=3, h2max=48)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC",
            "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
        _lib.orc_init()
    return _lib


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_D = ctypes.c_double


def _declare(L):
    L.orc_init.argtypes = []
    L.orc_num_threads.restype = _I
    L.orc_num_threads.argtypes = []
    L.orc_image_shift.argtypes = [_I, _D, _P]
    L.orc_tree_build.restype = _I64
    L.orc_tree_build.argtypes = [_I64, _P, _P, _D, _I, _I64, _P, _P, _P, _P, _P, _P, _P,
                                 _P, _P, _P]
    L.orc_tree_build_box.restype = _I64
    L.orc_tree_build_box.argtypes = [_I64, _P, _P, _D, _I, _P, _I64, _P, _P, _P, _P, _P, _P,
                                     _P, _P, _P, _P]
    L.orc_lists_count_roots.argtypes = [_I64, _P, _P, _P, _P, _P, _D, _D, _D, _I, _I, _P, _P,
                                        _P]
    L.orc_lists_fill_roots.argtypes = [_I64, _P, _P, _P, _P, _P, _D, _D, _D, _I, _I, _P, _P,
                                       _P, _P, _P, _P, _P]
    L.orc_fmm_walk.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _D, _D, _D, _I, _I, _P, _P,
                               _P, _P, _P, _P, _P, _P, _P, _P]
    L.orc_fmm_local.argtypes = [_I64, _P, _P, _P, _P, _P, _D, _D, _P, _P, _P, _P]
    L.orc_fmm_l2p.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P]
    L.orc_fmm_m2l_point.argtypes = [_P, _D, _I, _P, _P, _D, _P]
    L.orc_fmm_l2l_point.argtypes = [_P, _P, _P]
    L.orc_fmm_l2p_point.argtypes = [_P, _P, _P]
    L.orc_eval_sub.argtypes = [_I64, _P, _P, _D, _D, _P, _P, _P, _P, _I64, _P, _P, _P, _P, _P,
                               _P, _P, _P, _I64, _P, _I, _D, _I, _I, _P, _P]
    L.orc_lists_count.argtypes = [_I64, _P, _P, _P, _P, _P, _D, _D, _D, _I, _P, _P]
    L.orc_lists_fill.argtypes = [_I64, _P, _P, _P, _P, _P, _D, _D, _D, _I, _P, _P, _P,
                                 _P, _P, _P]
    L.orc_pc_point.argtypes = [_P, _P, _P, _D, _P]
    L.orc_moments.argtypes = [_I64, _P, _P, _P, _P]
    L.orc_set_quadrature.argtypes = [_I]
    L.orc_ewald_derivs.argtypes = [_P, _D, _I, _I, _I, _P]
    L.orc_ewald_root_point.argtypes = [_P, _P, _P, _D, _D, _I, _I, _P]
    L.orc_eval.argtypes = [_I64, _P, _P, _D, _D, _P, _P, _P, _P, _I64, _P, _P, _P, _P, _P,
                           _P, _P, _I64, _P, _I, _D, _I, _I, _P, _P]
    L.orc_direct_open.argtypes = [_I64, _P, _P, _D, _P, _P]
    L.orc_direct_periodic.argtypes = [_I64, _P, _P, _D, _D, _D, _I, _I, _P, _P]


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclasses.dataclass
class Tree:
    """Binary tree in node-left-right order; particles in tree order.

    perm[k] is the input index of the k-th particle in tree order.
    Per cell: first particle, count, children (-1 for leaves), centre of
    mass com[c], b_max, tight bounding box bbox[c] = (lo xyz, hi xyz) and
    packed moments mom[c] (32: mass, order 2 (6), order 3 (10), order 4
    (15), non-decreasing index tuples in lexicographic order).
    bucket_cell[b] is the cell of the b-th leaf (bucket)."""

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
    bucket: int
    roots: tuple = (0,)  # checklist seeds: (0,) for one tree, two for a forest

    @property
    def n_cell(self) -> int:
        return int(self.cell_first.shape[0])

    @property
    def n_bucket(self) -> int:
        return int(self.bucket_cell.shape[0])


@dataclasses.dataclass
class Lists:
    """Per-bucket CSR interaction lists; sources are cell indices, image
    ids 0 (the box) .. 26 (replicas, lexicographic over {-1,0,1}^3)."""

    pp_off: np.ndarray
    pp_src: np.ndarray
    pp_img: np.ndarray
    pc_off: np.ndarray
    pc_src: np.ndarray
    pc_img: np.ndarray
    n_images: int


def num_threads() -> int:
    return int(lib().orc_num_threads())


def image_shift(img: int, L: float) -> np.ndarray:
    out = np.zeros(3)
    lib().orc_image_shift(int(img), float(L), _p(out))
    return out


def build_tree(pos: np.ndarray, mass: np.ndarray, box_L: float, bucket: int = 16,
               root_box: Optional[np.ndarray] = None) -> Tree:
    """Tree of Sec. 3.1 over the particles; ``root_box`` (lo xyz, hi xyz)
    replaces the default root ([0, L)^3, or the tight bounding box when
    open)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    rb = None if root_box is None else np.ascontiguousarray(root_box, dtype=np.float64)
    n = pos.shape[0]
    # room for n/2 cells first (trees of buckets hold about 2n/bucket), the
    # 2n bound only if the builder reports that n/2 is not enough
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
        nb = np.zeros(1, np.int64)
        nc = lib().orc_tree_build_box(n, _p(pos), _p(mass), float(box_L), int(bucket), _p(rb),
                                      cap, _p(perm), _p(cf), _p(cc), _p(ch), _p(com), _p(bmax),
                                      _p(bbox), _p(mom), _p(bc), _p(nb))
        if nc >= 0:
            break
    if nc < 0:
        raise RuntimeError("oracle tree build failed")
    nb = int(nb[0])
    return Tree(perm, cf[:nc], cc[:nc], ch[:2 * nc].reshape(nc, 2), com[:3 * nc].reshape(nc, 3),
                bmax[:nc], bbox[:6 * nc].reshape(nc, 6), mom[:32 * nc].reshape(nc, 32), bc[:nb],
                float(box_L), int(bucket))


def build_forest(pos: np.ndarray, mass: np.ndarray, box_L: float, group: np.ndarray,
                 bucket: int = 16) -> Tree:
    """The two trees of Sec. 3.2: the fixed tree of the particles with
    group 0 and the very active tree of those with group 1, built over the
    same root box (that of all particles), stored as one forest: tree-order
    particles of the fixed tree first, then those of the very active tree;
    cells of the fixed tree first (root 0), then those of the very active
    tree (root n_cell of the fixed tree).  Both groups must be non-empty."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    group = np.asarray(group) != 0
    if box_L > 0:
        box = np.array([0.0, 0.0, 0.0, box_L, box_L, box_L])
    else:
        box = np.concatenate([pos.min(0), pos.max(0)])
    ids = [np.flatnonzero(~group), np.flatnonzero(group)]
    trees = [build_tree(pos[i], mass[i], box_L, bucket, box) for i in ids]
    t0, t1 = trees
    nc0, np0 = t0.n_cell, ids[0].size
    ch1 = t1.child.copy()
    ch1[ch1 >= 0] += nc0
    return Tree(np.concatenate([ids[0][t0.perm], ids[1][t1.perm]]),
                np.concatenate([t0.cell_first, t1.cell_first + np0]),
                np.concatenate([t0.cell_count, t1.cell_count]),
                np.concatenate([t0.child, ch1]), np.concatenate([t0.com, t1.com]),
                np.concatenate([t0.bmax, t1.bmax]), np.concatenate([t0.bbox, t1.bbox]),
                np.concatenate([t0.mom, t1.mom]),
                np.concatenate([t0.bucket_cell, t1.bucket_cell + nc0]).astype(np.int32),
                float(box_L), int(bucket), (0, nc0))


def build_lists(tree: Tree, theta: float, eps: float, n_images: Optional[int] = None,
                sinks: Optional[np.ndarray] = None) -> Lists:
    """Checklist walk of Sec. 3.1 for every bucket of the tree (or for the
    buckets with indices ``sinks``, whose lists then come in that order),
    seeded with the tree's roots."""
    L = tree.box_L
    if n_images is None:
        n_images = 27 if L > 0 else 1
    bc = tree.bucket_cell if sinks is None else \
        np.ascontiguousarray(tree.bucket_cell[np.asarray(sinks)], dtype=np.int32)
    nb = bc.shape[0]
    roots = np.ascontiguousarray(tree.roots, dtype=np.int32)
    pp_off = np.zeros(nb + 1, np.int64)
    pc_off = np.zeros(nb + 1, np.int64)
    args = (nb, _p(bc), _p(tree.child), _p(tree.com), _p(tree.bmax),
            _p(tree.bbox), float(theta), float(eps), float(L), int(n_images), roots.size,
            _p(roots))
    lib().orc_lists_count_roots(*args, _p(pp_off), _p(pc_off))
    pp_src = np.empty(int(pp_off[-1]), np.int32)
    pp_img = np.empty(int(pp_off[-1]), np.uint8)
    pc_src = np.empty(int(pc_off[-1]), np.int32)
    pc_img = np.empty(int(pc_off[-1]), np.uint8)
    lib().orc_lists_fill_roots(*args, _p(pp_off), _p(pc_off), _p(pp_src), _p(pp_img),
                               _p(pc_src), _p(pc_img))
    return Lists(pp_off, pp_src, pp_img, pc_off, pc_src, pc_img, int(n_images))


PART_PP, PART_PC, PART_EWALD = 1, 2, 4


def evaluate(tree: Tree, lists: Lists, pos_tree: np.ndarray, mass_tree: np.ndarray,
             eps: float, parts: int = 7, buckets: Optional[np.ndarray] = None,
             ewald: Optional[dict] = None):
    """Accelerations [n,3] and potentials [n] (tree order) of the particles
    in ``buckets`` (all if None; others are returned as zero)."""
    ew = dict(EXACT_EWALD if ewald is None else ewald)
    pos_tree = np.ascontiguousarray(pos_tree, dtype=np.float64)
    mass_tree = np.ascontiguousarray(mass_tree, dtype=np.float64)
    n = pos_tree.shape[0]
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    sel = None if buckets is None else np.ascontiguousarray(buckets, dtype=np.int32)
    lib().orc_eval(n, _p(pos_tree), _p(mass_tree), float(eps), float(tree.box_L),
                   _p(tree.cell_first), _p(tree.cell_count), _p(tree.com), _p(tree.mom),
                   tree.n_bucket, _p(tree.bucket_cell), _p(lists.pp_off), _p(lists.pp_src),
                   _p(lists.pp_img), _p(lists.pc_off), _p(lists.pc_src), _p(lists.pc_img),
                   0 if sel is None else sel.shape[0], _p(sel), int(parts),
                   float(ew["alpha"]), int(ew["rmax"]), int(ew["h2max"]), _p(acc), _p(pot))
    return acc, pot


@dataclasses.dataclass
class FmmLists:
    """Lists of the fast-multipole walk: per bucket PP entries (source
    leaf, image, sub = 0 for the whole leaf or k + 1 for its k-th
    particle) and PC entries; per cell CC / CP entries (source cell, or ~p
    for tree-order particle p) whose expansions go into the cell's local
    expansion."""

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


def build_fmm_lists(tree: Tree, pos_tree: np.ndarray, theta: float, eps: float,
                    n_images: Optional[int] = None) -> FmmLists:
    """The sink-cell walk with CC and CP interactions (Sec. 3.1)."""
    L = tree.box_L
    if n_images is None:
        n_images = 27 if L > 0 else 1
    pos_tree = np.ascontiguousarray(pos_tree, dtype=np.float64)
    nb, nc = tree.n_bucket, tree.n_cell
    pp_off = np.zeros(nb + 1, np.int64)
    pc_off = np.zeros(nb + 1, np.int64)
    cc_off = np.zeros(nc + 1, np.int64)
    head = (nc, _p(tree.cell_first), _p(tree.cell_count), _p(tree.child), _p(tree.com),
            _p(tree.bmax), _p(tree.bbox), _p(pos_tree), float(theta), float(eps), float(L),
            int(n_images))
    lib().orc_fmm_walk(*head, 0, _p(pp_off), None, None, None, _p(pc_off), None, None,
                       _p(cc_off), None, None)
    out = dict(pp_src=np.empty(pp_off[-1], np.int32), pp_img=np.empty(pp_off[-1], np.uint8),
               pp_sub=np.empty(pp_off[-1], np.uint8), pc_src=np.empty(pc_off[-1], np.int32),
               pc_img=np.empty(pc_off[-1], np.uint8), cc_src=np.empty(cc_off[-1], np.int32),
               cc_img=np.empty(cc_off[-1], np.uint8))
    lib().orc_fmm_walk(*head, 1, _p(pp_off), _p(out["pp_src"]), _p(out["pp_img"]),
                       _p(out["pp_sub"]), _p(pc_off), _p(out["pc_src"]), _p(out["pc_img"]),
                       _p(cc_off), _p(out["cc_src"]), _p(out["cc_img"]))
    return FmmLists(pp_off, out["pp_src"], out["pp_img"], out["pp_sub"], pc_off, out["pc_src"],
                    out["pc_img"], cc_off, out["cc_src"], out["cc_img"], int(n_images))


def fmm_local(tree: Tree, fl: FmmLists, pos_tree: np.ndarray, mass_tree: np.ndarray,
              eps: float) -> np.ndarray:
    """Local expansion of every cell: [n_cell, 364], the full tensors of
    orders 0..5 of d^a phi at the cell's centre of mass."""
    pos_tree = np.ascontiguousarray(pos_tree, dtype=np.float64)
    mass_tree = np.ascontiguousarray(mass_tree, dtype=np.float64)
    out = np.empty((tree.n_cell, 364))
    lib().orc_fmm_local(tree.n_cell, _p(tree.child), _p(tree.com), _p(tree.mom), _p(pos_tree),
                        _p(mass_tree), float(eps), float(tree.box_L), _p(fl.cc_off),
                        _p(fl.cc_src), _p(fl.cc_img), _p(out))
    return out


def fmm_evaluate(tree: Tree, fl: FmmLists, pos_tree: np.ndarray, mass_tree: np.ndarray,
                 eps: float, parts: int = 7, local: Optional[np.ndarray] = None,
                 ewald: Optional[dict] = None):
    """Accelerations and potentials (tree order) from the FMM lists: PP and
    PC of each bucket (bits 1, 2), the Ewald correction (bit 4) and, with
    bit 8, the buckets' local expansions evaluated at their particles."""
    ew = dict(EXACT_EWALD if ewald is None else ewald)
    pos_tree = np.ascontiguousarray(pos_tree, dtype=np.float64)
    mass_tree = np.ascontiguousarray(mass_tree, dtype=np.float64)
    n = pos_tree.shape[0]
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    if parts & 7:
        lib().orc_eval_sub(n, _p(pos_tree), _p(mass_tree), float(eps), float(tree.box_L),
                           _p(tree.cell_first), _p(tree.cell_count), _p(tree.com), _p(tree.mom),
                           tree.n_bucket, _p(tree.bucket_cell), _p(fl.pp_off), _p(fl.pp_src),
                           _p(fl.pp_img), _p(fl.pp_sub), _p(fl.pc_off), _p(fl.pc_src),
                           _p(fl.pc_img), 0, None, int(parts & 7), float(ew["alpha"]),
                           int(ew["rmax"]), int(ew["h2max"]), _p(acc), _p(pot))
    if parts & 8:
        if local is None:
            local = fmm_local(tree, fl, pos_tree, mass_tree, eps)
        a2, p2 = np.zeros((n, 3)), np.zeros(n)
        lib().orc_fmm_l2p(tree.n_bucket, _p(tree.bucket_cell), _p(tree.cell_first),
                          _p(tree.cell_count), _p(tree.com), _p(pos_tree),
                          _p(np.ascontiguousarray(local)), _p(a2), _p(p2))
        acc += a2
        pot += p2
    return acc, pot


def fmm_m2l_point(mom32, mass: float, part: bool, XS, XC, eps: float) -> np.ndarray:
    out = np.empty(364)
    m = np.ascontiguousarray(mom32 if mom32 is not None else np.zeros(32), dtype=np.float64)
    lib().orc_fmm_m2l_point(_p(m), float(mass), int(part), _p(np.asarray(XS, np.float64)),
                            _p(np.asarray(XC, np.float64)), float(eps), _p(out))
    return out


def fmm_l2l_point(L364, d) -> np.ndarray:
    out = np.empty(364)
    lib().orc_fmm_l2l_point(_p(np.ascontiguousarray(L364, np.float64)),
                            _p(np.asarray(d, np.float64)), _p(out))
    return out


def fmm_l2p_point(L364, h) -> np.ndarray:
    out = np.empty(4)
    lib().orc_fmm_l2p_point(_p(np.ascontiguousarray(L364, np.float64)),
                            _p(np.asarray(h, np.float64)), _p(out))
    return out


def direct_open(pos: np.ndarray, mass: np.ndarray, eps: float):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[0]
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    lib().orc_direct_open(n, _p(pos), _p(mass), float(eps), _p(acc), _p(pot))
    return acc, pot


def direct_periodic(pos: np.ndarray, mass: np.ndarray, eps: float, L: float,
                    ewald: Optional[dict] = None):
    ew = dict(CONVERGED_EWALD if ewald is None else ewald)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[0]
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    lib().orc_direct_periodic(n, _p(pos), _p(mass), float(eps), float(L), float(ew["alpha"]),
                              int(ew["rmax"]), int(ew["h2max"]), _p(acc), _p(pot))
    return acc, pot


def ewald_derivs(r, alpha: float, rmax: int, h2max: int, kmax: int = 5):
    """Derivative tensors of the unit-box Ewald kernel psi at r:
    list of arrays of shape (3,)*k for k = 0..kmax."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    out = np.zeros(sum(3 ** k for k in range(kmax + 1)))
    lib().orc_ewald_derivs(_p(r), float(alpha), int(rmax), int(h2max), int(kmax), _p(out))
    res, off = [], 0
    for k in range(kmax + 1):
        res.append(out[off:off + 3 ** k].reshape((3,) * k) if k else out[off])
        off += 3 ** k
    return res


def set_quadrature(npts: int) -> None:
    lib().orc_set_quadrature(int(npts))


def moments(pos: np.ndarray, mass: np.ndarray):
    """Centre of mass and packed moments (32) of a point set."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    com = np.zeros(3)
    mom = np.zeros(32)
    lib().orc_moments(pos.shape[0], _p(pos), _p(mass), _p(com), _p(mom))
    return com, mom


def pc_point(mom32: np.ndarray, com: np.ndarray, x: np.ndarray, eps: float) -> np.ndarray:
    """(ax, ay, az, phi) at x from one cell's multipole expansion."""
    out = np.zeros(4)
    lib().orc_pc_point(_p(np.ascontiguousarray(mom32, dtype=np.float64)),
                       _p(np.ascontiguousarray(com, dtype=np.float64)),
                       _p(np.ascontiguousarray(x, dtype=np.float64)), float(eps), _p(out))
    return out


def ewald_root_point(mom32, com, x, L: float, alpha: float, rmax: int, h2max: int):
    out = np.zeros(4)
    lib().orc_ewald_root_point(_p(np.ascontiguousarray(mom32, dtype=np.float64)),
                               _p(np.ascontiguousarray(com, dtype=np.float64)),
                               _p(np.ascontiguousarray(x, dtype=np.float64)), float(L),
                               float(alpha), int(rmax), int(h2max), _p(out))
    return out


def forces(ps, theta: float = 0.7, bucket: int = 16, parts: int = 7, buckets=None,
           ewald: Optional[dict] = None):
    """Whole pipeline for a ParticleSet: tree, lists, evaluation.
    Returns (tree, lists, acc, pot) with acc/pot in tree order."""
    tree = build_tree(ps.pos, ps.mass, ps.box_L, bucket)
    lists = build_lists(tree, theta, ps.eps)
    pos_t = ps.pos[tree.perm]
    mass_t = ps.mass[tree.perm]
    acc, pot = evaluate(tree, lists, pos_t, mass_t, ps.eps, parts, buckets, ewald)
    return tree, lists, acc, pot
