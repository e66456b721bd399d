"""The allocation-free bind (mgrav_bind_static): the library's static
per-GPU workspace in place of a caller buffer.  Its computes must equal
those of mgrav_bind with a workspace, bit for bit (same kernels, same
order of arithmetic), on two binds in a row, the second with a smaller
problem; a problem larger than the static workspace is refused on the host."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

try:  # imported at collection so its one-off start-up cost is not a test's
    import torch
except ImportError:  # pragma: no cover
    torch = None

pytestmark = pytest.mark.gpu


def _case(msg):
    print(f"\n[gpu case] {msg}", flush=True)


def _problem(ctx, ps):
    tree = oracle.build_tree(ps.pos, ps.mass, ps.box_L, 16)
    lists = oracle.build_lists(tree, 0.7, ps.eps)
    return ctx.upload(ps.pos[tree.perm], ps.mass[tree.perm], tree, lists, ps.eps, 0.7)


def _run(mg, ctx, n):
    acc, pot = ctx.outputs()
    ctx.compute(acc, pot)
    st = ctx.wait(120)
    return acc.cpu().numpy().reshape(3, -1).T.copy(), pot.cpu().numpy().copy(), st


def test_static_bind_equals_workspace_bind():
    if torch is None or not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_08621_amd as mg
    ref = mg.Context(0)
    stat = mg.Context(0)
    try:
        stat.set_launch_mode(mg.LAUNCH_DIRECT)
        sets = [("lattice_48", workloads.perturbed_lattice(48, 0.2, seed=61)),
                ("clustered_16", workloads.make(3, scale_n1d=16))]
        for label, ps in sets:
            _case(f"static bind {label} n={ps.n}: workspace bind, then static bind")
            tensors, p = _problem(ref, ps)
            assert ref.workspace_size(p) <= mg.STATIC_WORKSPACE_BYTES
            ref.bind(p, tensors)
            a_ref, p_ref, st_ref = _run(mg, ref, ps.n)
            stat.bind_static(p, tensors)
            a_s, p_s, st_s = _run(mg, stat, ps.n)
            print(f"  pp={st_s.n_pp_interactions} pc={st_s.n_pc_interactions} "
                  f"graph={st_s.graph_replay} max|da|={np.abs(a_s - a_ref).max():.3e}", flush=True)
            assert st_s.graph_replay == 0
            assert st_s.n_pp_interactions == st_ref.n_pp_interactions
            assert st_s.n_pc_interactions == st_ref.n_pc_interactions
            assert np.all(np.isfinite(a_s))
            assert np.array_equal(a_s, a_ref) and np.array_equal(p_s, p_ref)
            # a second compute on the same static bind gives the same again
            a_2, p_2, _ = _run(mg, stat, ps.n)
            assert np.array_equal(a_2, a_ref) and np.array_equal(p_2, p_ref)

        _case("static bind: a problem larger than the static workspace is refused on the host")
        big = mg.Problem.from_buffer_copy(p)
        big.n_pp = 8_000_000  # 128 MB of staged PP entries alone
        with pytest.raises(mg.MgravError) as e:
            stat.bind_static(big, tensors)
        assert e.value.status == mg.ERR_NO_MEMORY
        assert "static scratch" in str(e.value)
        # the refused bind changed nothing: the previous binding still computes
        a_3, p_3, _ = _run(mg, stat, ps.n)
        assert np.array_equal(a_3, a_ref) and np.array_equal(p_3, p_ref)
    finally:
        stat.close()
        ref.close()
