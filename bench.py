#!/usr/bin/env python3
"""Throughput of the gravity hot path on one MI355X.

One step = one pass of the whole device path over the bound workload:
staging of particles, cells and lists (mgrav_bind) followed by the PP + PC
evaluation and the Ewald correction (mgrav_compute), with inputs already
resident in HBM.  The default workload is one GPU's share of the
individual-time-step run: 512^3 clustered particles in a periodic box
(theta 0.7, buckets of 16), substeps with 100 %, 10 % and 1 % of them
active, the learned Ewald correction judged by exact Ewald; the line's
value is the 100 % step.  ``--config 1..4`` runs one of the smaller
workloads with every particle active.

Prints one JSON line.  The metric is PP + PC interactions per second;
``roofline`` covers the PP + PC kernel (FP32 vector ALU); ``cpu_baseline``
times the FP64 oracle on a bounded sample of the same buckets.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic FLOPs per interaction of the device kernels (hardware count:
# fused multiply-add = 2, reciprocal square root = 1).
FLOP_PP = 20
FLOP_PC = 240
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak (packed)
PEAK_FP32_NONPACKED = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz
PEAK_FP64_TFLOPS = 78.6      # MI355X published FP64 vector peak


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=5,
                    help="5 (default): the 512^3 clustered substeps; 1-4: one workload, all "
                         "active")
    ap.add_argument("--cpu-stride", type=int, default=1,
                    help="oracle baseline evaluates every k-th bucket")
    ap.add_argument("--cpu-buckets", type=int, default=16384,
                    help="config 5: about this many sink buckets in the oracle's sample")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle (CPU baseline; config 5: the sampled parity)")
    ap.add_argument("--no-fmm", action="store_true",
                    help="config 5: skip the fast-multipole leg (128^3 clustered set)")
    ap.add_argument("--no-kdk", action="store_true",
                    help="config 5: skip the integrator leg (one timed KDK base step)")
    ap.add_argument("--kdk-rungs", type=int, default=3)
    ap.add_argument("--no-queue-study", action="store_true",
                    help="skip the leg that times the work-queue layouts against each other")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep PP + PC kernel variant 0 instead of timing all variants first")
    ap.add_argument("--ewald-study", action="store_true",
                    help="instead of the throughput line: exact vs learned Ewald correction, "
                         "time against force error, on the chosen config (default 4)")
    ap.add_argument("--fmm-only", action="store_true",
                    help="instead of the throughput line: only the fast-multipole leg "
                         "(128^3 clustered set, against the bucket walk), as one JSON line")
    ap.add_argument("--train-samples", type=int, default=2_000_000)
    ap.add_argument("--train-epochs", type=int, default=30)
    ap.add_argument("--substep-ewald", choices=("fallback", "exact"), default="fallback",
                    help="config 5: learned Ewald correction judged by exact Ewald on a "
                         "sample, exact where it fails (default), or exact throughout")
    ap.add_argument("--fallback-tol", type=float, default=1e-4,
                    help="config 5: largest accepted sample error of the learned correction "
                         "(rms force error relative to the rms total force)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (reference "
                         "for the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); multi-GPU "
              "sharding of the bucket lists is described in the design notes, not built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1609_08621_amd as mg
    import workloads

    if args.ewald_study:
        ewald_study(args)
        return
    if args.fmm_only:
        ctx = mg.Context(0)
        print(json.dumps({"fmm": fmm_leg(ctx, args)}), flush=True)
        ctx.close()
        return
    if args.config == 5:
        substeps(args)
        return
    cfg = workloads.CONFIGS[args.config]
    ps = workloads.make(args.config)
    t0 = time.perf_counter()
    tree = mg.tree_build(ps.pos, ps.mass, ps.box_L, cfg.bucket)
    lists = mg.lists_build(tree, cfg.theta, ps.eps)
    prep_s = time.perf_counter() - t0
    pos_t, mass_t = ps.pos[tree.perm], ps.mass[tree.perm]
    print(f"[bench] {cfg.name}: n={ps.n} cells={tree.n_cell} buckets={tree.n_bucket} "
          f"pp_entries={lists.pp_src.size} pc_entries={lists.pc_src.size} "
          f"host prep {prep_s:.2f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    if args.calibrate_copy_mib > 0:
        nbytes = args.calibrate_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {args.calibrate_copy_mib} MiB done", file=sys.stderr,
              flush=True)
        del src, dst
    ctx = mg.Context(0)
    tensors, prob = ctx.upload(pos_t, mass_t, tree, lists, ps.eps, cfg.theta)
    ws = torch.empty(ctx.workspace_size(prob), dtype=torch.uint8, device=dev)
    acc = torch.zeros(3 * ps.n, dtype=torch.float32, device=dev)
    pot = torch.zeros(ps.n, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    # untimed set-up: pick the PP + PC kernel variant for these lists
    variants = mg.interact_variants()
    tuned = {"index": 0, "ms_per_variant": None}
    if not args.no_autotune:
        ctx.bind(prob, tensors, ws)
        v, ms = ctx.autotune(acc, pot, budget_ms=1500.0)
        tuned = {"index": v, "ms_per_variant": ms}
    tuned["pp_chunk"], tuned["waves_per_simd"], tuned["pc_prefetch"] = variants[tuned["index"]]
    print(f"[bench] PP + PC kernel variant {tuned}", file=sys.stderr, flush=True)

    def enqueue():
        # one step: re-stage the (moved) positions and compute every part
        ctx.bind(prob, tensors, ws)
        ctx.compute(acc, pot)

    def step():
        enqueue()
        return ctx.wait(60.0)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # throughput: the K steps are enqueued back to back on the stream, as a
    # GPU-resident integrator would; the host waits (and the library checks
    # the error bits) once, after the last step
    t0 = time.perf_counter()
    for _ in range(args.steps):
        enqueue()
    st = ctx.wait(60.0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    # kernel durations: the same K steps again, each waited for, reading the
    # HIP events recorded around each phase on the context's stream
    ms_k, ms_e, ms_c = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step()
        ms_k.append(st.ms_interact)
        ms_e.append(st.ms_ewald)
        ms_c.append(st.ms_total)
    torch.cuda.synchronize()
    ms_step_sync = 1e3 * (time.perf_counter() - t0) / args.steps
    tuned["launch"] = "graph" if st.graph_replay else "direct"
    n_int = st.n_pp_interactions + st.n_pc_interactions
    value = n_int / (ms_step * 1e-3)
    flops = st.n_pp_interactions * FLOP_PP + st.n_pc_interactions * FLOP_PC
    k_ms = float(np.mean(ms_k))
    achieved = flops / (k_ms * 1e-3) / 1e12
    k_ms_alone = k_ms
    if tuned["launch"] == "direct" and cfg.ewald == "exact":
        # direct launches run the exact Ewald correction beside the PP + PC
        # kernel, which then shares the GPU; its duration alone comes from
        # the graph launch, where the phases run one after the other
        ctx.set_launch_mode(mg.LAUNCH_GRAPH)
        step()
        ms_alone = [step().ms_interact for _ in range(min(args.steps, 20))]
        ctx.set_launch_mode(mg.LAUNCH_DIRECT)
        k_ms_alone = float(np.mean(ms_alone))
    print(f"[bench] step {ms_step:.3f} ms back to back, {ms_step_sync:.3f} ms with a host wait "
          f"per step (compute {np.mean(ms_c):.3f} ms: PP+PC kernel "
          f"{k_ms:.3f} ms, Ewald {np.mean(ms_e):.3f} ms), {value:.3e} interactions/s, "
          f"kernel {achieved:.1f} TFLOP/s", file=sys.stderr, flush=True)

    out = {
        "metric": "P-P+P-C interactions/s",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name} (n={ps.n}, theta={cfg.theta}, bucket={cfg.bucket}, "
                        f"eps={ps.eps:.6g}, Ewald {cfg.ewald}: alpha 2.6, 27 images, |h|^2<=10)",
            "n": ps.n, "theta": cfg.theta, "bucket": cfg.bucket,
            "parallelism": "single GPU",
        },
        "interact_variant": tuned,
        "particles_per_s": ps.n / (ms_step * 1e-3),
        "n_pp_interactions": st.n_pp_interactions,
        "n_pc_interactions": st.n_pc_interactions,
        "ms_per_step_with_host_wait": ms_step_sync,
        "ms_compute": float(np.mean(ms_c)),
        "ms_interact_kernel": k_ms,
        "ms_ewald": float(np.mean(ms_e)),
        "roofline": {
            "bound": "alu",
            "kernel": f"k_interact<{tuned['pp_chunk']}, {tuned['waves_per_simd']}, "
                      f"{'true' if tuned['pc_prefetch'] else 'false'}> "
                      "(PP + PC, FP32 vector ALU)",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "frac_of_nonpacked_peak": achieved / PEAK_FP32_NONPACKED,
            "kernel_ms": k_ms,
            "achieved_alone": flops / (k_ms_alone * 1e-3) / 1e12,
            "frac_alone": flops / (k_ms_alone * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
            "kernel_ms_alone": k_ms_alone,
            "alone_note": "achieved/frac: the kernel's mean duration in the timed steps, where "
                          "direct launches run the exact Ewald correction beside it; *_alone: "
                          "the same kernel with the phases in sequence (graph launch)",
            "flop_per_pp": FLOP_PP,
            "flop_per_pc": FLOP_PC,
            "traffic": None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                            "copy-calibrated)",
        },
    }

    detail = interact_traffic(cfg.name, tuned["pp_chunk"], tuned["waves_per_simd"],
                              tuned["pc_prefetch"])
    if detail is not None:
        out["roofline"]["traffic"] = detail.pop("bytes_per_launch")
        out["roofline"]["traffic_detail"] = detail
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, ps, cfg, tree, pos_t, mass_t, acc, pot)
    ctx.close()
    print(json.dumps(out), flush=True)


def counters_file(workload: str) -> str:
    """The committed counter summary of the PP + PC kernel on a workload
    (profiles/k_interact_<workload without _periodic>_counters.json)."""
    short = workload[:-len("_periodic")] if workload.endswith("_periodic") else workload
    return os.path.join(ROOT, "profiles", f"k_interact_{short}_counters.json")


def interact_source_digest() -> str:
    """Digest of the interact kernel's source (from ``struct RunArgs`` to
    the Ewald section of mgrav.hip): counters taken on other code are stale."""
    with open(os.path.join(ROOT, "paper_1609_08621_amd", "csrc", "mgrav.hip")) as f:
        src = f.read()
    a, b = src.index("struct RunArgs {"), src.index("// Ewald correction (FP64)")
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def ewald_source_digest() -> str:
    """Digest of the exact Ewald kernels' source (from the Ewald section of
    mgrav.hip to the surrogate's): a FLOP count taken on other code is stale."""
    with open(os.path.join(ROOT, "paper_1609_08621_amd", "csrc", "mgrav.hip")) as f:
        src = f.read()
    a = src.index("// Ewald correction (FP64)")
    b = src.index("k_ewald_judge", a)
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def ewald_flops_per_particle(workload: str):
    """FP64 FLOP per particle of the exact Ewald kernel on a workload, from
    the committed rocprofv3 summary (SQ_INSTS_VALU_FLOPS_FP64 of the
    dispatches over every particle, divided by their count), or None."""
    short = workload[:-len("_periodic")] if workload.endswith("_periodic") else workload
    path = os.path.join(ROOT, "profiles", f"k_ewald_{short}_counters.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("workload") != workload or rec.get("source_digest") != ewald_source_digest():
        return None
    return {"flop_per_particle": rec["flop_per_particle"], "source": os.path.relpath(path, ROOT)}


def interact_traffic(workload: str, pp_chunk: int, waves: int, prefetch: int):
    """HBM bytes per launch of the k_interact variant (pp_chunk, waves,
    prefetch) from
    the committed rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE,
    scaled by a copy of known size), or None when the summary is missing,
    for another workload or variant, or taken on different kernel source."""
    path = counters_file(workload)
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("workload") != workload or rec.get("source_digest") != interact_source_digest():
        return None
    key = f"{pp_chunk}x{waves}x{'true' if prefetch else 'false'}"
    var = rec.get("variants", {}).get(key)
    if var is None:
        return None
    return {"bytes_per_launch": var["traffic_bytes_per_launch"],
            "fetch_kib_raw": var["fetch_kib_per_dispatch"],
            "write_kib_raw": var["write_kib_per_dispatch"],
            "fetch_factor": rec["fetch_factor"], "write_factor": rec["write_factor"],
            "variant": key, "source": os.path.relpath(path, ROOT)}


def cpu_baseline(args, ps, cfg, tree, pos_t, mass_t, acc_dev, pot_dev):
    """The FP64 oracle, as it stands, on every k-th bucket of the same
    workload: interactions/s over that sample, plus the GPU's error there."""
    import numpy as np

    import oracle
    to = oracle.build_tree(ps.pos, ps.mass, ps.box_L, cfg.bucket)
    lo = oracle.build_lists(to, cfg.theta, ps.eps)
    sel = np.arange(0, to.n_bucket, args.cpu_stride, dtype=np.int32)
    cnt = to.cell_count
    nsink = cnt[to.bucket_cell[sel]].astype(np.int64)
    pp_src_count = np.array([cnt[lo.pp_src[lo.pp_off[b]:lo.pp_off[b + 1]]].sum() for b in sel])
    npc = (lo.pc_off[sel + 1] - lo.pc_off[sel])
    n_int = int((nsink * pp_src_count).sum() + (nsink * npc).sum())
    print(f"[bench] cpu baseline: oracle on {sel.size} of {to.n_bucket} buckets "
          f"({oracle.num_threads()} threads)", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ao, po = oracle.evaluate(to, lo, pos_t, mass_t, ps.eps, 7, buckets=sel)
    dt = time.perf_counter() - t0
    idx = np.concatenate([np.arange(to.cell_first[c], to.cell_first[c] + to.cell_count[c])
                          for c in to.bucket_cell[sel]])
    ag = acc_dev.cpu().numpy().reshape(3, -1).T[idx]
    a_ref = ao[idx]
    err = float(np.sqrt(np.mean(np.sum((ag - a_ref) ** 2, 1) / np.sum(a_ref ** 2, 1))))
    pg = pot_dev.cpu().numpy()[idx]
    # the periodic total potential is a small residual of the PP + PC part
    # and the Ewald correction, so the potential error is taken relative to
    # the PP + PC part (total minus the oracle's correction; untimed)
    _, pe = oracle.evaluate(to, lo, pos_t, mass_t, ps.eps, 4, buckets=sel)
    tree_part = po[idx] - pe[idx]
    perr = float(np.sqrt(np.sum((pg - po[idx]) ** 2) / np.sum(tree_part ** 2)))
    return {
        "value": n_int / dt,
        "unit": "interactions/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (("every sink bucket" if args.cpu_stride == 1 else
                    f"every {args.cpu_stride}th sink bucket") +
                   f" ({sel.size} of {to.n_bucket}, {idx.size} particles, {n_int} PP+PC "
                   f"interactions plus their Ewald corrections, one step of the workload) "
                   f"in {dt:.1f} s"),
        "seconds": dt,
        "gpu_rms_rel_acc_err_vs_oracle": err,
        "gpu_rel_pot_err_vs_oracle": perr,
        "pot_err_normalisation": "rms of the oracle's PP + PC potential",
    }


def sample_problem(tree, lists, stride):
    """Every ``stride``-th sink bucket of a tree and its lists, as a tree
    and lists of those buckets only (CSR re-based), for the oracle."""
    import numpy as np

    import oracle
    sel = np.arange(0, tree.n_bucket, stride, dtype=np.int64)

    def sub(off, *cols):
        lo, hi = off[sel], off[sel + 1]
        new_off = np.zeros(sel.size + 1, np.int64)
        np.cumsum(hi - lo, out=new_off[1:])
        take = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)]) if sel.size else \
            np.zeros(0, np.int64)
        return (new_off,) + tuple(np.ascontiguousarray(c[take]) for c in cols)

    pp_off, pp_src, pp_img = sub(lists.pp_off, lists.pp_src, lists.pp_img)
    pc_off, pc_src, pc_img = sub(lists.pc_off, lists.pc_src, lists.pc_img)
    lo = oracle.Lists(pp_off, pp_src, pp_img, pc_off, pc_src, pc_img, lists.n_images)
    to = oracle.Tree(tree.perm, tree.cell_first, tree.cell_count, tree.child, tree.com,
                     tree.bmax, tree.bbox, tree.mom,
                     np.ascontiguousarray(tree.bucket_cell[sel]), tree.box_L, 16)
    idx = np.concatenate([np.arange(tree.cell_first[c], tree.cell_first[c] + tree.cell_count[c])
                          for c in to.bucket_cell])
    nsink = tree.cell_count[to.bucket_cell].astype(np.int64)
    cs = np.zeros(pp_src.size + 1, np.int64)
    np.cumsum(tree.cell_count[pp_src], out=cs[1:])
    n_pp = int((nsink * (cs[pp_off[1:]] - cs[pp_off[:-1]])).sum())
    n_pc = int((nsink * np.diff(pc_off)).sum())
    return to, lo, sel, idx, n_pp + n_pc


def sample_problem_device(dtree, dlists, stride):
    """As sample_problem, from a tree and lists in device memory: the tree
    and the sampled buckets' list entries are copied to the host."""
    import numpy as np
    import torch

    import oracle
    th = dtree.to_host()
    sel = np.arange(0, th.n_bucket, stride, dtype=np.int64)
    pp_off = dlists.pp_off.cpu().numpy()
    pc_off = dlists.pc_off.cpu().numpy()

    def sub(off, src, img):
        lo, hi = off[sel], off[sel + 1]
        new_off = np.zeros(sel.size + 1, np.int64)
        np.cumsum(hi - lo, out=new_off[1:])
        take = torch.from_numpy(np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)]))
        take = take.to(src.device)
        return new_off, src.index_select(0, take).cpu().numpy(), \
            img.index_select(0, take).cpu().numpy()

    sp_off, pps, ppi = sub(pp_off, dlists.pp_src, dlists.pp_img)
    sc_off, pcs, pci = sub(pc_off, dlists.pc_src, dlists.pc_img)
    lo = oracle.Lists(sp_off, pps, ppi, sc_off, pcs, pci, dlists.n_images)
    to = oracle.Tree(th.perm, th.cell_first, th.cell_count, th.child, th.com, th.bmax, th.bbox,
                     th.mom, np.ascontiguousarray(th.bucket_cell[sel]), th.box_L, 16)
    idx = np.concatenate([np.arange(th.cell_first[c], th.cell_first[c] + th.cell_count[c])
                          for c in to.bucket_cell])
    nsink = th.cell_count[to.bucket_cell].astype(np.int64)
    cs = np.zeros(pps.size + 1, np.int64)
    np.cumsum(th.cell_count[pps], out=cs[1:])
    n_pp = int((nsink * (cs[sp_off[1:]] - cs[sp_off[:-1]])).sum())
    n_pc = int((nsink * np.diff(sc_off)).sum())
    return to, lo, sel, idx, n_pp + n_pc


def substeps(args):
    """The headline: individual time steps at one GPU's share, the 512^3
    clustered set (134 217 728 particles), forces for the active particles
    of substeps touching 100 %, 10 % and 1 % of them (the largest |a|, from
    a first full force computation).  A step is bind + compute with the
    substep's mask, inputs resident in HBM; the Ewald correction is the
    learned one judged by exact Ewald on a sample, exact where the judge
    rejects it.  The line's value is the 100 % step; the others are extra
    keys.  Prints one JSON line."""
    import numpy as np
    import torch

    import paper_1609_08621_amd as mg
    import workloads

    cfg = workloads.CONFIGS[5]
    t_all = time.perf_counter()
    t0 = time.perf_counter()
    ps = workloads.make(5)
    log(f"{cfg.name}: n={ps.n} generated in {time.perf_counter() - t0:.1f}s")
    n, eps = ps.n, ps.eps
    m_uniform = float(ps.mass[0])
    dev = torch.device("cuda", 0)
    ctx = mg.Context(0)
    # positions on the 2^32 grid of the particle store (Sec. 3.4): every
    # leg below sees the same values, whether it reads the store's integers
    # or their decoded doubles
    store = ctx.store_alloc(n, (0.0, 0.0, 0.0), 1.0 / 2 ** 32)
    ctx.store_encode(store, torch.from_numpy(ps.pos).to(dev), None, True)
    pos_in = ctx.store_decode(store)
    mass_in = torch.from_numpy(ps.mass).to(dev)
    del ps
    torch.cuda.synchronize()
    # the tree and the lists, built on the device (untimed set-up of the
    # steps; their times are reported)
    prep = {}
    for rep in range(2):  # the second build is the timed one (the first loads code)
        t0 = time.perf_counter()
        tree = ctx.tree_build(pos_in, mass_in, 1.0, cfg.bucket)
        torch.cuda.synchronize()
        prep["tree_s"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        lists = ctx.lists_build(tree, cfg.theta, eps)
        torch.cuda.synchronize()
        prep["lists_s"] = time.perf_counter() - t0
        if rep == 0:
            del lists
    del mass_in
    del pos_in
    store = ctx.store_permute(store, tree.perm)
    n_cell, n_bucket = int(tree.cell_first.shape[0]), int(tree.bucket_cell.shape[0])
    log(f"device tree: {n_cell} cells, {n_bucket} buckets in {prep['tree_s']:.2f}s; lists: "
        f"{lists.pp_src.numel()} PP and {lists.pc_src.numel()} PC entries in "
        f"{prep['lists_s']:.2f}s")
    tensors, prob = ctx.problem_device(tree, lists, eps, cfg.theta)
    ws = torch.empty(ctx.workspace_size(prob), dtype=torch.uint8, device=dev)
    acc = torch.zeros(3 * n, dtype=torch.float32, device=dev)
    pot = torch.zeros(n, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    log(f"workspace {ws.numel() / 2**30:.1f} GiB")
    if args.calibrate_copy_mib > 0:
        # a plain device copy of known size: the reference of the HBM
        # traffic counters (FETCH_SIZE, WRITE_SIZE)
        src = torch.ones((args.calibrate_copy_mib << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calibrate_copy_mib} MiB done")
        del src, dst
    sample = None
    if not args.no_cpu_baseline:
        stride = max(1, n_bucket // args.cpu_buckets)
        sample = sample_problem_device(tree, lists, stride)
    pos_t = tree.pos.cpu().numpy() if sample is not None else None
    mass_t = tree.mass.cpu().numpy() if sample is not None else None
    ctx.bind(prob, tensors, ws)
    tuned = {"index": 0, "ms_per_variant": None}
    if not args.no_autotune:
        v, ms = ctx.autotune(acc, pot, budget_ms=3000.0)
        tuned = {"index": v, "ms_per_variant": ms}
    tuned["pp_chunk"], tuned["waves_per_simd"], tuned["pc_prefetch"] = \
        mg.interact_variants()[tuned["index"]]
    log(f"PP + PC kernel variant {tuned}")

    # the full force with exact Ewald: the active sets of the substeps come
    # from its |a|, and the oracle's sample is compared with it
    ctx.compute(acc, pot)
    ctx.wait(300.0)
    a_full = acc.view(3, -1).t().cpu().numpy().astype(np.float64)
    p_full = pot.cpu().numpy().astype(np.float64)
    amag = np.sqrt(np.sum(a_full ** 2, 1))
    a_sample = p_sample = None
    if sample is not None:
        a_sample, p_sample = a_full[sample[3]].copy(), p_full[sample[3]].copy()
    del a_full, p_full

    ew_cfg = dict(mode=mg.EWALD_EXACT)
    ewald_info = {"mode": "exact (alpha 2.6, 27 images, |h|^2<=10)"}
    if args.substep_ewald == "fallback":
        # the learned correction, trained on the library's own exact kernel,
        # judged on every compute by exact Ewald on a sample of particles
        t0 = time.perf_counter()
        u = torch.from_numpy(workloads.octant_points(args.train_samples)).to(dev)
        psi = ctx.ewald_psi(u, 2.6, 1, 10)
        psi0 = float(ctx.ewald_psi(torch.zeros((1, 3), dtype=torch.float64, device=dev), 2.6,
                                   1, 10).cpu()[0, 0])
        ctx.mlp_attach(8192)
        ctx.mlp_set_weights(workloads.mlp_init().astype(np.float32))
        losses = ctx.mlp_train(u, psi, epochs=args.train_epochs, batch=8192, lr=3e-3,
                               lr_min=3e-5, psi0=psi0)
        del u, psi
        train_s = time.perf_counter() - t0
        ew_cfg = dict(mode=mg.EWALD_SURROGATE_FALLBACK, top_cells=1,
                      fallback_tol=args.fallback_tol)
        ewald_info = {
            "mode": "learned (root monopole) with exact fallback",
            "fallback_tol": args.fallback_tol, "train_samples": args.train_samples,
            "train_epochs": args.train_epochs, "train_seconds": train_s,
            "final_loss": float(losses[-1])}
        log(f"learned Ewald: trained in {train_s:.1f}s, final loss {losses[-1]:.3e}")

    rows = []
    head = None
    for frac in (1.0, 0.1, 0.01):
        mask = None
        if frac < 1.0:
            mask = torch.from_numpy(workloads.active_by_acceleration(amag, frac)).to(dev)

        def enqueue(ew=ew_cfg):
            ctx.bind(prob, tensors, ws)
            ctx.set_ewald(**ew)
            ctx.set_active(mask)
            ctx.compute(acc, pot)

        def step(ew=ew_cfg):
            enqueue(ew)
            return ctx.wait(300.0)

        for _ in range(max(1, min(args.warmup, 3))):
            step()
        torch.cuda.synchronize()
        steps = args.steps if frac == 1.0 else max(1, min(args.steps, 10))
        # throughput: the steps enqueued back to back on the stream, the host
        # waiting once after the last
        t0 = time.perf_counter()
        for _ in range(steps):
            enqueue()
        st = ctx.wait(300.0)
        torch.cuda.synchronize()
        ms_step = 1e3 * (time.perf_counter() - t0) / steps
        # kernel spans: the same steps again, each waited for
        ms_k, ms_c, ms_e = [], [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            st = step()
            ms_k.append(st.ms_interact)
            ms_c.append(st.ms_total)
            ms_e.append(st.ms_ewald)
        ms_step_sync = 1e3 * (time.perf_counter() - t0) / steps
        ewald_row = {"ms_ewald": float(np.mean(ms_e))}
        if args.substep_ewald == "fallback":
            ewald_row.update(exact_path_taken=st.ewald_fallback,
                             sample_err=st.ewald_sample_err,
                             sampled_particles=st.ewald_samples)
            # the same substep with exact Ewald throughout, for comparison:
            # whole computes (the exact correction may run beside the PP + PC
            # kernel, so its own span is no measure of its cost)
            ms_x = [step(dict(mode=mg.EWALD_EXACT)).ms_total for _ in range(3)]
            ewald_row["ms_compute_with_exact_ewald"] = float(np.median(ms_x))
            ewald_row["ms_compute_with_learned_or_fallback"] = float(np.mean(ms_c))
        n_int = st.n_pp_interactions + st.n_pc_interactions
        flops = st.n_pp_interactions * FLOP_PP + st.n_pc_interactions * FLOP_PC
        k_ms = float(np.mean(ms_k))
        row = {"active_fraction": frac, "active_particles": st.n_active_particles,
               "active_buckets": st.n_active_buckets, "steps": steps, "ms_per_step": ms_step,
               "ms_per_step_with_host_wait": ms_step_sync,
               "ms_compute": float(np.mean(ms_c)), "ms_interact_kernel": k_ms,
               "n_pp_interactions": st.n_pp_interactions, "n_pc_interactions": st.n_pc_interactions,
               "interactions_per_s": n_int / (ms_step * 1e-3),
               "particles_per_s": st.n_active_particles / (ms_step * 1e-3),
               "kernel_tflops": flops / (k_ms * 1e-3) / 1e12, "ewald": ewald_row,
               "launch": "graph" if st.graph_replay else "direct",
               "queue_layout": "locality" if st.queue_local else "cost order"}
        rows.append(row)
        if head is None:
            head = (st, flops, k_ms, steps)
        log(f"active {frac:.0%}: {row['active_particles']} particles, step {ms_step:.2f} ms, "
            f"{row['interactions_per_s']:.3e} interactions/s, {row['particles_per_s']:.3e} "
            f"particles/s, kernel {row['kernel_tflops']:.1f} TFLOP/s, Ewald {ewald_row}")
    ctx.set_active(None)

    # the particle store (Sec. 3.4): the same substeps reading positions as
    # the store's 32-bit integers and equal masses without an array
    store_rows = []
    tensors_q, prob_q = ctx.problem_device(tree, lists, eps, cfg.theta)
    prob_q.pos, prob_q.pos_q, prob_q.q_scale = None, store.q.data_ptr(), store.scale
    prob_q.mass, prob_q.mass_uniform = None, m_uniform
    tensors_q["q"] = store.q
    for frac in (1.0, 0.01):
        mask = None if frac == 1.0 else torch.from_numpy(
            workloads.active_by_acceleration(amag, frac)).to(dev)
        ms = {}
        for label, (pr, te) in (("double", (prob, tensors)), ("store", (prob_q, tensors_q))):
            def qstep():
                ctx.bind(pr, te, ws)
                ctx.set_ewald(**ew_cfg)
                ctx.set_active(mask)
                ctx.compute(acc, pot)
                return ctx.wait(300.0)
            qstep()
            reps = 3 if frac == 1.0 else 5
            t0 = time.perf_counter()
            for _ in range(reps):
                qstep()
            ms[label] = 1e3 * (time.perf_counter() - t0) / reps
        store_rows.append({"active_fraction": frac, "ms_per_step_double_positions": ms["double"],
                           "ms_per_step_store_positions": ms["store"]})
        log(f"store: active {frac:.0%}: double positions {ms['double']:.2f} ms, store "
            f"{ms['store']:.2f} ms per step")
    ctx.set_active(None)
    del tensors_q, prob_q

    # layouts of the PP + PC kernel's work queue: cost order against
    # locality order (per-die segments in tree order); the kernel's span,
    # mean of 3 waited steps after one untimed
    queue_rows = []
    for frac in (() if args.no_queue_study else (1.0, 0.1, 0.01)):
        mask = None if frac == 1.0 else torch.from_numpy(
            workloads.active_by_acceleration(amag, frac)).to(dev)
        ms, used = {}, None
        for label, order in (("lpt", mg.QUEUE_LPT), ("local", mg.QUEUE_LOCAL),
                             ("auto", mg.QUEUE_AUTO)):
            ctx.set_queue_order(order)
            ks = []
            for rep in range(4):
                ctx.bind(prob, tensors, ws)
                ctx.set_ewald(**ew_cfg)
                ctx.set_active(mask)
                ctx.compute(acc, pot)
                st_q = ctx.wait(300.0)
                if rep:
                    ks.append(st_q.ms_interact)
            ms[label] = float(np.mean(ks))
            if order == mg.QUEUE_AUTO:
                used = "local" if st_q.queue_local else "lpt"
        queue_rows.append({"active_fraction": frac, "ms_interact_lpt": ms["lpt"],
                           "ms_interact_local": ms["local"], "ms_interact_auto": ms["auto"],
                           "auto_layout": used})
        log(f"queue order: active {frac:.0%}: kernel {ms['lpt']:.2f} ms (cost order), "
            f"{ms['local']:.2f} ms (locality), auto = {used}")
    ctx.set_queue_order(mg.QUEUE_AUTO)
    ctx.set_active(None)

    # the exact Ewald correction alone (every particle, FP64): the span of
    # its phase (k_ewald_setup + k_ewald), mean of 3 after one untimed
    ctx.bind(prob, tensors, ws)
    ctx.set_ewald(mode=mg.EWALD_EXACT)
    ew_ms = []
    for rep in range(4):
        ctx.compute(acc, pot, mg.PART_EWALD)
        st_e = ctx.wait(300.0)
        if rep:
            ew_ms.append(st_e.ms_ewald)
    ew_ms = float(np.mean(ew_ms))
    ew_flop = ewald_flops_per_particle(cfg.name)
    ewald_roof = {"bound": "alu", "kernel": "k_ewald_setup + k_ewald (FP64 vector ALU)",
                  "ms": ew_ms, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                  "achieved": None, "frac": None, "flop_per_particle": None}
    if ew_flop is not None:
        ach = ew_flop["flop_per_particle"] * n / (ew_ms * 1e-3) / 1e12
        ewald_roof.update(achieved=ach, frac=ach / PEAK_FP64_TFLOPS,
                          flop_per_particle=ew_flop["flop_per_particle"],
                          flop_source=ew_flop["source"])
    log(f"exact Ewald alone: {ew_ms:.2f} ms, {ewald_roof['achieved']} TFLOP/s FP64")

    st, flops, k_ms, steps = head
    achieved = flops / (k_ms * 1e-3) / 1e12
    kname = (f"k_interact<{tuned['pp_chunk']}, {tuned['waves_per_simd']}, "
             f"{'true' if tuned['pc_prefetch'] else 'false'}>")
    out = {
        "metric": "P-P+P-C interactions/s",
        "value": rows[0]["interactions_per_s"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": rows[0]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name} (n={n}, 100 % active, theta={cfg.theta}, "
                        f"bucket={cfg.bucket}, eps={eps:.6g}, Ewald {ewald_info['mode']})",
            "n": n, "theta": cfg.theta, "bucket": cfg.bucket, "active_fraction": 1.0,
            "parallelism": "single GPU",
        },
        "particles_per_s": rows[0]["particles_per_s"],
        "n_pp_interactions": st.n_pp_interactions,
        "n_pc_interactions": st.n_pc_interactions,
        "interact_variant": tuned,
        "roofline": {
            "bound": "alu",
            "kernel": kname + " (PP + PC, FP32 vector ALU)",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "frac_of_nonpacked_peak": achieved / PEAK_FP32_NONPACKED,
            "kernel_ms": k_ms,
            "kernel_ms_source": "device wall-clock stamps of the kernel (first queue claim to "
                                "last wave's exit), mean over the waited 100 % steps",
            "flop_per_pp": FLOP_PP,
            "flop_per_pc": FLOP_PC,
            "traffic": None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                            "copy-calibrated)",
        },
        "substeps": rows,
        "ewald_roofline": ewald_roof,
        "queue_order": {
            "note": "PP + PC kernel span (ms) per work-queue layout: cost order (longest first) "
                    "against locality order (costliest buckets first, the rest in tree order "
                    "in one segment per die); the steps above use the automatic choice",
            "rows": queue_rows},
        "store_positions": {
            "note": "positions read as the 28-byte store's 32-bit integers (12 B per particle, "
                    "equal masses without an array) against double positions + masses (32 B)",
            "rows": store_rows},
        "ewald": ewald_info,
        "device_prep_seconds": {"tree": prep["tree_s"], "lists": prep["lists_s"],
                                "cells": n_cell, "buckets": n_bucket,
                                "pp_entries": int(lists.pp_src.numel()),
                                "pc_entries": int(lists.pc_src.numel())},
    }
    detail = interact_traffic(cfg.name, tuned["pp_chunk"], tuned["waves_per_simd"],
                              tuned["pc_prefetch"])
    if detail is not None:
        out["roofline"]["traffic"] = detail.pop("bytes_per_launch")
        out["roofline"]["traffic_detail"] = detail
    if sample is not None:
        out["cpu_baseline"] = cpu_baseline_sample(sample, pos_t, mass_t, eps, a_sample,
                                                  p_sample, st.n_pp_interactions +
                                                  st.n_pc_interactions)
    if not args.no_fmm:
        out["fmm"] = fmm_leg(ctx, args)
        ctx.set_interact_variant(tuned["index"])  # the 512^3 set's choice again
    if not args.no_kdk:
        del tensors, prob, ws, lists, tree
        torch.cuda.empty_cache()
        out["kdk"] = kdk_leg(ctx, store, m_uniform, eps, cfg, amag, args.kdk_rungs)
    ctx.close()
    out["bench_seconds"] = time.perf_counter() - t_all
    print(json.dumps(out), flush=True)


def fmm_leg(ctx, args):
    """The fast-multipole form (CC / CP interactions into local expansions
    about the sink cells, Sec. 3.1) against the bucket walk on the 128^3
    clustered set (2 097 152 particles, exact Ewald): the same tree, host
    walks for both list kinds, each step timed as bind + compute (+ the
    expansions' CC / CP, shift and evaluation for the FMM)."""
    import numpy as np
    import torch

    import paper_1609_08621_amd as mg
    import workloads
    cfg = workloads.CONFIGS[3]
    ps = workloads.make(3)
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    tree = mg.tree_build(ps.pos, ps.mass, ps.box_L, 16)
    pt, mt = ps.pos[tree.perm], ps.mass[tree.perm]
    lists = mg.lists_build(tree, cfg.theta, ps.eps)
    t_bucket = time.perf_counter() - t0
    t0 = time.perf_counter()
    fl = mg.fmm_lists_build(tree, pt, cfg.theta, ps.eps)
    t_fmm_walk = time.perf_counter() - t0
    res = {}
    acc_out = {}
    for label, ls in (("bucket", lists), ("fmm", fl)):
        keep, p = ctx.upload(pt, mt, tree, ls, ps.eps, cfg.theta)
        ws = torch.empty(ctx.workspace_size(p), dtype=torch.uint8, device=dev)
        acc = torch.zeros(3 * ps.n, dtype=torch.float32, device=dev)
        pot = torch.zeros(ps.n, dtype=torch.float32, device=dev)
        fl_dev = None
        if label == "fmm":
            fl_dev = {k: torch.from_numpy(getattr(fl, k)).to(dev)
                      for k in ("cc_off", "cc_src", "cc_img")}

        # each list kind with the PP + PC variant that suits it best
        ctx.bind(p, keep, ws)
        variant, _ = ctx.autotune(acc, pot, budget_ms=1000.0)
        res[label + "_variant"] = mg.interact_variants()[variant]

        def step():
            ctx.bind(p, keep, ws)
            ctx.compute(acc, pot)
            st = ctx.wait(120.0)
            if fl_dev is not None:
                ctx.fmm_apply(keep["pos"], keep["mass"], keep, fl_dev, ps.eps, ps.box_L, acc,
                              pot)
            return st
        step()
        torch.cuda.synchronize()
        reps = max(3, min(args.steps, 10))
        t0 = time.perf_counter()
        for _ in range(reps):
            st = step()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        res[label] = {"ms_per_step": ms, "n_pp_interactions": st.n_pp_interactions,
                      "n_pc_interactions": st.n_pc_interactions}
        acc_out[label] = acc.view(3, -1).t().double().cpu().numpy()
        del keep, ws, acc, pot
    res["fmm"]["n_cc_cp_entries"] = int(fl.cc_src.size)
    res["fmm"]["n_cp_entries"] = int((fl.cc_src < 0).sum())
    a, b = acc_out["fmm"], acc_out["bucket"]
    diff = float(np.sqrt(np.mean(np.sum((a - b) ** 2, 1) / np.sum(b ** 2, 1))))
    log(f"fmm: bucket walk step {res['bucket']['ms_per_step']:.2f} ms "
        f"(pp {res['bucket']['n_pp_interactions']}, pc {res['bucket']['n_pc_interactions']}); "
        f"fmm step {res['fmm']['ms_per_step']:.2f} ms (pp {res['fmm']['n_pp_interactions']}, "
        f"pc {res['fmm']['n_pc_interactions']}, cc+cp entries {fl.cc_src.size}); rms difference "
        f"of the two methods {diff:.2e}; host walks {t_bucket:.1f} s (tree + bucket lists), "
        f"{t_fmm_walk:.1f} s (fmm lists)")
    return {"workload": f"{cfg.name} (n={ps.n}, theta {cfg.theta}, exact Ewald)",
            "bucket_walk": dict(res["bucket"], pp_pc_variant=res["bucket_variant"]),
            "fmm": dict(res["fmm"], pp_pc_variant=res["fmm_variant"]),
            "rms_rel_difference_fmm_vs_bucket_walk": diff,
            "host_seconds_tree_and_bucket_lists": t_bucket,
            "host_seconds_fmm_lists": t_fmm_walk}


def kdk_leg(ctx, store, m_uniform, eps, cfg, amag, rung_max):
    """One base step of the hierarchical KDK integrator (Sec. 3.2) on the
    whole set, from rest, every force on the device tree, walk and PP + PC
    + Ewald path; the base step is 2^(R-1) times the first percentile of
    the particles' time steps, so the deepest rung holds about 1 % (their
    substeps take the fixed and very active trees)."""
    import numpy as np
    import torch

    from paper_1609_08621_amd.kdk import Integrator
    dti = 0.2 * np.sqrt(eps / np.maximum(amag, 1e-300))
    dt_base = float(np.quantile(dti, 0.01)) * (1 << (rung_max - 1))
    pos = ctx.store_decode(store)
    vel = torch.zeros_like(pos, dtype=torch.float32)
    t0 = time.perf_counter()
    it = Integrator(ctx, pos, vel, m_uniform, eps, cfg.theta, 1.0, dt_base, rung_max)
    del pos, vel
    it.start()
    t_start = time.perf_counter() - t0
    t0 = time.perf_counter()
    it.base_step()
    t_step = time.perf_counter() - t0
    rungs = np.bincount(it.store.rung.cpu().numpy(), minlength=rung_max + 1)
    subs = [{"boundary": k, "rung_lo": lo, "active": n, "dual_tree": d, "seconds": sec}
            for (k, lo, n, d), sec in zip(it.log, it.seconds)]
    updates = sum(n for (_, _, n, _) in it.log)
    log(f"kdk: base step {dt_base:.3e} of 2^{rung_max} substeps in {t_step:.2f}s "
        f"({updates} particle updates), rungs {rungs.tolist()}, substeps "
        f"{[(s['active'], s['dual_tree'], round(s['seconds'], 3)) for s in subs]}")
    # the fixed tree kept (Sec. 3.2): the deepest rung's particles as the
    # very active group; the forest of one call against the fixed tree
    # built once and the very active tree rebuilt alone behind it (the
    # integrator above rebuilds both)
    kept = None
    g = (it.store.rung >= rung_max).to(torch.uint8)
    n_va = int(g.sum().item())
    if 0 < n_va < it.n:
        pos = ctx.store_decode(it.store)
        mass = torch.full((it.n,), m_uniform, dtype=torch.float64, device=pos.device)
        t_forest, t_rebuild = [], []
        for rep in range(2):  # the second build is kept for the comparison
            if rep:
                del tf
            t0 = time.perf_counter()
            tf = ctx.tree_build(pos, mass, 1.0, cfg.bucket, group_dev=g)
            torch.cuda.synchronize()
            t_forest.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        kf = ctx.forest_keep(pos, mass, 1.0, g, cfg.bucket)
        torch.cuda.synchronize()
        t_keep = time.perf_counter() - t0
        for rep in range(2):
            t0 = time.perf_counter()
            tk = ctx.forest_rebuild(kf, pos, mass)
            torch.cuda.synchronize()
            t_rebuild.append(time.perf_counter() - t0)
        same = all(torch.equal(getattr(tk, f), getattr(tf, f))
                   for f in ("perm", "cell_first", "child", "bucket_cell", "mom"))
        kept = {"very_active": n_va, "seconds_forest_one_call": min(t_forest),
                "seconds_fixed_tree_kept": t_keep,
                "seconds_very_active_tree_rebuilt": min(t_rebuild),
                "equal_to_one_call_forest": same}
        log(f"kdk: fixed tree kept: forest in one call {min(t_forest):.3f}s, fixed tree "
            f"{t_keep:.3f}s once, very active tree ({n_va} particles) rebuilt "
            f"{min(t_rebuild):.4f}s; equal arrays {same}")
        del tf, tk, kf, pos, mass
    del it
    torch.cuda.empty_cache()
    return {"workload": f"{cfg.name} from rest, rungs 0..{rung_max}, dt_base {dt_base:.4e}",
            "seconds_first_force": t_start, "seconds_base_step": t_step,
            "particle_updates_per_s": updates / t_step, "rungs_after": rungs.tolist(),
            "substeps": subs, "fixed_tree_kept": kept,
            "note": "a substep = drift, device tree (both trees below 5 % active), lists, "
                    "bind, PP + PC + Ewald for the active particles, kick and new rungs"}


def cpu_baseline_sample(sample, pos_t, mass_t, eps, a_gpu, p_gpu, n_int_step):
    """The FP64 oracle, as it stands, on a deterministic sample of sink
    buckets of the step (same tree and lists as the device): interactions/s
    over the sample, the whole step extrapolated by interaction count, and
    the device's error there (100 % step, exact Ewald)."""
    import numpy as np

    import oracle
    tree, lists, sel, idx, n_int = sample
    log(f"cpu baseline: oracle on {sel.size} sampled buckets, {idx.size} particles, "
        f"{oracle.num_threads()} threads")
    t0 = time.perf_counter()
    ao, po = oracle.evaluate(tree, lists, pos_t, mass_t, eps, 7)
    dt = time.perf_counter() - t0
    a_ref, p_ref = ao[idx], po[idx]
    rel = np.sqrt(np.sum((a_gpu - a_ref) ** 2, 1) / np.sum(a_ref ** 2, 1))
    _, pe = oracle.evaluate(tree, lists, pos_t, mass_t, eps, 4)  # untimed: the Ewald part
    tree_part = p_ref - pe[idx]
    perr = float(np.sqrt(np.sum((p_gpu - p_ref) ** 2) / np.sum(tree_part ** 2)))
    stride = int(sel[1] - sel[0]) if sel.size > 1 else 1
    return {
        "value": n_int / dt,
        "unit": "interactions/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"every {stride}th sink bucket of the 100 % step ({sel.size} buckets, "
                   f"{idx.size} particles, {n_int} PP+PC interactions plus their exact Ewald "
                   f"corrections) in {dt:.1f} s; the whole step ({n_int_step} interactions) "
                   f"would take {dt * n_int_step / max(n_int, 1):.0f} s (extrapolated by "
                   f"interaction count)"),
        "seconds": dt,
        "extrapolated_step_seconds": dt * n_int_step / max(n_int, 1),
        "gpu_rms_rel_acc_err_vs_oracle": float(np.sqrt(np.mean(rel ** 2))),
        "gpu_max_rel_acc_err_vs_oracle": float(rel.max()),
        "gpu_p99_rel_acc_err_vs_oracle": float(np.quantile(rel, 0.99)),
        "gpu_rel_pot_err_vs_oracle": perr,
        "pot_err_normalisation": "rms of the oracle's PP + PC potential",
    }


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def ewald_study(args):
    """Exact Ewald variants (order, k-space cut-off) against the learned
    correction (root, 8 or 64 top cells): time of the Ewald phase (median of
    5, with its spread) against the rms error of the corrected acceleration
    under both normalisations, relative to the total force and relative to
    the correction itself, with a converged exact correction as reference.
    Prints one JSON line."""
    import numpy as np
    import torch

    import paper_1609_08621_amd as mg
    import workloads

    cnum = args.config if args.config != 2 else 4
    cfg = workloads.CONFIGS[cnum]
    ps = workloads.make(cnum)
    t0 = time.perf_counter()
    tree = mg.tree_build(ps.pos, ps.mass, ps.box_L, cfg.bucket)
    lists = mg.lists_build(tree, cfg.theta, ps.eps)
    print(f"[ewald] {cfg.name}: n={ps.n} host prep {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    ctx = mg.Context(0)
    tensors, prob = ctx.upload(ps.pos[tree.perm], ps.mass[tree.perm], tree, lists, ps.eps,
                               cfg.theta)
    ws = torch.empty(ctx.workspace_size(prob), dtype=torch.uint8, device=dev)
    acc = torch.zeros(3 * ps.n, dtype=torch.float32, device=dev)
    pot = torch.zeros(ps.n, dtype=torch.float32, device=dev)
    ctx.bind(prob, tensors, ws)

    spread = {}

    def run(parts, ew, reps=5):
        ctx.set_ewald(**ew)
        ms = []
        for _ in range(reps):
            ctx.compute(acc, pot, parts)
            st = ctx.wait(120.0)
            ms.append(st.ms_ewald if parts == mg.PART_EWALD else st.ms_interact)
        torch.cuda.synchronize()
        spread["min"], spread["max"] = float(np.min(ms)), float(np.max(ms))
        return acc.view(3, -1).double().clone(), float(np.median(ms))

    exact = dict(mode=mg.EWALD_EXACT)
    a_tree, ms_tree = run(mg.PART_PP | mg.PART_PC, dict(exact, alpha=2.6, real_layers=1,
                                                         h2max=10, order=4), reps=2)
    a_ref, _ = run(mg.PART_EWALD, dict(exact, alpha=2.0, real_layers=2, h2max=36, order=4), 1)
    a_tot = a_tree + a_ref
    norm = (a_tot ** 2).sum(0)

    norm_corr = (a_ref ** 2).sum(0)

    def err(a_corr):
        return float(torch.sqrt(torch.mean(((a_corr - a_ref) ** 2).sum(0) / norm)))

    def err_corr(a_corr):  # relative to the correction itself
        return float(torch.sqrt(torch.mean(((a_corr - a_ref) ** 2).sum(0) / norm_corr)))

    rows = []
    none_err = err(torch.zeros_like(a_ref))
    for order in (0, 2, 4):
        for h2 in (0, 1, 2, 3, 4, 6, 10):
            for alpha in (2.0, 2.6):
                a_c, ms = run(mg.PART_EWALD, dict(exact, alpha=alpha, real_layers=1, h2max=h2,
                                                  order=order))
                rows.append(dict(kind="exact", order=order, h2max=h2, alpha=alpha, ms=ms,
                                 ms_min=spread["min"], ms_max=spread["max"], err=err(a_c),
                                 err_rel_corr=err_corr(a_c)))
    # train the surrogate on the library's own exact kernel (alpha 2.6, |h|^2 <= 10)
    u = torch.from_numpy(workloads.octant_points(args.train_samples)).to(dev)
    psi = ctx.ewald_psi(u, 2.6, 1, 10)
    psi0 = float(ctx.ewald_psi(torch.zeros((1, 3), dtype=torch.float64, device=dev), 2.6, 1,
                               10).cpu()[0, 0])
    ctx.mlp_attach(8192)
    ctx.mlp_set_weights(workloads.mlp_init().astype(np.float32))
    t0 = time.perf_counter()
    losses = ctx.mlp_train(u, psi, epochs=args.train_epochs, batch=8192, lr=3e-3, lr_min=3e-5,
                           psi0=psi0)
    train_s = time.perf_counter() - t0
    for top in (1, 8, 64):
        a_c, ms = run(mg.PART_EWALD, dict(mode=mg.EWALD_SURROGATE, top_cells=top))
        rows.append(dict(kind="surrogate", top_cells=top, ms=ms, ms_min=spread["min"],
                         ms_max=spread["max"], err=err(a_c), err_rel_corr=err_corr(a_c)))
    ex = sorted([r for r in rows if r["kind"] == "exact"], key=lambda r: r["ms"])
    front, best = [], float("inf")
    for r in ex:  # Pareto front of the exact variants: faster and more accurate
        if r["err"] < best:
            front.append(r)
            best = r["err"]
    verdict = []
    for r in rows:
        if r["kind"] != "surrogate":
            continue
        ok = [f for f in front if f["err"] <= r["err"]]
        cheapest = min(ok, key=lambda f: f["ms"]) if ok else None
        verdict.append(dict(top_cells=r["top_cells"], surrogate_ms=r["ms"], surrogate_err=r["err"],
                            exact_ms_at_equal_or_better_err=None if cheapest is None else cheapest["ms"],
                            exact_variant=cheapest,
                            surrogate_faster=None if cheapest is None else r["ms"] < cheapest["ms"]))
    out = dict(metric="Ewald correction: time vs rms force error (relative to total force)",
               config=dict(workload=cfg.name, n=ps.n, theta=cfg.theta),
               reference="exact, alpha 2.0, real layers 2, |h|^2 <= 36, order 4",
               no_correction_err=none_err, tree_kernel_ms=ms_tree, train_seconds=train_s,
               train_samples=args.train_samples, train_epochs=args.train_epochs,
               final_loss=float(losses[-1]), variants=rows, pareto_exact=front, verdict=verdict,
               cheapest_within_1e_2=min((r for r in rows if r["err"] <= 1e-2),
                                        key=lambda r: r["ms"], default=None))
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
