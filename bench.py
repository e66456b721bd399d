#!/usr/bin/env python3
"""Throughput of the gravity hot path on one MI355X.

One step = one pass of the whole device path over the bound workload:
staging of particles, cells and lists (mgrav_bind) followed by the PP + PC
evaluation and the Ewald correction (mgrav_compute), with inputs already
resident in HBM.  The workload is the periodic perturbed lattice (64^3
particles, theta 0.7, buckets of 16, exact Ewald), seeded and synthetic.

Prints one JSON line.  The metric is PP + PC interactions per second;
``roofline`` covers the PP + PC kernel (FP32 vector ALU); ``cpu_baseline``
times the FP64 oracle on a bounded sample of the same buckets.
"""
import argparse
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
FLOP_PC = 242
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak (packed)
PEAK_FP32_NONPACKED = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--cpu-stride", type=int, default=4,
                    help="oracle baseline evaluates every k-th bucket")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    def step():
        ctx.bind(prob, tensors, ws)
        ctx.compute(acc, pot)
        return ctx.wait(60.0)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ms_k, ms_e, ms_c = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step()
        ms_k.append(st.ms_interact)
        ms_e.append(st.ms_ewald)
        ms_c.append(st.ms_total)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    n_int = st.n_pp_interactions + st.n_pc_interactions
    value = n_int / (ms_step * 1e-3)
    flops = st.n_pp_interactions * FLOP_PP + st.n_pc_interactions * FLOP_PC
    k_ms = float(np.mean(ms_k))
    achieved = flops / (k_ms * 1e-3) / 1e12
    print(f"[bench] step {ms_step:.3f} ms (compute {np.mean(ms_c):.3f} ms: PP+PC kernel "
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
        "particles_per_s": ps.n / (ms_step * 1e-3),
        "n_pp_interactions": st.n_pp_interactions,
        "n_pc_interactions": st.n_pc_interactions,
        "ms_compute": float(np.mean(ms_c)),
        "ms_interact_kernel": k_ms,
        "ms_ewald": float(np.mean(ms_e)),
        "roofline": {
            "bound": "alu",
            "kernel": "k_interact (PP + PC, FP32 vector ALU)",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "frac_of_nonpacked_peak": achieved / PEAK_FP32_NONPACKED,
            "flop_per_pp": FLOP_PP,
            "flop_per_pc": FLOP_PC,
            "traffic": None,
        },
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, ps, cfg, tree, pos_t, mass_t, acc, pot)
    ctx.close()
    print(json.dumps(out), flush=True)


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
    perr = float(np.sqrt(np.sum((pg - po[idx]) ** 2) / np.sum(po[idx] ** 2)))
    return {
        "value": n_int / dt,
        "unit": "interactions/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"every {args.cpu_stride}th sink bucket ({sel.size} of {to.n_bucket}, "
                  f"{idx.size} particles, {n_int} PP+PC interactions plus their Ewald "
                  f"corrections) in {dt:.1f} s",
        "seconds": dt,
        "gpu_rms_rel_acc_err_vs_oracle": err,
        "gpu_rel_pot_err_vs_oracle": perr,
    }


if __name__ == "__main__":
    main()
