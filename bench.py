"""Benchmark of the batched docking hot path on one MI355X.

One step = the whole hot path over one batch of synthetic input already
resident in device memory: receptor grid maps (dock_load_pocket), the
sampler (initial poses + S Metropolis steps of L Adam refinements for T
trajectories of every ligand; dock_sample, batched form) and best-pose
selection (dock_best_poses).

    python bench.py [--steps K] [--warmup W] [--workload C2]

Prints one JSON line.  value = pose score+gradient evaluations per second over
whole steps (evaluations per ligand = T * (1 + S * (L + 1))); ligands docked/s,
the plain per-ligand form's rate and the batched/plain ratio ride along.
`roofline` is measured for the sampler kernel (the dominant kernel) with HIP
events around each of its launches on the launch stream; `cpu_baseline` times
the FP64 oracle on a bounded sample of the same workload.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

# FP32 vector peak without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2
# flops (FMA) x 2.4 GHz.  MI355X's published 157.3 TFLOP/s counts packed FP32,
# which the library is compiled without.
PEAK_FP32_TFLOPS = 78.6
PEAK_FP32_PACKED_TFLOPS = 157.3
N_LOCAL = 10


def flops_per_eval(n_atoms, n_pairs, n_tors):
    """Algorithmic FP32 operations of one score+gradient evaluation plus its
    Adam update, counted from the method's arithmetic: per atom 120 (placement
    18, trilinear value and gradient 84, torque terms 18), per intra pair 30,
    per torsion 124 (Rodrigues matrix, composition, gradient, Adam), per pose
    150 (rotation, rigid gradient, energy reduction, six Adam updates)."""
    return 120.0 * n_atoms + 30.0 * n_pairs + 124.0 * n_tors + 150.0


def measured_traffic(kernel_key):
    """HBM bytes per MC-step launch of one sampler bucket from the committed
    FETCH_SIZE / WRITE_SIZE counter runs (calibrated on a copy kernel), or
    None when the kernel sources changed since those runs."""
    import glob
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2510_24186_amd", "csrc", "*"))):
        h.update(open(p, "rb").read())
    if h.hexdigest() != rec.get("source_sha256"):
        return None
    launch = rec["launches"].get(kernel_key)
    return None if launch is None else float(launch["bytes"])


def ligand_table(D, H):
    rows = []
    for i in range(H.n):
        info = D.dock_ligand_info(H, i)
        rows.append((info["n_atoms"], info["n_pairs"], info["n_tors"]))
    return np.array(rows, np.float64)


def load_pocket(D, pk):
    return D.dock_load_pocket(pk.xyz, pk.type, pk.origin, pk.spacing, pk.dims)


def one_step(D, pk, H, T, S, form, use_graph, seed):
    pocket = load_pocket(D, pk)
    run = D.dock_sample(pocket, H, n_traj=T, n_steps=S, n_local=N_LOCAL, seed=seed, form=form,
                        use_graph=use_graph)
    v = run.view()
    import torch
    E_best = torch.empty((v.n_ligands, v.n_traj), device="cuda")
    q_best = torch.empty((v.n_ligands, v.n_traj, v.q_stride), device="cuda")
    D.lib.dock_run_copy_state(run.handle, None, None, D.binding._dptr(q_best), D.binding._dptr(E_best),
                              None, None, D.binding._stream(None))
    best = D.dock_best_poses(H, T, E_best, q_best, top_n=8, want_xyz=True)
    return pocket, run, best


# ------------------------------------------------------------------ CPU baseline

def _oracle_worker(args):
    name, lig_idx, T, S, seed = args
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import topology, score as SC, sampler as SM, params as P
    pk, L, _ = synth.workload(name)
    topo = topology.from_ligands(L, lig_idx)
    sc = SC.LazyScorer(pk[0], weights=np.asarray(P.TRIDS_WEIGHTS, np.float32).astype(np.float64))
    prm = SM.SamplerParams(n_traj=T, n_steps=S, n_local=N_LOCAL, seed=seed)
    SM.sample(sc, topo, lig_idx, prm)            # fills the lazily computed map nodes
    t0 = time.perf_counter()
    SM.sample(sc, topo, lig_idx, prm)            # timed: sampling only
    dt = time.perf_counter() - t0
    return T * (1 + S * (N_LOCAL + 1)), dt


def cpu_baseline(name, n_lig_total, T_sample=32, S_sample=8, n_sample=8):
    """The oracle on `n_sample` ligands (spread over the size range), one
    process per ligand; returns evals/s summed over the workers."""
    from oracle import topology
    _, L, _ = synth.workload(name)
    sizes = np.diff(L.atom_off)
    order = np.argsort(sizes, kind="stable")
    picks = [int(order[int(round(k * (len(order) - 1) / max(1, n_sample - 1)))]) for k in range(n_sample)]
    cores = min(n_sample, os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(name, i, T_sample, S_sample, 1) for i in picks])
    wall = time.perf_counter() - t0
    evals = sum(r[0] for r in res)
    busy = sum(r[1] for r in res)
    per_core = evals / busy
    del topology
    return dict(value=per_core * cores, unit="evals/s", cores=cores, kind="oracle",
                sample="%d ligands of the workload spread over its size range (N %s), %d trajectories x %d MC "
                       "steps x %d Adam steps each, one process per ligand; sampling time only (map nodes "
                       "computed in an untimed identical first pass); wall %.1fs"
                       % (n_sample, "/".join(str(int(sizes[i])) for i in picks), T_sample, S_sample, N_LOCAL,
                          wall))


# ------------------------------------------------------------------ main

def _event_ms(fn):
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    res = fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b), res


def extras(D, pk, L, T, S, n_sub=32):
    """Side measurements on the same pocket: the map build, the adjoint of
    the map build, and the sampler on a 32-ligand subset (spread over the
    size range) in the direct pair mode and with the E_MDN term.  Device
    time from events on the current stream (the stream the calls use)."""
    import torch
    out = {}
    ms, pocket = _event_ms(lambda: load_pocket(D, pk))
    out["map_build_ms"] = round(ms, 3)
    lam = torch.randn((8, 3) + tuple(pk.dims[::-1]), device="cuda")
    dx = torch.zeros((len(pk.xyz), 3), device="cuda")
    dth = torch.zeros(13, dtype=torch.float64, device="cuda")
    D.dock_pocket_map_adjoint(pocket, lam, dx, dth)
    ms, _ = _event_ms(lambda: D.dock_pocket_map_adjoint(pocket, lam, dx, dth))
    out["map_adjoint_ms"] = round(ms, 3)
    order = np.argsort(np.diff(L.atom_off), kind="stable")
    sub = np.sort(order[np.linspace(0, len(order) - 1, n_sub).astype(int)])
    Ls = L.subset(sub)
    Hs = D.dock_load_ligands(Ls.atom_off, Ls.element, Ls.n_h, Ls.xyz, Ls.bond_off, Ls.bonds, Ls.rotatable,
                             pocket_index=Ls.pocket_index)
    evals = n_sub * T * (1 + S * (N_LOCAL + 1))
    modes = {}
    residue = synth.make_residues(pk)
    n_res = int(residue.max()) + 1
    p_grid = pocket
    p_direct = D.dock_load_pocket(pk.xyz, pk.type, pk.origin, pk.spacing, pk.dims, inter_mode=D.INTER_DIRECT)
    p_mdn = D.dock_load_pocket(pk.xyz, pk.type, pk.origin, pk.spacing, pk.dims, residue=residue)
    for name, pp in (("grid", p_grid), ("direct", p_direct), ("grid+E_MDN", p_mdn)):
        if name == "grid+E_MDN":
            D.dock_ligands_set_mdn(Hs, synth.make_mdn_params(int(Ls.atom_off[-1]), n_res, 4, seed=5))
        # a short untimed run first (kernel loading, first-touch of the tables)
        D.dock_sample(pp, Hs, n_traj=T, n_steps=2, n_local=N_LOCAL, seed=1, form=D.FORM_BATCHED)
        ms, run = _event_ms(lambda: D.dock_sample(pp, Hs, n_traj=T, n_steps=S, n_local=N_LOCAL, seed=1,
                                                  form=D.FORM_BATCHED))
        modes[name] = dict(ms=round(ms, 3), evals_per_s=round(evals / (ms * 1e-3), 1))
    out["sampler_modes"] = dict(ligands=n_sub, n_traj=T, n_steps=S, n_res=n_res, mdn_gaussians=4, **modes)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-ligand form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the side measurements (map build and adjoint, direct and E_MDN modes)")
    ap.add_argument("--graph", type=int, default=0, help="replay sampler launches as a hipGraph")
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the sampler has no multi-GPU path (ligands and "
              "trajectories shard across GPUs with no communication); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2510_24186_amd as D

    assert torch.cuda.is_available()
    pockets, L, wl = synth.workload(args.workload)
    if len(pockets) != 1:
        raise SystemExit("bench workloads use one pocket")
    pk = pockets[0]
    T, S = wl["T"], wl["S"]
    H = D.dock_load_ligands(L.atom_off, L.element, L.n_h, L.xyz, L.bond_off, L.bonds, L.rotatable,
                            pocket_index=L.pocket_index)
    tab = ligand_table(D, H)
    evals_lig = T * (1 + S * (N_LOCAL + 1))
    evals_total = evals_lig * H.n
    flops_lig = np.array([flops_per_eval(*r) for r in tab]) * evals_lig
    print("workload %s: %d ligands (N %d-%d, mean %.1f; pairs mean %.0f), T %d, S %d, L %d, %d evals/step"
          % (args.workload, H.n, tab[:, 0].min(), tab[:, 0].max(), tab[:, 0].mean(), tab[:, 1].mean(), T, S,
             N_LOCAL, evals_total), file=sys.stderr, flush=True)

    def step(k):
        return one_step(D, pk, H, T, S, D.FORM_BATCHED, args.graph, seed=k)

    if args.calib_copy_mib:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the sampler kernel's counters in the same profiled run
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for k in range(args.warmup):
        step(1000 + k)
        torch.cuda.synchronize()
        print("warmup step %d done" % k, file=sys.stderr, flush=True)
    kern_ms, launch_stats = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    keep = []
    for k in range(args.steps):
        pocket, run, best = step(k)
        keep.append((pocket, run, best))
        if len(keep) > 2:
            keep.pop(0)
        kern_ms.append(D.dock_run_kernel_ms(run))
        launch_stats.append(D.dock_run_launch_stats(run))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print("timed %d steps in %.3fs" % (args.steps, t1 - t0), file=sys.stderr, flush=True)
    ms_step = 1e3 * (t1 - t0) / args.steps
    plan = D.dock_run_plan(keep[-1][1])

    # roofline of the sampler kernel: algorithmic FP32 work of the MC-step
    # launches / their event-measured durations, per lane configuration
    lb = plan["lig_bucket"]
    per_bucket = {}
    for st in launch_stats:
        for l in st:
            if l["init"] or l["ms"] <= 0:
                continue
            b = l["bucket"]
            flop = float(np.sum(flops_lig[lb == b])) * (S * (N_LOCAL + 1)) / (1 + S * (N_LOCAL + 1))
            d = per_bucket.setdefault(b, dict(lanes=int(l["lanes_per_pose"]), apl=int(l["atoms_per_lane"]),
                                              block=int(l["block"]), grid=int(l["grid"]),
                                              items=int(l["n_items"]), ms=[], flop=flop,
                                              ligands=int(np.sum(lb == b))))
            d["ms"].append(l["ms"])
    # lane buckets run concurrently (side streams): the dominant kernel is
    # the one with the most work, its duration as measured while overlapped
    dom = max(per_bucket.values(), key=lambda d: d["flop"])
    achieved = dom["flop"] / (np.mean(dom["ms"]) * 1e-3) / 1e12
    traffic = measured_traffic("%d,%d,%d,0" % (dom["lanes"], dom["apl"], dom["block"]))
    roofline = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / PEAK_FP32_TFLOPS, 4),
                    traffic=None if traffic is None else round(traffic),
                    frac_of_packed_peak=round(achieved / PEAK_FP32_PACKED_TFLOPS, 4),
                    kernel="sample_kernel<%d,%d,%d>" % (dom["lanes"], dom["apl"], dom["block"]),
                    launch_ms=round(float(np.mean(dom["ms"])), 3),
                    sampler_tflops=round(float(np.sum(flops_lig)) / (float(np.mean(kern_ms)) * 1e-3) / 1e12, 3),
                    buckets=[dict(lanes=d["lanes"], atoms_per_lane=d["apl"], ligands=d["ligands"],
                                  block=d["block"], grid=d["grid"], work_items=d["items"],
                                  ms=round(float(np.mean(d["ms"])), 3),
                                  tflops=round(d["flop"] / (np.mean(d["ms"]) * 1e-3) / 1e12, 3))
                             for d in per_bucket.values()])

    evals_per_s = evals_total / (ms_step * 1e-3)
    sampler_ms = float(np.mean(kern_ms))
    out = dict(metric="pose score+grad evals/s and ligands docked/s, batched vs plain, 1 MI355X",
               value=round(evals_per_s, 1), unit="evals/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(ms_step, 3), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload="%s: 1 pocket of %d receptor atoms, grid %dx%dx%d x 8 types at %.3f A; "
                                    "%d ligands of %d-%d heavy atoms and 0-%d torsions; %d trajectories x %d MC "
                                    "steps x %d Adam steps; TRIDS physics terms"
                                    % (args.workload, len(pk.xyz), *pk.dims, pk.spacing, H.n, tab[:, 0].min(),
                                       tab[:, 0].max(), tab[:, 2].max(), T, S, N_LOCAL),
                           n_ligands=H.n, n_traj=T, n_steps=S, n_local=N_LOCAL, evals_per_step=evals_total),
               ligands_per_s=round(H.n / (ms_step * 1e-3), 2),
               sampler_evals_per_s=round(evals_total / (sampler_ms * 1e-3), 1),
               sampler_ms=round(sampler_ms, 3),
               roofline=roofline)
    if not args.no_plain:
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        one_step(D, pk, H, T, S, D.FORM_PLAIN, 0, seed=0)
        torch.cuda.synchronize()
        plain_ms = 1e3 * (time.perf_counter() - tp0)
        out["plain"] = dict(ms_per_step=round(plain_ms, 3), evals_per_s=round(evals_total / (plain_ms * 1e-3), 1),
                            ligands_per_s=round(H.n / (plain_ms * 1e-3), 2))
        out["batched_vs_plain"] = round(plain_ms / ms_step, 3)
        print("plain form: %.1f ms per step" % plain_ms, file=sys.stderr, flush=True)
    if not args.no_extras:
        out["extras"] = extras(D, pk, L, T, S)
        print("extras done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload, H.n)
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
