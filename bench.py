"""Benchmark of the batched docking hot path on one MI355X.

One step = the whole hot path over one batch of synthetic input already
resident in device memory: receptor grid maps of every pocket (built in
place by dock_pocket_rebuild), the sampler (initial poses + S Metropolis steps of L
Adam refinements for T trajectories of every ligand; dock_sample, batched
form, all pockets in one call), best-pose selection (dock_best_poses) and,
for the mixed-pocket workload, the adjoint of the summed best-pose energies
to every pocket's per-term maps and weights (dock_score_adjoint).

    python bench.py [--steps K] [--warmup W] [--workload C5|C4|C2|C1]

Default workload: mixed pockets (16 pockets of 800-3,000 atoms with 48^3-96^3
x 8 maps, 65,536 ligands of 10-70 heavy atoms assigned round-robin, 64
trajectories x 200 MC steps x 10 Adam steps, adjoint enabled), the largest
one-GPU configuration.  Prints one JSON line.  value = pose score+gradient
evaluations per second over whole steps (evaluations per ligand =
T * (1 + S * (L + 1))); ligands docked/s, the plain per-ligand form's rate on
a size-stratified subset and the batched/plain ratio ride along.  `roofline`
is measured for the dominant sampler kernel with HIP events around each of
its launches on the launch stream; `cpu_baseline` times the FP64 oracle on a
bounded, size-stratified sample of the same workload.
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

# MI355X published FP32 vector peak (counts packed FP32, two operations per
# lane per cycle); the library is compiled without packed FP32, so one lane
# retires at most one FMA per cycle: 256 CUs x 4 SIMDs x 16 lanes x 2 flops
# x 2.4 GHz = 78.6 TFLOP/s is the reachable ceiling, reported beside.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_NONPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
L2_LINE_BYTES = 128
N_LOCAL = 10
PAPER_MEM_MB = 380.0   # Table 5: GPU memory per docking, RTX A6000 (context only)


def flops_per_eval(n_atoms, n_pairs, n_tors):
    """Algorithmic FP32 operations of one score + gradient evaluation: per atom
    ~15 for the placement, ~65 for the trilinear value and gradient, ~25 for
    the chain rule; ~50 per intra-ligand pair; ~60 per torsion."""
    return 105.0 * n_atoms + 50.0 * n_pairs + 60.0 * n_tors


def kernel_record(workload, kernel_key):
    """Counter record of one sampler launch of a workload from
    profiles/traffic.json (HBM bytes calibrated on a copy kernel, L2
    requests, VALU busy), or None when the kernel sources changed since those
    runs."""
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
    return rec.get("workloads", {}).get(workload, {}).get(kernel_key)


def ligand_table(D, H):
    rows = []
    for i in range(H.n):
        info = D.dock_ligand_info(H, i)
        rows.append((info["n_atoms"], info["n_pairs"], info["n_tors"]))
    return np.array(rows, np.float64)


def load_pockets(D, pks, keep):
    return [D.dock_load_pocket(pk.xyz, pk.type, pk.origin, pk.spacing, pk.dims, keep_per_term=keep)
            for pk in pks]


class Step:
    """The hot path over one batch: every pocket's maps built (in place, in
    the handles made once), the sampler, the best poses and, with `adjoint`,
    the adjoint of the summed best-pose energies.  The run is created by the
    first step (buffers, plan and work items) and restarted with a new seed
    by the later ones."""

    def __init__(self, D, pks, H, T, S, adjoint, use_graph):
        import torch
        self.D, self.H, self.T, self.S = D, H, T, S
        self.adjoint = adjoint
        self.use_graph = use_graph
        self.pockets = load_pockets(D, pks, adjoint)
        self.run = None
        self.lig = torch.arange(H.n, dtype=torch.int32, device="cuda")
        self.ones = torch.ones(H.n, device="cuda")
        self.w = torch.tensor(np.stack([D.dock_pocket_terms(pp)[2] for pp in self.pockets]), device="cuda")

    def __call__(self, seed):
        import torch
        D = self.D
        for pp in self.pockets:
            D.dock_pocket_rebuild(pp)
        if self.run is None:
            self.run = D.dock_sample(self.pockets, self.H, n_traj=self.T, n_steps=self.S, n_local=N_LOCAL,
                                     seed=seed, form=D.FORM_BATCHED, use_graph=self.use_graph)
        else:
            D.dock_run_restart(self.run, seed)
        v = self.run.view()
        E_best = torch.empty((v.n_ligands, v.n_traj), device="cuda")
        q_best = torch.empty((v.n_ligands, v.n_traj, v.q_stride), device="cuda")
        D.lib.dock_run_copy_state(self.run.handle, None, None, D.binding._dptr(q_best), D.binding._dptr(E_best),
                                  None, None, D.binding._stream(None))
        best = D.dock_best_poses(self.H, self.T, E_best, q_best, top_n=8, want_xyz=True)
        out = dict(best=best)
        if self.adjoint:
            # every pocket's kept per-term maps (G = None), weights as loaded
            dG = [torch.zeros((8, pp.n_terms, pp.dims[2], pp.dims[1], pp.dims[0]), device="cuda")
                  for pp in self.pockets]
            dw = torch.zeros_like(self.w)
            D.dock_score_adjoint(self.pockets, self.H, self.lig, self.w, self.ones,
                                 q=best["q"][:, 0].contiguous(), G=None, dLdG=dG, dLdw=dw, deterministic=1)
            out.update(dLdG=dG, dLdw=dw)
        return out


# ------------------------------------------------------------------ CPU baseline

def _oracle_worker(args):
    pocket, ligs, i, lig_id, T, S, seed = args
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import topology, score as SC, sampler as SM, params as P
    topo = topology.from_ligands(ligs, i)
    sc = SC.LazyScorer(pocket, weights=np.asarray(P.TRIDS_WEIGHTS, np.float32).astype(np.float64))
    prm = SM.SamplerParams(n_traj=T, n_steps=S, n_local=N_LOCAL, seed=seed)
    SM.sample(sc, topo, lig_id, prm)            # fills the lazily computed map nodes
    t0 = time.perf_counter()
    SM.sample(sc, topo, lig_id, prm)            # timed: sampling only
    dt = time.perf_counter() - t0
    return T * (1 + S * (N_LOCAL + 1)), dt


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pks, L, n_sample=256, T_sample=4, S_sample=1):
    """The oracle on a size-stratified sample of the workload's ligands (each
    against its own pocket), one process per host core (at most 16); returns
    evals/s over the workers' busy time times the worker count."""
    sizes = np.diff(L.atom_off)
    order = np.argsort(sizes, kind="stable")
    n_sample = min(n_sample, L.n_ligands)
    picks = sorted({int(order[int(round(k * (len(order) - 1) / max(1, n_sample - 1)))]) for k in range(n_sample)})
    sub = L.subset(picks)
    cores = synth.default_workers()
    jobs = [(pks[int(L.pocket_index[l])], sub, a, l, T_sample, S_sample, 1) for a, l in enumerate(picks)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_worker, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    evals = sum(r[0] for r in res)
    busy = sum(r[1] for r in res)
    return dict(value=round(evals / busy * cores, 1), unit="evals/s", cores=cores, kind="oracle",
                host_cpus=os.cpu_count(), cpu_model=_cpu_model(),
                sample="subset: %d ligands stratified by size (N %d-%d) of the %d, %d trajectories x %d MC steps "
                       "x %d Adam steps each, one process per ligand on %d workers; sampling time only (map "
                       "nodes computed in an untimed identical first pass); wall %.1fs"
                       % (len(picks), sizes[picks].min(), sizes[picks].max(), L.n_ligands, T_sample, S_sample,
                          N_LOCAL, cores, wall))


# ------------------------------------------------------------------ side measurements

def _event_ms(fn):
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    res = fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b), res


def workload_rate(D, name, steps=1, workers=1, plain=False):
    """One untimed and `steps` timed whole steps of a one-pocket workload;
    with `plain`, also the plain form over all of its ligands."""
    import torch
    pks, L, wl = synth.workload(name, workers=workers)
    H = D.dock_load_ligands(L.atom_off, L.element, L.n_h, L.xyz, L.bond_off, L.bonds, L.rotatable,
                            pocket_index=L.pocket_index)
    T, S = wl["T"], wl["S"]
    step = Step(D, pks, H, T, S, adjoint=False, use_graph=0)
    step(900)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(k)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    ev = H.n * T * (1 + S * (N_LOCAL + 1))
    kms = D.dock_run_kernel_ms(step.run)
    out = dict(ligands=H.n, n_traj=T, n_steps=S, ms_per_step=round(ms, 2),
               evals_per_s=round(ev / (ms * 1e-3), 1), ligands_per_s=round(H.n / (ms * 1e-3), 1),
               sampler_ms=round(kms, 2))
    if plain:
        # both forms timed alike: sampling from a new run, best poses
        forms = {}
        for fname, form in (("batched", D.FORM_BATCHED), ("plain", D.FORM_PLAIN)):
            fms = _form_ms(D, step.pockets, H, T, S, form)
            forms[fname] = dict(ms=round(fms, 2), evals_per_s=round(ev / (fms * 1e-3), 1),
                                ligands_per_s=round(H.n / (fms * 1e-3), 2))
        out["forms"] = forms
        out["batched_vs_plain"] = round(forms["plain"]["ms"] / forms["batched"]["ms"], 3)
    return out


def _form_ms(D, pockets, H, T, S, form):
    """Wall time of one dock_sample call of the given form (the plain form:
    one launch per ligand, in order, on one stream) over every ligand of H,
    best poses included, after a one-step warm-up."""
    import torch
    D.dock_sample(pockets, H, n_traj=T, n_steps=1, n_local=N_LOCAL, seed=3, form=form, use_graph=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run = D.dock_sample(pockets, H, n_traj=T, n_steps=S, n_local=N_LOCAL, seed=0, form=form, use_graph=0)
    v = run.view()
    E_best = torch.empty((v.n_ligands, v.n_traj), device="cuda")
    q_best = torch.empty((v.n_ligands, v.n_traj, v.q_stride), device="cuda")
    D.lib.dock_run_copy_state(run.handle, None, None, D.binding._dptr(q_best), D.binding._dptr(E_best),
                              None, None, D.binding._stream(None))
    D.dock_best_poses(H, T, E_best, q_best, top_n=8, want_xyz=True)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0)


def _docking_buffers_bytes(pocket, L, T, top_n=8):
    """Device bytes one docking of the largest ligand of L holds, counted
    from the buffer sizes (a device-memory delta is blurred by the
    allocators' caching): the combined maps (8 types x nodes x 4 B), the
    run's state (current and best q and E, evaluation counts: T x
    (2 q_stride + 3) x 4 B; q_stride = 6 + max torsions of L) and the best-
    pose outputs (top_n x (E, E_screen, index, q, xyz))."""
    nodes = int(np.prod(pocket.dims))
    n_max = int(np.max(np.diff(L.atom_off)))
    qs = 6 + max(int(np.sum(L.rotatable[L.bond_off[i]:L.bond_off[i + 1]])) for i in range(L.n_ligands))
    return 8 * nodes * 4 + T * (2 * qs + 3) * 4 + top_n * (3 + qs + 3 * n_max) * 4


def paper_shape_rate(D, n_single=8):
    """Dockings in the paper's sampling shape (1,024 copies x 8 MC steps x
    10 Adam steps per ligand; Methods, "Conformation sampling") on the
    screening workload's pocket and ligands: single mode, one ligand per
    call (mean over `n_single` ligands spread over the size range), and
    batch mode, all 256 ligands in one call.  Sampling plus best poses,
    wall time.  Context for the paper's per-docking times (Table 5), which
    were taken on other hardware with a pipeline that includes more than
    this path."""
    pks, L, wl = synth.workload("C2")
    T, S = 1024, 8
    pockets = load_pockets(D, pks, False)
    H = D.dock_load_ligands(L.atom_off, L.element, L.n_h, L.xyz, L.bond_off, L.bonds, L.rotatable,
                            pocket_index=L.pocket_index)
    order = np.argsort(np.diff(L.atom_off), kind="stable")
    pick = np.sort(order[np.linspace(0, len(order) - 1, n_single).astype(int)])
    single = []
    for i in pick:
        Li = L.subset(np.array([i]))
        Hi = D.dock_load_ligands(Li.atom_off, Li.element, Li.n_h, Li.xyz, Li.bond_off, Li.bonds, Li.rotatable,
                                 pocket_index=Li.pocket_index)
        single.append(_form_ms(D, pockets, Hi, T, S, D.FORM_BATCHED))
    batch = _form_ms(D, pockets, H, T, S, D.FORM_BATCHED)
    ev = T * (1 + S * (N_LOCAL + 1))
    return dict(n_traj=T, n_steps=S, n_local=N_LOCAL, evals_per_docking=ev,
                single_ms_per_docking=round(float(np.mean(single)), 3), single_ligands=int(len(pick)),
                single_buffers_mb=round(_docking_buffers_bytes(pockets[0], L, T) / 2**20, 2),
                batch_ligands=H.n, batch_ms=round(batch, 2), batch_ms_per_pair=round(batch / H.n, 4),
                batch_evals_per_s=round(ev * H.n / (batch * 1e-3), 1),
                paper_context="Table 5 (RTX A6000, whole pipeline): 2.3 s per docking single, 0.33 s per pair batch")


def differentiation_rate(D):
    """The differentiation workload (2,000-atom pocket, Vina-form terms, 64
    ligands x 32 poses): forward (dock_score_terms) and adjoint
    (dock_score_adjoint, float atomics and deterministic) device times."""
    import torch
    pks, L, wl = synth.workload("C3")
    pk = pks[0]
    w = synth.vina_weights(np.random.default_rng(33))
    p = D.dock_load_pocket(pk.xyz, pk.type, pk.origin, pk.spacing, pk.dims, preset=D.PRESET_VINA, weights=w,
                           keep_per_term=True)
    H = D.dock_load_ligands(L.atom_off, L.element, L.n_h, L.xyz, L.bond_off, L.bonds, L.rotatable,
                            pocket_index=L.pocket_index)
    rng = np.random.default_rng(34)
    T = wl["T"]
    Q = np.zeros((L.n_ligands * T, H.q_stride), np.float32)
    for i in range(L.n_ligands):
        info = D.dock_ligand_info(H, i)
        n_dof = 6 + info["n_tors"]
        Q[i * T:(i + 1) * T, :n_dof] = synth.random_poses(n_dof, info["box_min"], info["box_max"], T, rng)
    q = torch.tensor(Q, device="cuda")
    lig = torch.tensor(np.repeat(np.arange(L.n_ligands), T).astype(np.int32), device="cuda")
    wt = torch.tensor(w[None], device="cuda")
    G = D.dock_pocket_maps(p, per_term=True)
    dLdE = torch.ones(len(Q), device="cuda")
    dG, dw, dq = torch.zeros_like(G), torch.zeros_like(wt), torch.zeros_like(q)
    out = {}
    for rep in range(2):
        f_ms, _ = _event_ms(lambda: D.dock_score_terms(p, H, lig, wt, q=q, G=[G]))
        a_ms, _ = _event_ms(lambda: D.dock_score_adjoint(p, H, lig, wt, dLdE, q=q, G=[G], dLdG=[dG], dLdw=dw,
                                                         dLdq=dq, deterministic=0))
        d_ms, _ = _event_ms(lambda: D.dock_score_adjoint(p, H, lig, wt, dLdE, q=q, G=[G], dLdG=[dG], dLdw=dw,
                                                         dLdq=dq, deterministic=1))
        out = dict(poses=len(Q), forward_ms=round(f_ms, 3), adjoint_ms=round(a_ms, 3),
                   adjoint_deterministic_ms=round(d_ms, 3),
                   poses_per_s_forward_adjoint=round(len(Q) / ((f_ms + a_ms) * 1e-3), 1))
    return out


def extras(D, pk, L, T, S, n_sub=32):
    """Side measurements on one pocket: the map build, the adjoint of the map
    build, and the sampler on a 32-ligand subset (spread over the size range)
    in the grid, direct pair and grid + E_MDN modes.  Device time from events
    on the current stream (the stream the calls use)."""
    import torch
    out = {}
    ms, pocket = _event_ms(lambda: D.dock_load_pocket(pk.xyz, pk.type, pk.origin, pk.spacing, pk.dims))
    out["map_build_ms"] = round(ms, 3)
    out["map_build_pocket"] = "%d atoms, %dx%dx%d nodes x 8 types" % (len(pk.xyz), *pk.dims)
    lam = torch.randn((8, 3) + tuple(pk.dims[::-1]), device="cuda")
    dx = torch.zeros((len(pk.xyz), 3), device="cuda")
    dth = torch.zeros(13, dtype=torch.float64, device="cuda")
    D.dock_pocket_map_adjoint(pocket, lam, dx, dth)
    ms, _ = _event_ms(lambda: D.dock_pocket_map_adjoint(pocket, lam, dx, dth))
    out["map_adjoint_ms"] = round(ms, 3)
    order = np.argsort(np.diff(L.atom_off), kind="stable")
    sub = np.sort(order[np.linspace(0, len(order) - 1, n_sub).astype(int)])
    Ls = L.subset(sub)
    Ls.pocket_index = np.zeros(len(sub), np.int32)
    Hs = D.dock_load_ligands(Ls.atom_off, Ls.element, Ls.n_h, Ls.xyz, Ls.bond_off, Ls.bonds, Ls.rotatable,
                             pocket_index=Ls.pocket_index)
    evals = n_sub * T * (1 + S * (N_LOCAL + 1))
    modes = {}
    residue = synth.make_residues(pk)
    n_res = int(residue.max()) + 1
    p_direct = D.dock_load_pocket(pk.xyz, pk.type, pk.origin, pk.spacing, pk.dims, inter_mode=D.INTER_DIRECT)
    p_mdn = D.dock_load_pocket(pk.xyz, pk.type, pk.origin, pk.spacing, pk.dims, residue=residue)
    for name, pp in (("grid", pocket), ("direct", p_direct), ("grid+E_MDN", p_mdn)):
        if name == "grid+E_MDN":
            D.dock_ligands_set_mdn(Hs, synth.make_mdn_params(int(Ls.atom_off[-1]), n_res, 4, seed=5))
        # a short untimed run first (kernel loading, first-touch of the tables)
        D.dock_sample(pp, Hs, n_traj=T, n_steps=2, n_local=N_LOCAL, seed=1, form=D.FORM_BATCHED)
        ms, run = _event_ms(lambda: D.dock_sample(pp, Hs, n_traj=T, n_steps=S, n_local=N_LOCAL, seed=1,
                                                  form=D.FORM_BATCHED))
        modes[name] = dict(ms=round(ms, 3), evals_per_s=round(evals / (ms * 1e-3), 1))
        del run
    out["sampler_modes"] = dict(ligands=n_sub, n_traj=T, n_steps=S, n_res=n_res, mdn_gaussians=4, **modes)
    return out


def plain_rate(D, pks, L, H_full, T, S, n_sub=256):
    """The plain form (one launch per ligand, in order, on one stream) on a
    size-stratified subset of the workload, all pockets in the call."""
    order = np.argsort(np.diff(L.atom_off), kind="stable")
    sub = np.sort(order[np.linspace(0, len(order) - 1, min(n_sub, L.n_ligands)).astype(int)])
    Ls = L.subset(sub)
    Hs = D.dock_load_ligands(Ls.atom_off, Ls.element, Ls.n_h, Ls.xyz, Ls.bond_off, Ls.bonds, Ls.rotatable,
                             pocket_index=Ls.pocket_index)
    pockets = load_pockets(D, pks, False)
    ms = _form_ms(D, pockets, Hs, T, S, D.FORM_PLAIN)
    ev = len(sub) * T * (1 + S * (N_LOCAL + 1))
    return dict(ligands=len(sub), subset="stratified by size", ms=round(ms, 2),
                evals_per_s=round(ev / (ms * 1e-3), 1), ligands_per_s=round(len(sub) / (ms * 1e-3), 2))


# ------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C5")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-ligand form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the side measurements (other workloads, map build and adjoint, modes)")
    ap.add_argument("--graph", type=int, default=0, help="replay sampler launches as a hipGraph")
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--workers", type=int, default=None,
                    help="processes drawing the synthetic inputs (1: in this process, e.g. under a profiler)")
    ap.add_argument("--inputs", default=None,
                    help="file of drawn inputs: loaded when it exists, else written after drawing")
    ap.add_argument("--extras-only", default="workloads,differentiation,modes,paper_shape",
                    help="comma list of side measurements to run (workloads, differentiation, modes, "
                         "paper_shape)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the sampler has no multi-GPU path (ligands and "
              "trajectories shard across GPUs with no communication); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    name = args.workload
    workers = synth.default_workers() if args.workers is None else max(1, args.workers)
    # inputs are drawn before the GPU is touched (the drawing pool forks no
    # process that holds the device)
    t0 = time.perf_counter()
    if args.inputs and os.path.exists(args.inputs):
        import pickle
        with open(args.inputs, "rb") as f:
            saved = pickle.load(f)   # written by this script (below)
        assert saved[0] == name, "inputs file holds another workload"
        pks, L, wl = saved[1:]
    else:
        pks, L, wl = synth.workload(name, workers=workers)
        if args.inputs:
            import pickle
            with open(args.inputs, "wb") as f:
                pickle.dump((name, pks, L, wl), f)
    print("workload %s drawn in %.1fs" % (name, time.perf_counter() - t0), file=sys.stderr, flush=True)

    import torch
    import paper_2510_24186_amd as D

    assert torch.cuda.is_available()
    free0, total_mem = torch.cuda.mem_get_info()
    T, S = wl["T"], wl["S"]
    adjoint = name == "C5"
    # host preparation (typing, torsion trees, pair lists, pass schedules)
    # and upload of the ligands: outside the timed steps, reported beside
    t_prep = time.perf_counter()
    H = D.dock_load_ligands(L.atom_off, L.element, L.n_h, L.xyz, L.bond_off, L.bonds, L.rotatable,
                            pocket_index=L.pocket_index)
    prep_s = time.perf_counter() - t_prep
    tab = ligand_table(D, H)
    evals_lig = T * (1 + S * (N_LOCAL + 1))
    evals_total = evals_lig * H.n
    flops_lig = np.array([flops_per_eval(*r) for r in tab]) * evals_lig
    print("workload %s: %d pockets, %d ligands (N %d-%d, mean %.1f; pairs mean %.0f), T %d, S %d, L %d, "
          "%d evals/step" % (name, len(pks), H.n, tab[:, 0].min(), tab[:, 0].max(), tab[:, 0].mean(),
                             tab[:, 1].mean(), T, S, N_LOCAL, evals_total), file=sys.stderr, flush=True)
    step = Step(D, pks, H, T, S, adjoint, args.graph)

    if args.calib_copy_mib:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the sampler kernel's counters in the same profiled run
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    min_free = free0
    for k in range(args.warmup):
        step(1000 + k)
        torch.cuda.synchronize()
        min_free = min(min_free, torch.cuda.mem_get_info()[0])
        print("warmup step %d done" % k, file=sys.stderr, flush=True)
    kern_ms, launch_stats = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    keep = None
    for k in range(args.steps):
        keep = step(k)
        kern_ms.append(D.dock_run_kernel_ms(step.run))     # waits for the sampler launches
        launch_stats.append(D.dock_run_launch_stats(step.run))
        min_free = min(min_free, torch.cuda.mem_get_info()[0])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    min_free = min(min_free, torch.cuda.mem_get_info()[0])
    print("timed %d steps in %.3fs" % (args.steps, t1 - t0), file=sys.stderr, flush=True)
    ms_step = 1e3 * (t1 - t0) / args.steps
    plan = D.dock_run_plan(step.run)
    if args.graph:
        # graph replays record no per-launch events: the roofline's launch
        # durations come from one more step of the same plan, launched eagerly
        keep = None
        eager = Step(D, pks, H, T, S, adjoint, 0)
        eager(2000)
        torch.cuda.synchronize()
        launch_stats = [D.dock_run_launch_stats(eager.run)]
        del eager
        print("eager step for the launch durations done", file=sys.stderr, flush=True)

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
                                              ligands=int(np.sum(lb == b)),
                                              atom_evals=float(np.sum(tab[lb == b, 0])) * T * S * (N_LOCAL + 1)))
            d["ms"].append(l["ms"])
    # lane buckets run concurrently (side streams): the dominant kernel is
    # the one with the most work, its duration as measured while overlapped
    dom = max(per_bucket.values(), key=lambda d: d["flop"])
    launch_ms = float(np.mean(dom["ms"]))
    achieved = dom["flop"] / (launch_ms * 1e-3) / 1e12
    kkey = "%d,%d,%d,%d" % (dom["lanes"], dom["apl"], dom["block"], dom["grid"])
    rec = kernel_record(name, kkey)
    sampler_ms = float(np.mean(kern_ms))
    roofline = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / PEAK_FP32_TFLOPS, 4),
                    traffic=None if rec is None else round(rec["hbm_bytes"]),
                    frac_of_nonpacked_peak=round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4),
                    kernel="sample_kernel<%d,%d,%d>" % (dom["lanes"], dom["apl"], dom["block"]),
                    launch_timing="eager step after the graph-replayed ones" if args.graph else "timed steps",
                    launch_ms=round(launch_ms, 3),
                    flop_per_launch=dom["flop"],
                    gather_bytes_per_launch=dom["atom_evals"] * 32.0,
                    gather_gbs=round(dom["atom_evals"] * 32.0 / (launch_ms * 1e-3) / 1e9, 1),
                    sampler_tflops=round(float(np.sum(flops_lig)) / (sampler_ms * 1e-3) / 1e12, 3),
                    buckets=[dict(lanes=d["lanes"], atoms_per_lane=d["apl"], ligands=d["ligands"],
                                  block=d["block"], grid=d["grid"], work_items=d["items"],
                                  ms=round(float(np.mean(d["ms"])), 3),
                                  tflops=round(d["flop"] / (np.mean(d["ms"]) * 1e-3) / 1e12, 3))
                             for d in per_bucket.values()])
    if rec is not None:
        # counters of the same kernel and workload (profiles/), per launch
        roofline.update(hbm_gbs=round(rec["hbm_bytes"] / (launch_ms * 1e-3) / 1e9, 1),
                        hbm_frac=round(rec["hbm_bytes"] / (launch_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                        l2_gbs=round(rec["l2_req"] * L2_LINE_BYTES / (launch_ms * 1e-3) / 1e9, 1),
                        l2_hit=rec.get("l2_hit"), valu_busy=rec.get("valu_busy"),
                        counters_ms=rec.get("ms"))

    evals_per_s = evals_total / (ms_step * 1e-3)
    pk_atoms = [len(p.xyz) for p in pks]
    sides = sorted({p.dims[0] for p in pks})
    out = dict(metric="pose score+grad evals/s and ligands docked/s, batched vs plain, 1 MI355X",
               value=round(evals_per_s, 1), unit="evals/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(ms_step, 3), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload="%s: %d pocket(s) of %d-%d receptor atoms, grids %s^3 x 8 types at %.3f A; "
                                    "%d ligands of %d-%d heavy atoms and 0-%d torsions%s; %d trajectories x %d "
                                    "MC steps x %d Adam steps; TRIDS physics terms%s"
                                    % (name, len(pks), min(pk_atoms), max(pk_atoms), "/".join(map(str, sides)),
                                       pks[0].spacing, H.n, tab[:, 0].min(), tab[:, 0].max(), tab[:, 2].max(),
                                       ", ligand k in pocket k mod %d" % len(pks) if len(pks) > 1 else "",
                                       T, S, N_LOCAL,
                                       "; adjoint of the summed best-pose energies to every pocket's per-term "
                                       "maps and weights in each step" if adjoint else ""),
                           n_pockets=len(pks), n_ligands=H.n, n_traj=T, n_steps=S, n_local=N_LOCAL,
                           evals_per_step=evals_total, adjoint=adjoint),
               ligands_per_s=round(H.n / (ms_step * 1e-3), 2),
               sampler_evals_per_s=round(evals_total / (sampler_ms * 1e-3), 1),
               sampler_ms=round(sampler_ms, 3),
               mem_peak_mb=round((free0 - min_free) / 2**20, 1),
               ligand_prep_s=round(prep_s, 2),
               ligand_prep_threads=min(64, int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)),
               mem_context="paper (Table 5): ~%d MB per docking on an RTX A6000" % PAPER_MEM_MB,
               roofline=roofline)
    del keep
    if not args.no_plain:
        pr = plain_rate(D, pks, L, H, T, S)
        out["plain"] = pr
        out["batched_vs_plain"] = round(out["ligands_per_s"] / pr["ligands_per_s"], 3)
        print("plain form: %.1f ligands/s" % pr["ligands_per_s"], file=sys.stderr, flush=True)
    if not args.no_extras:
        ex = {}
        which = set(args.extras_only.split(","))
        if "workloads" in which:
            others = [w for w in ("C4", "C2", "C1") if w != name]
            ex["workloads"] = {w: workload_rate(D, w, workers=workers, plain=w in ("C2", "C1")) for w in others}
            print("other workloads done", file=sys.stderr, flush=True)
        if "differentiation" in which:
            ex["differentiation"] = differentiation_rate(D)
        if "paper_shape" in which:
            ex["paper_shape"] = paper_shape_rate(D)
            print("paper-shaped dockings done", file=sys.stderr, flush=True)
        if "modes" in which:
            ex.update(extras(D, pks[0], L, T, S))
        out["extras"] = ex
        print("extras done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pks, L)
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
