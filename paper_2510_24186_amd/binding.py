"""ctypes binding of libdock.so with the C ABI's names.

Argument marshalling only: every computation happens in the HIP library.
Device arrays are torch CUDA tensors (HIP under ROCm); streams are torch
streams (default: the current stream).  If libdock.so is missing the import
fails loudly: there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdock.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libdock.so is not built (run `python paper_2510_24186_amd/build.py`): %s"
                      % LIB_PATH)
lib = C.CDLL(LIB_PATH)

DOCK_OK = 0
PRESET_TRIDS, PRESET_VINA = 0, 1
LOCAL_ADAM, LOCAL_LINESEARCH, LOCAL_SGD, LOCAL_RMSPROP, LOCAL_ADAGRAD, LOCAL_ADAMW = range(6)
FORM_PLAIN, FORM_BATCHED = 0, 1
INTER_GRID, INTER_DIRECT = 0, 1
ERRORS = {-1: "DOCK_E_ARG", -2: "DOCK_E_TOPOLOGY", -3: "DOCK_E_LIMIT", -4: "DOCK_E_OOM", -5: "DOCK_E_HIP"}

_p = C.c_void_p
_i32 = C.c_int32
_f32 = C.c_float


class PocketDesc(C.Structure):
    _fields_ = [("n_atoms", _i32), ("xyz", _p), ("type", _p), ("origin", _f32 * 3),
                ("spacing", _f32), ("dims", _i32 * 3), ("preset", _i32), ("weights", _p),
                ("keep_per_term", _i32), ("inter_mode", _i32), ("residue", _p), ("mdn_weight", _f32)]


class LigandDesc(C.Structure):
    _fields_ = [("n_ligands", _i32), ("atom_off", _p), ("element", _p), ("n_h", _p), ("xyz", _p),
                ("bond_off", _p), ("bonds", _p), ("rotatable", _p), ("box_min", _p),
                ("box_max", _p), ("pocket_index", _p), ("host_only", _i32)]


class LigandInfo(C.Structure):
    _fields_ = [("n_atoms", _i32), ("n_tors", _i32), ("n_frags", _i32), ("n_pairs", _i32),
                ("root", _i32), ("height", _i32), ("pocket", _i32), ("c0", _f32 * 3),
                ("box_min", _f32 * 3), ("box_max", _f32 * 3), ("n_pass", _i32), ("pass_lanes", _i32),
                ("pass_apl", _i32), ("pull_cap", _i32), ("stage_bytes", _i32)]


class SampleParams(C.Structure):
    _fields_ = [("n_traj", _i32), ("n_steps", _i32), ("n_local", _i32), ("local_opt", _i32),
                ("lr", _f32), ("beta1", _f32), ("beta2", _f32), ("eps", _f32), ("mc_beta", _f32),
                ("seed", C.c_uint32), ("form", _i32), ("use_graph", _i32),
                ("steps_per_launch", _i32), ("record_trace", _i32), ("lanes_per_pose", _i32),
                ("rms_alpha", _f32), ("weight_decay", _f32), ("trace_lig_stride", _i32),
                ("trace_traj", _i32)]


class RunView(C.Structure):
    _fields_ = [("n_ligands", _i32), ("n_traj", _i32), ("q_stride", _i32), ("step", _i32),
                ("q_cur", _p), ("E_cur", _p), ("q_best", _p), ("E_best", _p), ("n_evals", _p),
                ("trace", _p), ("trace_cap", _i32), ("trace_lig_stride", _i32), ("trace_traj", _i32),
                ("n_trace", _i32)]


def _sig(name, res, *args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("dock_last_error", C.c_char_p)
_sig("dock_abi_version", C.c_int)
_sig("dock_load_pocket", C.c_int, C.POINTER(PocketDesc), _p, C.POINTER(_p))
_sig("dock_pocket_maps", C.c_int, _p, _i32, C.POINTER(_p), C.POINTER(C.c_int64))
_sig("dock_pocket_rebuild", C.c_int, _p, _p)
_sig("dock_pocket_copy_maps", C.c_int, _p, _i32, _p, _p)
_sig("dock_pocket_terms", C.c_int, _p, C.POINTER(_i32), C.POINTER(_i32), _p)
_sig("dock_free_pocket", C.c_int, _p)
_sig("dock_load_ligands", C.c_int, C.POINTER(LigandDesc), _p, C.POINTER(_p))
_sig("dock_ligand_info", C.c_int, _p, _i32, C.POINTER(LigandInfo))
_sig("dock_ligand_topology", C.c_int, _p, _i32, _p, _p, _p, _p, _p, _p, _p)
_sig("dock_ligands_count", C.c_int, _p, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32),
     C.POINTER(C.c_int64))
_sig("dock_free_ligands", C.c_int, _p)
_sig("dock_score_grad", C.c_int, _p, _i32, _p, C.c_int64, _p, _p, _i32, _p, _p, _p, _i32, _p)
_sig("dock_score_terms", C.c_int, _p, _i32, _p, C.c_int64, _p, _p, _i32, _p, _i32, _p, _p, _p, _p)
_sig("dock_score_adjoint", C.c_int, _p, _i32, _p, C.c_int64, _p, _p, _i32, _p, _i32, _p, _p, _p, _p, _p,
     _p, _p, _i32, _p)
_sig("dock_sample_params_default", None, C.POINTER(SampleParams))
_sig("dock_sample", C.c_int, _p, _i32, _p, C.POINTER(SampleParams), _p, C.POINTER(_p))
_sig("dock_run_advance", C.c_int, _p, _i32, _p)
_sig("dock_run_restart", C.c_int, _p, C.c_uint32, _p)
_sig("dock_autotune", C.c_int, _p, _i32, _p, C.POINTER(SampleParams), _i32, _p)
_sig("dock_autotune_report", C.c_int, C.c_char_p, _i32, C.POINTER(_i32))
_sig("dock_autotune_clear", C.c_int)
_sig("dock_autotune_set", C.c_int, C.c_char_p, _i32, _i32, _i32, _i32, _f32)
_sig("dock_run_view_get", C.c_int, _p, C.POINTER(RunView))
_sig("dock_run_copy_state", C.c_int, _p, _p, _p, _p, _p, _p, _p, _p)
_sig("dock_run_set_state", C.c_int, _p, _p, _p, _p, _p, _i32, _p)
_sig("dock_run_kernel_ms", C.c_int, _p, C.POINTER(_f32))
_sig("dock_free_run", C.c_int, _p)
_sig("dock_philox", C.c_int, _p, C.c_uint32, C.c_uint32, C.c_int64, _p, _p)
_sig("dock_screen_rank", C.c_int, _p, C.c_int64, _i32, _i32, _p, _p, _p)
_sig("dock_screen_rank_noalloc", C.c_int, _p, C.c_int64, _i32, _i32, _p, _p, _p)
_sig("dock_pocket_map_adjoint", C.c_int, _p, _p, _p, _p, _p)
_sig("dock_ligands_set_mdn", C.c_int, _p, _i32, _i32, _p)
_sig("dock_best_poses", C.c_int, _p, _i32, _p, _p, _i32, _i32, _f32, _f32, _p, _p, _p, _p, _p, _i32,
     _p, _p)


class LaunchStat(C.Structure):
    _fields_ = [("bucket", _i32), ("lanes_per_pose", _i32), ("atoms_per_lane", _i32), ("block", _i32),
                ("grid", _i32), ("n_items", _i32), ("init", _i32), ("step_count", _i32), ("ms", _f32)]


_sig("dock_run_launch_stats", C.c_int, _p, C.POINTER(LaunchStat), _i32, C.POINTER(_i32))
_sig("dock_run_plan", C.c_int, _p, _p, _p, _p, C.POINTER(_i32))


class DockError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERRORS.get(code, code), msg))
        self.code = code


def _check(rc):
    if rc != DOCK_OK:
        raise DockError(rc, (lib.dock_last_error() or b"").decode())


def _np(a, dt):
    return np.ascontiguousarray(np.asarray(a, dtype=dt))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_p)


def _stream(stream):
    import torch
    if stream is None:
        return _p(torch.cuda.current_stream().cuda_stream)
    return _p(getattr(stream, "cuda_stream", stream))


def _dptr(t):
    return None if t is None else _p(t.data_ptr())


def _cuda_check(t, dtype, name):
    import torch
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError("%s must be a contiguous %s CUDA tensor" % (name, dtype))
    return t


# ------------------------------------------------------------------ pocket

class Pocket:
    def __init__(self, handle, preset, n_terms, dims, keep):
        self.handle = handle
        self.preset = preset
        self.n_terms = n_terms
        self.dims = tuple(dims)
        self.keep_per_term = keep

    def free(self):
        if self.handle:
            _check(lib.dock_free_pocket(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def dock_load_pocket(xyz, types, origin, spacing, dims, preset=PRESET_TRIDS, weights=None,
                     keep_per_term=False, inter_mode=INTER_GRID, residue=None, mdn_weight=1.0,
                     stream=None):
    xyz = _np(xyz, np.float32).reshape(-1, 3)
    types = _np(types, np.uint8)
    d = PocketDesc()
    d.n_atoms = len(xyz)
    d.xyz = _ptr(xyz)
    d.type = _ptr(types)
    d.origin = (_f32 * 3)(*[float(v) for v in origin])
    d.spacing = float(spacing)
    d.dims = (_i32 * 3)(*[int(v) for v in dims])
    d.preset = int(preset)
    w = None if weights is None else _np(weights, np.float32)
    d.weights = _ptr(w)
    d.keep_per_term = int(bool(keep_per_term))
    d.inter_mode = int(inter_mode)
    res = None if residue is None else _np(residue, np.int32)
    d.residue = _ptr(res)
    d.mdn_weight = float(mdn_weight)
    h = _p()
    _check(lib.dock_load_pocket(C.byref(d), _stream(stream), C.byref(h)))
    pr = _i32()
    nk = _i32()
    _check(lib.dock_pocket_terms(h, C.byref(pr), C.byref(nk), None))
    return Pocket(h, pr.value, nk.value, dims, bool(keep_per_term))


def dock_pocket_terms(pocket):
    pr, nk = _i32(), _i32()
    w = np.zeros(5, np.float32)
    _check(lib.dock_pocket_terms(pocket.handle, C.byref(pr), C.byref(nk), _ptr(w)))
    return pr.value, nk.value, w[:nk.value].copy()


def dock_pocket_rebuild(pocket, stream=None):
    """Builds the pocket's maps again in place on the stream."""
    _check(lib.dock_pocket_rebuild(pocket.handle, _stream(stream)))


def dock_pocket_maps(pocket, per_term=False, stream=None):
    """A copy of the maps as a CUDA tensor [8, (K,) nz, ny, nx]."""
    import torch
    nx, ny, nz = pocket.dims
    shape = (8, pocket.n_terms, nz, ny, nx) if per_term else (8, nz, ny, nx)
    out = torch.empty(shape, dtype=torch.float32, device="cuda")
    _check(lib.dock_pocket_copy_maps(pocket.handle, int(per_term), _dptr(out), _stream(stream)))
    return out


# ------------------------------------------------------------------ ligands

class Ligands:
    def __init__(self, handle, n, max_atoms, max_tors, total_atoms, host_only):
        self.handle = handle
        self.n = n
        self.max_atoms = max_atoms
        self.max_tors = max_tors
        self.total_atoms = total_atoms
        self.host_only = host_only

    @property
    def q_stride(self):
        return 6 + self.max_tors

    def free(self):
        if self.handle:
            _check(lib.dock_free_ligands(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def dock_load_ligands(atom_off, element, n_h, xyz, bond_off, bonds, rotatable, box_min=None,
                      box_max=None, pocket_index=None, host_only=False, stream=None):
    keep = dict(atom_off=_np(atom_off, np.int32), element=_np(element, np.uint8),
                n_h=_np(n_h, np.uint8), xyz=_np(xyz, np.float32).reshape(-1, 3),
                bond_off=_np(bond_off, np.int32), bonds=_np(bonds, np.int32).reshape(-1, 2),
                rotatable=_np(rotatable, np.uint8))
    d = LigandDesc()
    d.n_ligands = len(keep["atom_off"]) - 1
    for k, v in keep.items():
        setattr(d, k, _ptr(v))
    for k, v in (("box_min", box_min), ("box_max", box_max)):
        if v is not None:
            keep[k] = _np(v, np.float32).reshape(-1, 3)
            setattr(d, k, _ptr(keep[k]))
    if pocket_index is not None:
        keep["pocket_index"] = _np(pocket_index, np.int32)
        d.pocket_index = _ptr(keep["pocket_index"])
    d.host_only = int(bool(host_only))
    h = _p()
    _check(lib.dock_load_ligands(C.byref(d), None if host_only else _stream(stream), C.byref(h)))
    n, ma, mt, ta = _i32(), _i32(), _i32(), C.c_int64()
    _check(lib.dock_ligands_count(h, C.byref(n), C.byref(ma), C.byref(mt), C.byref(ta)))
    return Ligands(h, n.value, ma.value, mt.value, ta.value, bool(host_only))


def dock_ligands_set_mdn(L, params):
    """params: [total_atoms, n_res, n_gauss, 3] (pi, mu, sigma), caller atom order."""
    a = _np(params, np.float32)
    if a.ndim != 4 or a.shape[3] != 3:
        raise ValueError("params must be [total_atoms, n_res, n_gauss, 3]")
    _check(lib.dock_ligands_set_mdn(L.handle, a.shape[1], a.shape[2], _ptr(a)))


def dock_ligand_info(L, i):
    info = LigandInfo()
    _check(lib.dock_ligand_info(L.handle, int(i), C.byref(info)))
    return dict(n_atoms=info.n_atoms, n_tors=info.n_tors, n_frags=info.n_frags,
                n_pairs=info.n_pairs, root=info.root, height=info.height, pocket=info.pocket,
                c0=np.array(info.c0[:], np.float32), box_min=np.array(info.box_min[:], np.float32),
                box_max=np.array(info.box_max[:], np.float32), n_pass=info.n_pass,
                pass_lanes=info.pass_lanes, pass_apl=info.pass_apl, pull_cap=info.pull_cap,
                stage_bytes=info.stage_bytes)


def dock_ligand_topology(L, i):
    info = dock_ligand_info(L, i)
    n, F, nt, P = info["n_atoms"], info["n_frags"], info["n_tors"], info["n_pairs"]
    out = dict(type=np.zeros(n, np.uint8), atom_frag=np.zeros(n, np.int32),
               frag_parent=np.zeros(F, np.int32), tors_frag=np.zeros(nt, np.int32),
               tors_atoms=np.zeros((nt, 2), np.int32), pairs=np.zeros((P, 2), np.int32),
               bfs=np.zeros(F, np.int32))
    _check(lib.dock_ligand_topology(L.handle, int(i), _ptr(out["type"]), _ptr(out["atom_frag"]),
                                    _ptr(out["frag_parent"]), _ptr(out["tors_frag"]),
                                    _ptr(out["tors_atoms"]), _ptr(out["pairs"]), _ptr(out["bfs"])))
    out.update(info)
    return out


# ------------------------------------------------------------------ score

def _pocket_array(pockets):
    if isinstance(pockets, Pocket):
        pockets = [pockets]
    arr = (_p * len(pockets))(*[p.handle for p in pockets])
    return arr, len(pockets)


def dock_score_grad(pockets, L, pose_lig, q, want_grad=True, want_xyz=False, stream=None):
    """E [P], dE/dq [P, q_stride] (or None), xyz [P, max_atoms, 3] (or None)."""
    import torch
    pose_lig = _cuda_check(pose_lig, torch.int32, "pose_lig")
    q = _cuda_check(q, torch.float32, "q")
    n = pose_lig.shape[0]
    qs = q.shape[1]
    E = torch.empty(n, dtype=torch.float32, device=q.device)
    g = torch.zeros((n, qs), dtype=torch.float32, device=q.device) if want_grad else None
    xyz = (torch.zeros((n, L.max_atoms, 3), dtype=torch.float32, device=q.device)
           if want_xyz else None)
    arr, npk = _pocket_array(pockets)
    _check(lib.dock_score_grad(arr, npk, L.handle, n, _dptr(pose_lig), _dptr(q), qs, _dptr(E),
                               _dptr(g), _dptr(xyz), 3 * L.max_atoms, _stream(stream)))
    return E, g, xyz


# ------------------------------------------------------------------ differentiable form

def _ptr_array(ts, n):
    if ts is None:
        return None
    return (_p * n)(*[None if t is None else t.data_ptr() for t in ts])


def _terms_common(pockets, L, pose_lig, q, xyz, G, w):
    import torch
    if isinstance(pockets, Pocket):
        pockets = [pockets]
    arr, npk = _pocket_array(pockets)
    pose_lig = _cuda_check(pose_lig, torch.int32, "pose_lig")
    q = _cuda_check(q, torch.float32, "q")
    xyz = _cuda_check(xyz, torch.float32, "xyz")
    w = _cuda_check(w, torch.float32, "w")
    if G is not None:
        G = [None if t is None else _cuda_check(t, torch.float32, "G") for t in G]
    return pockets, arr, npk, pose_lig, q, xyz, G, w


def dock_score_terms(pockets, L, pose_lig, w, q=None, xyz=None, G=None, stream=None):
    """E of each pose with caller maps G (list per pocket, None = kept maps)
    and weights w [n_pockets, K]."""
    import torch
    pockets, arr, npk, pose_lig, q, xyz, G, w = _terms_common(pockets, L, pose_lig, q, xyz, G, w)
    n = pose_lig.shape[0]
    E = torch.empty(n, dtype=torch.float32, device=pose_lig.device)
    qs = q.shape[1] if q is not None else 0
    xs = 3 * L.max_atoms
    _check(lib.dock_score_terms(arr, npk, L.handle, n, _dptr(pose_lig), _dptr(q), qs, _dptr(xyz), xs,
                                _ptr_array(G, npk), _dptr(w), _dptr(E), _stream(stream)))
    return E


def dock_score_adjoint(pockets, L, pose_lig, w, dLdE, q=None, xyz=None, G=None, dLdG=None, dLdw=None,
                       dLdq=None, dLdx=None, deterministic=False, stream=None):
    """Accumulates (+=) gradients of sum_p dLdE[p] E_p into the given buffers
    (deterministic: bitwise repeatable dL/dG and dL/dw)."""
    import torch
    pockets, arr, npk, pose_lig, q, xyz, G, w = _terms_common(pockets, L, pose_lig, q, xyz, G, w)
    dLdE = _cuda_check(dLdE, torch.float32, "dLdE")
    n = pose_lig.shape[0]
    qs = q.shape[1] if q is not None else 0
    xs = 3 * L.max_atoms
    _check(lib.dock_score_adjoint(arr, npk, L.handle, n, _dptr(pose_lig), _dptr(q), qs, _dptr(xyz), xs,
                                  _ptr_array(G, npk), _dptr(w), _dptr(dLdE), _ptr_array(dLdG, npk),
                                  _dptr(dLdw), _dptr(dLdq), _dptr(dLdx), int(bool(deterministic)),
                                  _stream(stream)))


# ------------------------------------------------------------------ sampling

class Run:
    def __init__(self, handle, L, n_traj, pockets=()):
        self.handle = handle
        self.L = L  # the run reads the ligand and pocket handles until it is freed
        self.pockets = list(pockets)
        self.n_traj = n_traj

    def view(self):
        v = RunView()
        _check(lib.dock_run_view_get(self.handle, C.byref(v)))
        return v

    def free(self):
        if self.handle:
            lib.dock_free_run(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sample_params(**kw):
    p = SampleParams()
    lib.dock_sample_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError("unknown sampler parameter %s" % k)
        setattr(p, k, v)
    return p


def dock_sample(pockets, L, stream=None, **params):
    p = sample_params(**params)
    arr, npk = _pocket_array(pockets)
    h = _p()
    _check(lib.dock_sample(arr, npk, L.handle, C.byref(p), _stream(stream), C.byref(h)))
    return Run(h, L, p.n_traj, [pockets] if isinstance(pockets, Pocket) else pockets)


def dock_autotune(pockets, L, trial_steps=2, stream=None, **params):
    """Tune group width and block size per lane configuration; returns the cache."""
    import json
    p = sample_params(**params)
    arr, npk = _pocket_array(pockets)
    _check(lib.dock_autotune(arr, npk, L.handle, C.byref(p), int(trial_steps), _stream(stream)))
    return dock_autotune_report()


def dock_autotune_report():
    import json
    need = _i32()
    _check(lib.dock_autotune_report(None, 0, C.byref(need)))
    buf = C.create_string_buffer(need.value)
    _check(lib.dock_autotune_report(buf, need.value, C.byref(need)))
    return json.loads(buf.value.decode())


def dock_autotune_clear():
    _check(lib.dock_autotune_clear())


def dock_autotune_save(path):
    """Writes the autotuner cache (every (arch, lanes, atoms per lane) entry)
    to a JSON file."""
    import json
    with open(path, "w") as f:
        json.dump(dock_autotune_report(), f, indent=1)


def dock_autotune_load(path):
    """Restores cache entries saved by dock_autotune_save; returns how many."""
    import json
    entries = json.load(open(path))
    for e in entries:
        _check(lib.dock_autotune_set(str(e["arch"]).encode(), int(e["lanes"]), int(e["atoms_per_lane"]),
                                     int(e["chosen_lanes"]), int(e["block"]), float(e.get("trial_ms", 0.0))))
    return len(entries)


def dock_run_advance(run, n_steps, stream=None):
    _check(lib.dock_run_advance(run.handle, int(n_steps), _stream(stream)))


def dock_run_restart(run, seed, stream=None):
    """Redraws the initial poses with `seed` and reruns the run's MC steps in
    place (same results as a new dock_sample with that seed)."""
    _check(lib.dock_run_restart(run.handle, int(seed) & 0xFFFFFFFF, _stream(stream)))


def dock_run_state(run, trace=False, stream=None):
    """Copies of the run state as CUDA tensors."""
    import torch
    v = run.view()
    nt = v.n_ligands * v.n_traj
    dev = "cuda"
    out = dict(q_cur=torch.empty((v.n_ligands, v.n_traj, v.q_stride), device=dev),
               E_cur=torch.empty((v.n_ligands, v.n_traj), device=dev),
               q_best=torch.empty((v.n_ligands, v.n_traj, v.q_stride), device=dev),
               E_best=torch.empty((v.n_ligands, v.n_traj), device=dev),
               n_evals=torch.empty((v.n_ligands, v.n_traj), dtype=torch.int32, device=dev),
               step=v.step, q_stride=v.q_stride)
    tr = None
    if trace:
        if not v.trace_cap:
            raise ValueError("run was not created with record_trace")
        # [logged ligand (l / trace_lig_stride), trajectory < trace_traj, row, column]
        tr = torch.empty((v.n_trace // v.trace_traj, v.trace_traj, v.trace_cap, 2 * v.q_stride + 1), device=dev)
        out["trace"] = tr
    _check(lib.dock_run_copy_state(run.handle, _dptr(out["q_cur"]), _dptr(out["E_cur"]),
                                   _dptr(out["q_best"]), _dptr(out["E_best"]),
                                   _dptr(out["n_evals"]), _dptr(tr), _stream(stream)))
    del nt
    return out


def dock_run_set_state(run, q_cur, E_cur, q_best, E_best, step, stream=None):
    _check(lib.dock_run_set_state(run.handle, _dptr(q_cur), _dptr(E_cur), _dptr(q_best),
                                  _dptr(E_best), int(step), _stream(stream)))


def dock_run_launch_stats(run):
    n = _i32()
    _check(lib.dock_run_launch_stats(run.handle, None, 0, C.byref(n)))
    arr = (LaunchStat * max(1, n.value))()
    _check(lib.dock_run_launch_stats(run.handle, arr, n.value, C.byref(n)))
    return [{f: getattr(arr[i], f) for f, _ in LaunchStat._fields_} for i in range(n.value)]


def dock_run_plan(run):
    nb = _i32()
    _check(lib.dock_run_plan(run.handle, None, None, None, C.byref(nb)))
    lb = np.zeros(run.L.n, np.int32)
    lanes = np.zeros(max(1, nb.value), np.int32)
    apl = np.zeros(max(1, nb.value), np.int32)
    _check(lib.dock_run_plan(run.handle, _ptr(lb), _ptr(lanes), _ptr(apl), C.byref(nb)))
    return dict(lig_bucket=lb, lanes=lanes[:nb.value], apl=apl[:nb.value])


def dock_run_kernel_ms(run):
    ms = _f32()
    _check(lib.dock_run_kernel_ms(run.handle, C.byref(ms)))
    return ms.value


def dock_best_poses(L, n_traj, E_best, q_best, top_n=8, rmsd_cluster=1.0, w_tor=0.01,
                    want_xyz=True, stream=None):
    import torch
    E_best = _cuda_check(E_best.contiguous(), torch.float32, "E_best")
    q_best = _cuda_check(q_best.contiguous(), torch.float32, "q_best")
    qs = q_best.shape[-1]
    n = L.n
    dev = E_best.device
    out = dict(E=torch.empty((n, top_n), device=dev), E_screen=torch.empty((n, top_n), device=dev),
               q=torch.empty((n, top_n, qs), device=dev),
               idx=torch.empty((n, top_n), dtype=torch.int32, device=dev),
               xyz=torch.zeros((n, top_n, L.max_atoms, 3), device=dev) if want_xyz else None,
               n=torch.empty(n, dtype=torch.int32, device=dev))
    _check(lib.dock_best_poses(L.handle, int(n_traj), _dptr(E_best), _dptr(q_best), qs, int(top_n),
                               float(rmsd_cluster), float(w_tor), _dptr(out["E"]),
                               _dptr(out["E_screen"]), _dptr(out["q"]), _dptr(out["idx"]),
                               _dptr(out["xyz"]), 3 * L.max_atoms, _dptr(out["n"]), _stream(stream)))
    return out


def dock_philox(counters, k0, k1, stream=None):
    """counters: int32/uint32-valued CUDA tensor [n, 4] -> [n, 4] outputs (int32 view)."""
    import torch
    c = counters.to(torch.int32).contiguous()
    out = torch.empty_like(c)
    _check(lib.dock_philox(_dptr(c), int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF, c.shape[0],
                           _dptr(out), _stream(stream)))
    return out


def dock_screen_rank(scores, top_k, stride=1, stream=None):
    """scores: float32 CUDA tensor holding one score per ligand every `stride`
    elements -> (score [top_k], ligand index [top_k]), ascending."""
    import torch
    s = _cuda_check(scores.contiguous(), torch.float32, "scores")
    n = (s.numel() + stride - 1) // stride
    out_s = torch.empty(int(top_k), dtype=torch.float32, device=s.device)
    out_i = torch.empty(int(top_k), dtype=torch.int32, device=s.device)
    _check(lib.dock_screen_rank(_dptr(s), n, int(stride), int(top_k), _dptr(out_s), _dptr(out_i),
                                _stream(stream)))
    return out_s, out_i


def dock_screen_rank_noalloc(scores, top_k, score_out, lig_out, stride=1, n=None, stream=None):
    """dock_screen_rank into caller-allocated outputs (float32 / int32 CUDA
    tensors of at least top_k entries) with the library's static scratch:
    the call itself allocates nothing.  n defaults to the number of scores
    in `scores` at `stride`."""
    import torch
    s = _cuda_check(scores, torch.float32, "scores")
    _cuda_check(score_out, torch.float32, "score_out")
    _cuda_check(lig_out, torch.int32, "lig_out")
    if score_out.numel() < top_k or lig_out.numel() < top_k:
        raise ValueError("outputs hold fewer than top_k entries")
    if n is None:
        n = (s.numel() + stride - 1) // stride
    _check(lib.dock_screen_rank_noalloc(_dptr(s), int(n), int(stride), int(top_k), _dptr(score_out),
                                        _dptr(lig_out), _stream(stream)))
    return score_out, lig_out


def dock_pocket_map_adjoint(pocket, dLdG, dLdxyz=None, dLdtheta=None, stream=None):
    """dLdG: float32 CUDA tensor [8, 3, nz, ny, nx]; accumulates into dLdxyz
    (float32 [n_atoms, 3]) and dLdtheta (float64 [13]) when given."""
    import torch
    g = _cuda_check(dLdG.contiguous(), torch.float32, "dLdG")
    if dLdxyz is not None:
        _cuda_check(dLdxyz, torch.float32, "dLdxyz")
    if dLdtheta is not None:
        _cuda_check(dLdtheta, torch.float64, "dLdtheta")
    _check(lib.dock_pocket_map_adjoint(pocket.handle, _dptr(g), _dptr(dLdxyz) if dLdxyz is not None else None,
                                       _dptr(dLdtheta) if dLdtheta is not None else None, _stream(stream)))


def dock_abi_version():
    return lib.dock_abi_version()
