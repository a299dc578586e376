"""The C ABI from C: tests/c/dock_c_example.c (C99, plain pointers, device
memory from the HIP runtime) builds against include/dock.h and libdock.so
with strict warnings, and on the GPU its scores, gradients, sampler results
and best poses equal the Python binding's bit for bit on the same inputs
(same library, same kernels, same seed)."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import synth
from oracle import params as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2510_24186_amd")
SRC = os.path.join(ROOT, "tests", "c", "dock_c_example.c")


def _build(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    if not os.path.exists(os.path.join(PKG, "libdock.so")):
        pytest.skip("libdock.so not built")
    exe = str(tmp_path / "dock_c_example")
    cmd = [cc, "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-isystem", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"), SRC, "-o", exe,
           "-L", PKG, "-ldock", "-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath," + PKG,
           "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def test_c_example_builds_and_links(tmp_path):
    _build(tmp_path)


def _problem():
    pk = synth.make_pocket(300, grid=32, seed=3)
    L = synth.pack_ligands([synth.make_ligand(n, t, np.random.default_rng(70 + n)) for n, t in
                            ((6, 1), (14, 3), (23, 5), (40, 6))])
    L.pocket_index = np.zeros(L.n_ligands, np.int32)
    return pk, L


def _write_input(path, pk, L, w, pose_lig, Q, T, S, seed, top_n):
    i32 = lambda *v: struct.pack("<%di" % len(v), *v)  # noqa: E731
    with open(path, "wb") as f:
        f.write(i32(len(pk.xyz), P.PRESET_TRIDS, *[int(d) for d in pk.dims], len(w)))
        f.write(np.asarray(list(pk.origin) + [pk.spacing], "<f4").tobytes())
        f.write(np.asarray(w, "<f4").tobytes())
        f.write(np.asarray(pk.xyz, "<f4").tobytes())
        f.write(np.asarray(pk.type, np.uint8).tobytes())
        f.write(i32(L.n_ligands, int(L.atom_off[-1]), int(L.bond_off[-1])))
        f.write(np.asarray(L.atom_off, "<i4").tobytes())
        f.write(np.asarray(L.element, np.uint8).tobytes())
        f.write(np.asarray(L.n_h, np.uint8).tobytes())
        f.write(np.asarray(L.xyz, "<f4").tobytes())
        f.write(np.asarray(L.bond_off, "<i4").tobytes())
        f.write(np.asarray(L.bonds, "<i4").tobytes())
        f.write(np.asarray(L.rotatable, np.uint8).tobytes())
        f.write(i32(len(pose_lig), Q.shape[1]))
        f.write(np.asarray(pose_lig, "<i4").tobytes())
        f.write(np.asarray(Q, "<f4").tobytes())
        f.write(i32(T, S, seed, top_n))


@pytest.mark.gpu
def test_c_example_matches_binding(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import _gpu as G
    D = G.lib()
    exe = _build(tmp_path)
    pk, L = _problem()
    w = G.weights32(P.PRESET_TRIDS)
    p = G.load_pocket(pk, P.PRESET_TRIDS, w)
    H = G.load_ligands(L)
    rng = np.random.default_rng(12)
    qs = H.q_stride
    pose_lig = np.repeat(np.arange(L.n_ligands, dtype=np.int32), 8)
    Q = np.zeros((len(pose_lig), qs), np.float32)
    Q[:, :3] = rng.normal(size=(len(pose_lig), 3)).astype(np.float32) * 2.0
    Q[:, 3:] = rng.uniform(-np.pi, np.pi, size=(len(pose_lig), qs - 3)).astype(np.float32)
    T, S, seed, top_n = 64, 6, 21, 4
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write_input(fin, pk, L, w, pose_lig, Q, T, S, seed, top_n)
    G.say("C consumer:", L.n_ligands, "ligands,", len(pose_lig), "poses,", T, "trajectories x", S, "steps")
    r = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    n = L.n_ligands
    sizes = [len(pose_lig), len(pose_lig) * qs, n * T, n * top_n, n * top_n, n]
    raw = open(fout, "rb").read()
    assert len(raw) == 4 * sum(sizes)
    parts, off = [], 0
    for k, m in enumerate(sizes):
        parts.append(np.frombuffer(raw, "<i4" if k >= 4 else "<f4", m, off))
        off += 4 * m
    cE, cg, cEb, cbE, cbi, cbn = parts
    # the same calls through the Python binding
    E, g, _ = D.dock_score_grad(p, H, torch.tensor(pose_lig, device="cuda"), torch.tensor(Q, device="cuda"))
    run = D.dock_sample(p, H, n_traj=T, n_steps=S, seed=seed, form=D.FORM_BATCHED)
    st = D.dock_run_state(run)
    best = D.dock_best_poses(H, T, st["E_best"], st["q_best"], top_n=top_n, want_xyz=False)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(cE, E.cpu().numpy())
    np.testing.assert_array_equal(cg, g.cpu().numpy().ravel())
    np.testing.assert_array_equal(cEb, st["E_best"].cpu().numpy().ravel())
    np.testing.assert_array_equal(cbE, best["E"].cpu().numpy().ravel())
    np.testing.assert_array_equal(cbi, best["idx"].cpu().numpy().ravel())
    np.testing.assert_array_equal(cbn, best["n"].cpu().numpy())
    assert np.all(np.isfinite(cE)) and np.all(cbn >= 1)
    run.free()
