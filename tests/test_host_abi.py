"""CPU tests of libdock's host half (no GPU calls).

* the shared library loads and exports every function include/dock.h declares;
* host-side typing, fragments, torsion tree, pair list, root, c0 and box are
  bit-exact against the FP64 oracle on generated ligands;
* invalid inputs return the documented error codes.
"""
import os
import re

import numpy as np
import pytest

import synth
from oracle import topology

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

D = pytest.importorskip("paper_2510_24186_amd")


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "dock.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(dock_\w+)\s*\(", txt, flags=re.M)))


def test_every_declared_symbol_is_exported():
    names = _declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(D.lib, n), n
    assert D.dock_abi_version() == 2


def _load(L, host_only=True, **kw):
    return D.dock_load_ligands(L.atom_off, L.element, L.n_h, L.xyz, L.bond_off, L.bonds, L.rotatable,
                               host_only=host_only, **kw)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_topology_bit_exact_against_oracle(seed):
    L = synth.make_ligands(60, lambda r: int(r.integers(1, 71)), lambda r: int(r.integers(0, 16)),
                           seed=100 + seed)
    H = _load(L)
    for i in range(L.n_ligands):
        o = topology.from_ligands(L, i)
        g = D.dock_ligand_topology(H, i)
        assert g["n_atoms"] == o.n_atoms and g["n_tors"] == o.n_tors and g["n_frags"] == o.n_frags
        assert np.array_equal(g["type"], o.types)
        assert np.array_equal(g["atom_frag"], o.atom_frag)
        assert np.array_equal(g["frag_parent"], o.frag_parent)
        assert np.array_equal(g["bfs"], o.bfs)
        assert np.array_equal(g["tors_frag"], o.tors_frag)
        assert np.array_equal(g["tors_atoms"], np.stack([o.tors_a, o.tors_b], 1).reshape(-1, 2))
        assert np.array_equal(g["pairs"], o.pairs)
        assert g["root"] == o.root and g["height"] == o.height
        assert np.array_equal(g["c0"], o.c0.astype(np.float32))
        assert np.array_equal(g["box_min"], o.box_min.astype(np.float32))
        assert np.array_equal(g["box_max"], o.box_max.astype(np.float32))


def test_supplied_box_and_pocket_index():
    L = synth.make_ligands(3, 12, 3, seed=7)
    bmin = np.full((3, 3), -2.0, np.float32)
    bmax = np.full((3, 3), 2.5, np.float32)
    H = _load(L, box_min=bmin, box_max=bmax, pocket_index=[0, 2, 1])
    for i in range(3):
        info = D.dock_ligand_info(H, i)
        assert np.all(info["box_min"] == -2.0) and np.all(info["box_max"] == 2.5)
    assert [D.dock_ligand_info(H, i)["pocket"] for i in range(3)] == [0, 2, 1]


def _one(element, n_h, xyz, bonds, rot):
    n = len(element)
    return D.dock_load_ligands([0, n], element, n_h, xyz, [0, len(bonds)], bonds, rot, host_only=True)


def _code(fn):
    with pytest.raises(D.DockError) as e:
        fn()
    return e.value.code


def test_error_codes():
    xyz = np.arange(12, dtype=np.float32).reshape(4, 3)
    # rotatable bond inside a ring
    assert _code(lambda: _one([0] * 3, [2] * 3, xyz[:3], [(0, 1), (1, 2), (2, 0)], [1, 0, 0])) == -2
    # disconnected
    assert _code(lambda: _one([0] * 4, [2] * 4, xyz, [(0, 1), (2, 3)], [0, 0])) == -2
    # NaN coordinate
    bad = xyz.copy(); bad[1, 1] = np.nan
    assert _code(lambda: _one([0] * 4, [2] * 4, bad, [(0, 1), (1, 2), (2, 3)], [0, 0, 0])) == -2
    # too many atoms
    n = 129
    big = np.zeros((n, 3), np.float32); big[:, 0] = np.arange(n) * 1.5
    assert _code(lambda: _one([0] * n, [2] * n, big, [(i, i + 1) for i in range(n - 1)], [0] * (n - 1))) == -3
    # unknown element
    assert _code(lambda: _one([9, 0], [0, 0], xyz[:2], [(0, 1)], [0])) == -1
    # inverted box
    assert _code(lambda: D.dock_load_ligands([0, 2], [0, 0], [3, 3], xyz[:2], [0, 1], [(0, 1)], [0],
                                             box_min=[[1, 1, 1]], box_max=[[0, 0, 0]],
                                             host_only=True)) == -1
    # host-only handles cannot be scored
    H = _one([0, 0], [3, 3], xyz[:2], [(0, 1)], [0])
    assert D.dock_ligand_info(H, 0)["n_atoms"] == 2
    with pytest.raises(D.DockError):
        D.dock_ligand_info(H, 5)


def test_residue_and_mixture_argument_errors():
    # pocket residue indices must cover 0 .. n_res - 1 (checked before any
    # device work); mixture parameters need a device-backed ligand handle
    xyz = np.arange(12, dtype=np.float32).reshape(4, 3)
    types = np.zeros(4, np.uint8)
    for residue in ([0, 0, 2, 2], [0, -1, 1, 1]):
        assert _code(lambda: D.dock_load_pocket(xyz, types, [0, 0, 0], 0.5, (4, 4, 4),
                                                residue=np.array(residue, np.int32), stream=0)) == -1
    H = _one([0, 0], [3, 3], xyz[:2], [(0, 1)], [0])
    assert _code(lambda: D.dock_ligands_set_mdn(H, np.ones((2, 3, 2, 3), np.float32))) == -1


def test_noalloc_rank_refuses_sizes_beyond_its_scratch():
    # checked on the host before any device work: ceil(n / 2048) * top_k
    # above the static scratch, bad top_k, null outputs
    cap = 262144
    fake = 4096  # a non-null address that the refused calls never touch
    f = D.lib.dock_screen_rank_noalloc
    n = 2048 * (cap // 1024) + 1  # 257 blocks x 1024 kept
    assert f(fake, n, 1, 1024, fake, fake, None) == -3
    assert f(fake, n, 1, 1021, fake, fake, None) == -3  # 257 x 1021 > 262,144
    assert f(fake, 10, 1, 0, fake, fake, None) == -1
    assert f(fake, 10, 1, 1025, fake, fake, None) == -1
    assert f(fake, 10, 1, 8, None, fake, None) == -1
    assert f(fake, -1, 1, 8, fake, fake, None) == -1


def test_autotune_cache_saved_and_restored(tmp_path):
    # no device work: the cache is host state
    D.dock_autotune_clear()
    assert D.dock_autotune_report() == []
    D.lib.dock_autotune_set(b"gfx950", 32, 2, 32, 128, 1.5)
    assert D.lib.dock_autotune_set(b"gfx950", 16, 1, 32, 256, 2.0) == 0
    assert D.lib.dock_autotune_set(b"gfx950", 32, 2, 64, 256, 1.0) == -1   # two per lane keeps its width
    assert D.lib.dock_autotune_set(b"gfx950", 64, 1, 64, 32, 1.0) == -1    # block smaller than a group
    assert D.lib.dock_autotune_set(b"", 64, 1, 64, 64, 1.0) == -1
    before = D.dock_autotune_report()
    path = str(tmp_path / "tune.json")
    D.dock_autotune_save(path)
    D.dock_autotune_clear()
    assert D.dock_autotune_load(path) == 2
    assert D.dock_autotune_report() == before
    assert {(e["lanes"], e["atoms_per_lane"], e["chosen_lanes"], e["block"]) for e in before} == \
        {(32, 2, 32, 128), (16, 1, 32, 256)}
    D.dock_autotune_clear()


def test_parallel_preparation_matches_one_thread(monkeypatch):
    # ligand preparation and packing run on OMP_NUM_THREADS host threads;
    # the result must not depend on how many
    L = synth.make_ligands(700, lambda r: int(r.integers(5, 71)), lambda r: int(r.integers(0, 16)), seed=8)
    got = []
    for nt in ("1", "6"):
        monkeypatch.setenv("OMP_NUM_THREADS", nt)
        H = D.dock_load_ligands(L.atom_off, L.element, L.n_h, L.xyz, L.bond_off, L.bonds, L.rotatable,
                                host_only=True)
        got.append([D.dock_ligand_topology(H, i) for i in range(L.n_ligands)])
    for a, b in zip(*got):
        assert a.keys() == b.keys()
        for k in a:
            assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def test_parallel_preparation_reports_the_first_failing_ligand(monkeypatch):
    # ligands 3 and 5 (of 8) are disconnected: the error names ligand 3
    monkeypatch.setenv("OMP_NUM_THREADS", "4")
    parts = [synth.make_ligand(6, 1, np.random.default_rng(k)) for k in range(8)]
    for k in (3, 5):
        parts[k]["bonds"] = parts[k]["bonds"][:-1]
        parts[k]["rotatable"] = parts[k]["rotatable"][:-1]
    L = synth.pack_ligands(parts)
    with pytest.raises(D.DockError) as ei:
        D.dock_load_ligands(L.atom_off, L.element, L.n_h, L.xyz, L.bond_off, L.bonds, L.rotatable,
                            host_only=True)
    assert ei.value.code == -2 and "ligand 3:" in str(ei.value)
