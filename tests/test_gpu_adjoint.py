"""GPU tests of the differentiable form (hand-written adjoint kernel behind a
torch.autograd.Function) against the FP64 oracle.

* tiny pocket, both presets, poses as DOFs and as coordinates: E, dL/dG at
  every node, dL/dw, dL/dq, dL/dx against the oracle's analytic adjoint;
* the differentiation workload (2,000-atom pocket, Vina-form terms, weights
  ~ N(w0, 0.1|w0|), 64 ligands x 32 poses): per-pose E and dL/dq on sampled
  poses against the oracle, dL/dx against FP64 central differences
  (h = 1e-4), and at full size the exact identities
  sum_nodes dL/dG[t][k] = w_k * sum_p dLdE_p * (#atoms of type t in pose p)
  and dL/dw from the forward's linearity in w.
"""
import numpy as np
import pytest

import synth
from oracle import topology, maps as MAPS, score as SC, adjoint as ADJ, fk as FK, params as P
from tests import _gpu as G
from tests._tiny import tiny_pocket, tiny_ligand

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G.lib()


def _poses(L, H, topos, n_per, rng):
    qs = H.q_stride
    Q, lig = [], []
    for i, t in enumerate(topos):
        q = np.zeros((n_per, qs), np.float32)
        q[: n_per // 2, :t.n_dof] = G.poses_for(t, n_per // 2, rng, "near")
        q[n_per // 2:, :t.n_dof] = G.poses_for(t, n_per - n_per // 2, rng, "uniform")
        Q.append(q)
        lig += [i] * n_per
    return np.concatenate(Q), np.array(lig, np.int32)


def _lazy_terms(pk, preset, grid, xs):
    """Oracle per-term maps filled at the nodes the given coordinates touch."""
    nx, ny, nz = pk.dims
    Gd = np.zeros((8, P.n_terms(preset), nz, ny, nx))
    c = np.concatenate([SC.cells(grid, x.reshape(-1, 3)) for x in xs])
    idx = []
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                idx.append(((c[:, 2] + dz) * ny + c[:, 1] + dy) * nx + c[:, 0] + dx)
    flat = np.unique(np.concatenate(idx))
    vals = MAPS.build_maps(pk, preset, nodes=flat)
    z, rem = np.divmod(flat, nx * ny)
    y, x = np.divmod(rem, nx)
    Gd[:, :, z, y, x] = vals
    return Gd


@pytest.mark.parametrize("det", [0, 1])
@pytest.mark.parametrize("preset", [P.PRESET_TRIDS, P.PRESET_VINA])
@pytest.mark.parametrize("mode", ["q", "xyz"])
def test_adjoint_tiny_against_oracle(D, preset, mode, det):
    G.say("adjoint tiny preset", preset, "mode", mode, "deterministic", det)
    pk = tiny_pocket(n=30, radius=7.0, grid=32)
    grid = SC.grid_of(pk)
    K = P.n_terms(preset)
    rng = np.random.default_rng(10 + preset)
    w = (np.asarray(P.default_weights(preset)) * (1 + 0.1 * rng.normal(size=K))).astype(np.float32)
    p = G.load_pocket(pk, preset, w, keep=True)
    L = synth.pack_ligands([synth.make_ligand(n, t, np.random.default_rng(n)) for n, t in
                            ((5, 1), (9, 3), (14, 4))])
    L.pocket_index = np.zeros(L.n_ligands, np.int32)
    H = G.load_ligands(L)
    topos = [topology.from_ligands(L, i) for i in range(L.n_ligands)]
    Q, lig = _poses(L, H, topos, 8, rng)
    dLdE = rng.normal(size=len(Q)).astype(np.float32)
    Gref = MAPS.build_maps(pk, preset)
    Ggpu = D.dock_pocket_maps(p, per_term=True)
    wt = torch.tensor(w[None], device="cuda")
    lt = torch.tensor(lig, device="cuda")
    X = np.zeros((len(Q), H.max_atoms, 3), np.float32)
    for i, t in enumerate(topos):
        X[lig == i, :t.n_atoms] = FK.fk(t, Q[lig == i, :t.n_dof].astype(np.float64)).astype(np.float32)
    kw = dict(q=torch.tensor(Q, device="cuda")) if mode == "q" else dict(xyz=torch.tensor(X, device="cuda"))
    E = D.dock_score_terms(p, H, lt, wt, G=[Ggpu], **kw).cpu().numpy()
    dLdG = torch.zeros_like(Ggpu)
    dLdw = torch.zeros_like(wt)
    dLdq = torch.zeros((len(Q), H.q_stride), device="cuda") if mode == "q" else None
    dLdx = torch.zeros((len(Q), H.max_atoms, 3), device="cuda")
    D.dock_score_adjoint(p, H, lt, wt, torch.tensor(dLdE, device="cuda"), G=[Ggpu], dLdG=[dLdG], dLdw=dLdw,
                         dLdq=dLdq, dLdx=dLdx, deterministic=det, **kw)
    torch.cuda.synchronize()
    if det:
        # a second deterministic call repeats every output bit for bit
        again = [torch.zeros_like(t) if t is not None else None for t in (dLdG, dLdw, dLdq, dLdx)]
        D.dock_score_adjoint(p, H, lt, wt, torch.tensor(dLdE, device="cuda"), G=[Ggpu], dLdG=[again[0]],
                             dLdw=again[1], dLdq=again[2], dLdx=again[3], deterministic=1, **kw)
        torch.cuda.synchronize()
        for a, b in zip((dLdG, dLdw, dLdq, dLdx), again):
            if a is not None:
                assert torch.equal(a, b)
    dLdG = dLdG.cpu().numpy().astype(np.float64)
    ref_G = np.zeros_like(Gref)
    ref_w = np.zeros(K)
    for i, t in enumerate(topos):
        sel = lig == i
        if mode == "q":
            A = ADJ.adjoint(Gref, w, grid, preset, t, dLdE[sel], q=Q[sel, :t.n_dof].astype(np.float64))
            Er = ADJ.energy(Gref, w, grid, preset, t, q=Q[sel, :t.n_dof].astype(np.float64))
        else:
            xs = X[sel, :t.n_atoms].astype(np.float64)
            A = ADJ.adjoint(Gref, w, grid, preset, t, dLdE[sel], x=xs)
            Er = ADJ.energy(Gref, w, grid, preset, t, x=xs)
        ref_G += A["dLdG"]
        ref_w += A["dLdw"]
        sc = SC.Scorer(pk, preset, weights=w.astype(np.float64), G=Gref)
        S_abs = sc.score(t, Q[sel, :t.n_dof].astype(np.float64))["S_abs"] if mode == "q" else np.abs(Er) + 1
        assert np.all(np.abs(E[sel] - Er) <= 1e-5 * np.maximum(np.abs(Er), S_abs)), (E[sel], Er)
        gx = dLdx.cpu().numpy()[sel, :t.n_atoms]
        sx = np.linalg.norm(A["dLdx"].reshape(sel.sum(), -1), axis=1)
        err = np.linalg.norm((gx - A["dLdx"]).reshape(sel.sum(), -1), axis=1)
        assert np.all(err <= 1e-4 * sx + 1e-4), (err, sx)
        if mode == "q":
            gq = dLdq.cpu().numpy()[sel, :t.n_dof]
            err = np.linalg.norm(gq - A["dLdq"], axis=1)
            assert np.all(err <= 1e-4 * np.linalg.norm(A["dLdq"], axis=1) + 1e-4)
    np.testing.assert_allclose(dLdw.cpu().numpy()[0], ref_w, rtol=1e-5, atol=1e-4 * np.abs(ref_w).max())
    scale = np.abs(ref_G).max()
    G.say("dLdG max |diff| / max |ref|", np.abs(dLdG - ref_G).max() / scale)
    assert np.abs(dLdG - ref_G).max() <= 1e-5 * scale + 1e-7
    # no contribution leaks outside the nodes the oracle touches
    assert np.all(dLdG[np.abs(ref_G) == 0] == 0) or np.abs(dLdG[np.abs(ref_G) == 0]).max() < 1e-6 * scale


def test_autograd_function_matches_direct_adjoint(D):
    pk = tiny_pocket(n=30, radius=7.0, grid=32)
    preset = P.PRESET_VINA
    w = np.asarray(P.VINA_WEIGHTS, np.float32)
    p = G.load_pocket(pk, preset, w, keep=True)
    L = tiny_ligand(9, 3, seed=4)
    L.pocket_index = np.zeros(1, np.int32)
    H = G.load_ligands(L)
    topo = topology.from_ligands(L, 0)
    rng = np.random.default_rng(3)
    Q = np.zeros((16, H.q_stride), np.float32)
    Q[:, :topo.n_dof] = G.poses_for(topo, 16, rng, "near")
    Gt = D.dock_pocket_maps(p, per_term=True).requires_grad_(True)
    wt = torch.tensor(w[None], device="cuda", requires_grad=True)
    qt = torch.tensor(Q, device="cuda", requires_grad=True)
    lt = torch.zeros(16, dtype=torch.int32, device="cuda")
    E = D.dock_score(p, H, lt, wt, Gt, q=qt)
    c = torch.linspace(-1, 1, 16, device="cuda")
    (E * c).sum().backward()
    dG = torch.zeros_like(Gt)
    dw = torch.zeros_like(wt)
    dq = torch.zeros_like(qt)
    D.dock_score_adjoint(p, H, lt, wt.detach(), c.contiguous(), q=qt.detach(), G=[Gt.detach()], dLdG=[dG],
                         dLdw=dw, dLdq=dq)
    torch.cuda.synchronize()
    np.testing.assert_allclose(Gt.grad.cpu().numpy(), dG.cpu().numpy(), rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(wt.grad.cpu().numpy(), dw.cpu().numpy(), rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(qt.grad.cpu().numpy(), dq.cpu().numpy(), rtol=1e-5, atol=1e-5)


def test_adjoint_differentiation_workload(D):
    """2,000-atom pocket, Vina-form terms, weights ~ N(w0, 0.1|w0|), 64
    ligands x 32 poses with q uniform in range (the differentiation workload)."""
    pk, L, wl = synth.workload("C3")
    pk = pk[0]
    preset = P.PRESET_VINA
    K = 5
    w = synth.vina_weights(np.random.default_rng(33))
    G.say("C3: weights", w)
    p = G.load_pocket(pk, preset, w, keep=True)
    H = G.load_ligands(L)
    topos = [topology.from_ligands(L, i) for i in range(L.n_ligands)]
    rng = np.random.default_rng(34)
    T = wl["T"]
    Q = np.zeros((L.n_ligands * T, H.q_stride), np.float32)
    lig = np.repeat(np.arange(L.n_ligands), T).astype(np.int32)
    for i, t in enumerate(topos):
        Q[lig == i, :t.n_dof] = synth.random_poses(t.n_dof, t.box_min, t.box_max, T, rng)
    c = rng.normal(size=len(Q)).astype(np.float32)
    Gt = D.dock_pocket_maps(p, per_term=True).requires_grad_(True)
    wt = torch.tensor(w[None], device="cuda", requires_grad=True)
    qt = torch.tensor(Q, device="cuda", requires_grad=True)
    lt = torch.tensor(lig, device="cuda")
    ct = torch.tensor(c, device="cuda")
    E = D.dock_score(p, H, lt, wt, Gt, q=qt)
    (E * ct).sum().backward()
    torch.cuda.synchronize()
    En = E.detach().cpu().numpy()
    dG = Gt.grad.cpu().numpy().astype(np.float64)
    dw = wt.grad.cpu().numpy()[0].astype(np.float64)
    dq = qt.grad.cpu().numpy()
    # (1) node sums of dL/dG: corner weights of every atom sum to one
    counts = np.zeros((len(Q), 8))
    for i, t in enumerate(topos):
        counts[lig == i] = np.bincount(t.types, minlength=8)
    expect = np.einsum("p,pt->t", c.astype(np.float64), counts)[:, None] * w[None].astype(np.float64)
    got = dG.reshape(8, K, -1).sum(-1)
    G.say("node-sum identity max rel err", np.abs(got - expect).max() / np.abs(expect).max())
    assert np.allclose(got, expect, rtol=1e-4, atol=1e-4 * np.abs(expect).max())
    # (2) dL/dw from linearity of the forward in w (GPU forward, FP64 sum)
    for k in range(K):
        e = np.zeros((1, K), np.float32); e[0, k] = 1.0
        Ep = D.dock_score_terms(p, H, lt, wt.detach() + torch.tensor(e, device="cuda"), q=qt.detach()).cpu().numpy()
        Em = D.dock_score_terms(p, H, lt, wt.detach() - torch.tensor(e, device="cuda"), q=qt.detach()).cpu().numpy()
        fd = float(np.dot(c.astype(np.float64), (Ep.astype(np.float64) - Em) / 2.0))
        assert abs(fd - dw[k]) <= 2e-4 * (abs(dw[k]) + np.abs(c).sum()), (k, fd, dw[k])
    # (3) sampled poses against the oracle (two per ligand): per-pose E and
    #     dL/dq, and dL/dx against FP64 central differences with h = 1e-4
    dx_gpu = torch.zeros((len(Q), H.max_atoms, 3), device="cuda")
    D.dock_score_adjoint(p, H, lt, wt.detach(), ct, q=qt.detach(), G=[Gt.detach()], dLdx=dx_gpu)
    dx_gpu = dx_gpu.cpu().numpy()
    grid = SC.grid_of(pk)
    picks = np.concatenate([np.flatnonzero(lig == i)[:2] for i in range(L.n_ligands)])
    xs = [FK.fk(topos[lig[j]], Q[j:j + 1, :topos[lig[j]].n_dof].astype(np.float64)) for j in picks]
    Gd = _lazy_terms(pk, preset, grid, xs)
    w64 = w.astype(np.float64)
    worst = [0.0, 0.0, 0.0]
    n_fd = n_e = n_g = 0
    for j in picks:
        t = topos[lig[j]]
        qj = Q[j:j + 1, :t.n_dof].astype(np.float64)
        ref = SC.Scorer(pk, preset, weights=w64, G=Gd).score(t, qj)
        A = ADJ.adjoint(Gd, w64, grid, preset, t, np.array([c[j]], np.float64), q=qj)
        Er = ADJ.energy(Gd, w64, grid, preset, t, q=qj)[0]
        if ref["margin_E"][0] > G.MARGIN:
            worst[0] = max(worst[0], abs(En[j] - Er) / (1e-5 * max(abs(Er), ref["S_abs"][0])))
            n_e += 1
        if ref["margin"][0] <= 2e-4:
            continue
        n_g += 1
        gq = dq[j, :t.n_dof]
        worst[1] = max(worst[1], np.linalg.norm(gq - A["dLdq"][0]) / (1e-4 * np.linalg.norm(A["dLdq"][0]) + 1e-4))
        if n_fd < 24:
            n_fd += 1
            x = ref["x"]
            h = 1e-4
            fd = np.zeros_like(x)
            for a in range(t.n_atoms):
                for cc in range(3):
                    xp = x.copy(); xp[0, a, cc] += h
                    xm = x.copy(); xm[0, a, cc] -= h
                    fd[0, a, cc] = c[j] * (ADJ.energy(Gd, w64, grid, preset, t, x=xp)[0]
                                           - ADJ.energy(Gd, w64, grid, preset, t, x=xm)[0]) / (2 * h)
            gx = dx_gpu[j, :t.n_atoms]
            worst[2] = max(worst[2], np.linalg.norm(gx - fd[0]) / (1e-4 * np.linalg.norm(fd[0]) + 1e-4))
    G.say("C3 sampled: worst E/tol %.3g dLdq/tol %.3g dLdx-vs-FD/tol %.3g (%d of %d poses: %d E, %d gradient, "
          "%d FD)" % (*worst, n_g, len(picks), n_e, n_g, n_fd))
    assert worst[0] <= 1.0 and worst[1] <= 1.0 and worst[2] <= 1.0
    # the margins only drop poses near a decision; the checks must not thin out
    assert n_e >= 0.9 * len(picks) and n_g >= 0.75 * len(picks) and n_fd == 24
    assert n_fd >= 12


def test_deterministic_adjoint_differentiation_workload(D):
    """The differentiation workload (64 ligands x 32 poses, Vina-form terms):
    two deterministic adjoints agree bit for bit in dL/dG, dL/dw, dL/dq and
    dL/dx; the atomic mode agrees with them within FP32 summation error in
    dL/dG and dL/dw and exactly in dL/dq and dL/dx (the intra-pair forces are
    fixed point in both modes); node sums of dL/dG satisfy the exact
    identity; sampled nodes match the oracle's adjoint."""
    pk, L, wl = synth.workload("C3")
    pk = pk[0]
    preset, K = P.PRESET_VINA, 5
    w = synth.vina_weights(np.random.default_rng(33))
    p = G.load_pocket(pk, preset, w, keep=True)
    H = G.load_ligands(L)
    topos = [topology.from_ligands(L, i) for i in range(L.n_ligands)]
    rng = np.random.default_rng(35)
    T = wl["T"]
    Q = np.zeros((L.n_ligands * T, H.q_stride), np.float32)
    lig = np.repeat(np.arange(L.n_ligands), T).astype(np.int32)
    for i, t in enumerate(topos):
        Q[lig == i, :t.n_dof] = synth.random_poses(t.n_dof, t.box_min, t.box_max, T, rng)
    c = rng.normal(size=len(Q)).astype(np.float32)
    Gg = D.dock_pocket_maps(p, per_term=True)
    wt = torch.tensor(w[None], device="cuda")
    qt = torch.tensor(Q, device="cuda")
    lt = torch.tensor(lig, device="cuda")
    ct = torch.tensor(c, device="cuda")

    def run(det):
        out = dict(G=torch.zeros_like(Gg), w=torch.zeros_like(wt), q=torch.zeros_like(qt),
                   x=torch.zeros((len(Q), H.max_atoms, 3), device="cuda"))
        D.dock_score_adjoint(p, H, lt, wt, ct, q=qt, G=[Gg], dLdG=[out["G"]], dLdw=out["w"], dLdq=out["q"],
                             dLdx=out["x"], deterministic=det)
        torch.cuda.synchronize()
        return out

    d1, d2, a1 = run(1), run(1), run(0)
    for k in d1:
        assert torch.equal(d1[k], d2[k]), k
    assert torch.equal(d1["q"], a1["q"]) and torch.equal(d1["x"], a1["x"])
    gd, ga = d1["G"].cpu().numpy().astype(np.float64), a1["G"].cpu().numpy().astype(np.float64)
    scale = np.abs(gd).max()
    G.say("C3 deterministic vs atomic: dL/dG max |diff| / max %.3g, dL/dw %s vs %s"
          % (np.abs(gd - ga).max() / scale, d1["w"].cpu().numpy(), a1["w"].cpu().numpy()))
    assert np.abs(gd - ga).max() <= 1e-5 * scale
    np.testing.assert_allclose(d1["w"].cpu().numpy(), a1["w"].cpu().numpy(), rtol=1e-4,
                               atol=1e-5 * np.abs(c).sum())
    counts = np.zeros((len(Q), 8))
    for i, t in enumerate(topos):
        counts[lig == i] = np.bincount(t.types, minlength=8)
    expect = np.einsum("p,pt->t", c.astype(np.float64), counts)[:, None] * w[None].astype(np.float64)
    got = gd.reshape(8, K, -1).sum(-1)
    assert np.allclose(got, expect, rtol=1e-4, atol=1e-4 * np.abs(expect).max())
    # nodes touched by a few ligands' poses, against the oracle's adjoint of
    # exactly those poses (a separate deterministic call over them alone)
    sub = np.flatnonzero(np.isin(lig, [0, 17, 40]))
    xs = [FK.fk(topos[lig[j]], Q[j:j + 1, :topos[lig[j]].n_dof].astype(np.float64)) for j in sub]
    grid = SC.grid_of(pk)
    Gd = _lazy_terms(pk, preset, grid, xs)
    ref = np.zeros_like(Gd)
    for i in (0, 17, 40):
        sel = sub[lig[sub] == i]
        t = topos[i]
        ref += ADJ.adjoint(Gd, w.astype(np.float64), grid, preset, t, c[sel].astype(np.float64),
                           q=Q[sel, :t.n_dof].astype(np.float64))["dLdG"]
    dsub = torch.zeros_like(Gg)
    D.dock_score_adjoint(p, H, lt[sub].contiguous(), wt, ct[sub].contiguous(), q=qt[sub].contiguous(), G=[Gg],
                         dLdG=[dsub], deterministic=1)
    torch.cuda.synchronize()
    dsub = dsub.cpu().numpy().astype(np.float64)
    sc2 = np.abs(ref).max()
    G.say("C3 subset dL/dG vs oracle: max |diff| / max %.3g" % (np.abs(dsub - ref).max() / sc2))
    assert np.abs(dsub - ref).max() <= 1e-5 * sc2


def _three_pockets():
    pks = [tiny_pocket(n=30, radius=7.0, grid=32, seed=21), tiny_pocket(n=45, radius=8.0, grid=36, seed=22),
           tiny_pocket(n=20, radius=6.0, grid=26, seed=23)]
    return pks


@pytest.mark.parametrize("preset", [P.PRESET_TRIDS, P.PRESET_VINA])
def test_several_pockets_score_and_adjoint_against_oracle(D, preset):
    """Three pockets of different sizes and grids in one call, ligands
    assigned round-robin (ligand k -> pocket k mod 3), per-pocket weights:
    E and dE/dq per pose, and the deterministic adjoint (dL/dG per pocket,
    dL/dw per pocket row, dL/dq) against the oracle pocket by pocket."""
    pks = _three_pockets()
    K = P.n_terms(preset)
    rng = np.random.default_rng(50 + preset)
    W = [(np.asarray(P.default_weights(preset)) * (1 + 0.1 * rng.normal(size=K))).astype(np.float32)
         for _ in pks]
    ps = [G.load_pocket(pk, preset, W[i], keep=True) for i, pk in enumerate(pks)]
    L = synth.pack_ligands([synth.make_ligand(n, t, np.random.default_rng(100 + n)) for n, t in
                            ((6, 1), (9, 3), (12, 2), (14, 4), (8, 0), (20, 5))])
    L.pocket_index = (np.arange(L.n_ligands) % 3).astype(np.int32)
    H = G.load_ligands(L)
    topos = [topology.from_ligands(L, i) for i in range(L.n_ligands)]
    Q, lig = _poses(L, H, topos, 8, rng)
    G.say("three pockets, preset", preset, ":", len(Q), "poses")
    lt = torch.tensor(lig, device="cuda")
    qt = torch.tensor(Q, device="cuda")
    # score + gradient with each pocket's combined maps
    E, g, _ = D.dock_score_grad(ps, H, lt, qt)
    E, g = E.cpu().numpy(), g.cpu().numpy()
    for i, t in enumerate(topos):
        sel = lig == i
        pi = int(L.pocket_index[i])
        ref = SC.Scorer(pks[pi], preset, weights=W[pi].astype(np.float64)).score(t, Q[sel, :t.n_dof].astype(np.float64))
        G.compare_eval(E[sel], g[sel], ref, t.n_dof, "ligand %d pocket %d" % (i, pi))
    # differentiable form across the pockets
    Gs = [D.dock_pocket_maps(pp, per_term=True) for pp in ps]
    wt = torch.tensor(np.stack(W), device="cuda")
    dLdE = rng.normal(size=len(Q)).astype(np.float32)
    dG = [torch.zeros_like(x) for x in Gs]
    dw = torch.zeros_like(wt)
    dq = torch.zeros_like(qt)
    Et = D.dock_score_terms(ps, H, lt, wt, q=qt, G=Gs).cpu().numpy()
    D.dock_score_adjoint(ps, H, lt, wt, torch.tensor(dLdE, device="cuda"), q=qt, G=Gs, dLdG=dG, dLdw=dw, dLdq=dq,
                         deterministic=1)
    torch.cuda.synchronize()
    dw, dq = dw.cpu().numpy(), dq.cpu().numpy()
    for pi, pk in enumerate(pks):
        grid = SC.grid_of(pk)
        Gref = MAPS.build_maps(pk, preset)
        refG = np.zeros_like(Gref)
        refw = np.zeros(K)
        for i, t in enumerate(topos):
            if L.pocket_index[i] != pi:
                continue
            sel = lig == i
            qq = Q[sel, :t.n_dof].astype(np.float64)
            A = ADJ.adjoint(Gref, W[pi].astype(np.float64), grid, preset, t, dLdE[sel].astype(np.float64), q=qq)
            Er = ADJ.energy(Gref, W[pi].astype(np.float64), grid, preset, t, q=qq)
            S_abs = SC.Scorer(pk, preset, weights=W[pi].astype(np.float64), G=Gref).score(t, qq)["S_abs"]
            assert np.all(np.abs(Et[sel] - Er) <= 1e-5 * np.maximum(np.abs(Er), S_abs))
            refG += A["dLdG"]
            refw += A["dLdw"]
            err = np.linalg.norm(dq[sel, :t.n_dof] - A["dLdq"], axis=1)
            assert np.all(err <= 1e-4 * np.linalg.norm(A["dLdq"], axis=1) + 1e-4)
        got = dG[pi].cpu().numpy().astype(np.float64)
        sc = np.abs(refG).max()
        G.say("pocket %d: dL/dG max |diff| / max %.3g" % (pi, np.abs(got - refG).max() / sc))
        assert np.abs(got - refG).max() <= 1e-5 * sc + 1e-7
        np.testing.assert_allclose(dw[pi], refw, rtol=1e-5, atol=1e-4 * np.abs(refw).max())


@pytest.mark.parametrize("n_rec,radius,grid", [(12, 5.0, 14), (40, 7.0, 24)])
def test_map_build_adjoint_against_oracle(D, n_rec, radius, grid):
    from oracle import map_adjoint as MA
    pk = tiny_pocket(n=n_rec, radius=radius, grid=grid, seed=7)
    G.say("map adjoint pocket", n_rec, "atoms, grid", pk.dims)
    w = G.weights32(P.PRESET_TRIDS)
    p = G.load_pocket(pk, P.PRESET_TRIDS, w, keep=True)
    rng = np.random.default_rng(n_rec)
    lam = rng.normal(size=(8, 3) + tuple(pk.dims[::-1])).astype(np.float32)
    dx = torch.zeros((n_rec, 3), device="cuda")
    dth = torch.zeros(13, dtype=torch.float64, device="cuda")
    D.dock_pocket_map_adjoint(p, torch.tensor(lam, device="cuda"), dx, dth)
    torch.cuda.synchronize()
    ref_x, ref_t = MA.map_adjoint(pk, lam.reshape(8, 3, -1).astype(np.float64))
    gx, gt = dx.cpu().numpy().astype(np.float64), dth.cpu().numpy()
    ex = np.abs(gx - ref_x).max() / max(1.0, np.abs(ref_x).max())
    et = np.abs(gt - ref_t) / np.maximum(1.0, np.abs(ref_t))
    G.say("map adjoint: dL/dr rel err %.3g, dL/dtheta rel err %.3g" % (ex, et.max()))
    assert ex <= 1e-6
    assert et.max() <= 1e-9, (MA.THETA_NAMES[int(et.argmax())], gt, ref_t)
    # outputs accumulate
    D.dock_pocket_map_adjoint(p, torch.tensor(lam, device="cuda"), dx, dth)
    torch.cuda.synchronize()
    np.testing.assert_allclose(dth.cpu().numpy(), 2 * gt, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dx.cpu().numpy(), 2 * gx, rtol=1e-6, atol=1e-6)


def test_map_build_adjoint_rejects_other_presets(D):
    pk = tiny_pocket(n=12, radius=5.0, grid=14, seed=7)
    p = G.load_pocket(pk, P.PRESET_VINA, G.weights32(P.PRESET_VINA), keep=True)
    lam = torch.zeros((8, 5) + tuple(pk.dims[::-1]), device="cuda")
    with pytest.raises(D.DockError):
        D.dock_pocket_map_adjoint(p, lam)
