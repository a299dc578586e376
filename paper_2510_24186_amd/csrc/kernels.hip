// HIP kernels of the docking hot path for gfx950 and their launchers.
//
//  map_kernel     receptor grid maps (one thread per node, receptor atoms
//                 staged through LDS, terms and sums in FP64)
//  score_kernel   E and dE/dq of caller-supplied poses
//  sample_kernel  Metropolis MC + local refinement; one LPP-lane group per
//                 trajectory, trajectory state in registers for a whole
//                 chunk of MC steps; plain (one launch per ligand) or
//                 persistent (device work queue over ragged-packed items)
//  best_kernel    per ligand: bitonic sort of the trajectories' best
//                 energies, greedy RMSD clustering, top N
//  rank_kernel    screening rank across ligands: blocks of 2,048 scores
//                 sorted in LDS and cut to the k smallest, pass by pass
#include <float.h>
#include <math.h>

#include <algorithm>

#include "dock_device.h"
#include "dock_kernels.h"

namespace dock {

// ================================================================ maps

// ((dx*dx + dy*dy) + dz*dz) with every operation rounded separately.  The
// default contraction would fuse a product into the following sum (one
// rounding fewer), which moves d2 by an ulp and flips cutoff decisions that
// sit on the boundary.
__device__ __forceinline__ float d2_rounded(float dx, float dy, float dz) {
#pragma clang fp contract(off)
  const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
  return (xx + yy) + zz;
}

template <int K>
__global__ void __launch_bounds__(256) map_kernel(MapArgs a) {
  __shared__ float4 tile[256];
  __shared__ TypePair stab[kTypes * kTypes];
  if (threadIdx.x < kTypes * kTypes) stab[threadIdx.x] = a.tab[threadIdx.x];
  const int nx = a.grid.dims[0], ny = a.grid.dims[1], nz = a.grid.dims[2];
  const long long total = (long long)nx * ny * nz;
  const long long node = (long long)blockIdx.x * 256 + threadIdx.x;
  const bool live = node < total;
  const int ix = int(node % nx), iy = int((node / nx) % ny), iz = int(node / ((long long)nx * ny));
  // node coordinate: FP64 origin + spacing * index, rounded once to FP32
  const float px = float(double(a.grid.origin[0]) + double(a.grid.spacing) * ix);
  const float py = float(double(a.grid.origin[1]) + double(a.grid.spacing) * iy);
  const float pz = float(double(a.grid.origin[2]) + double(a.grid.spacing) * iz);
  const float cmax2 = a.preset == DOCK_PRESET_TRIDS ? 100.0f : 64.0f;
  double acc[kTypes][K];
#pragma unroll
  for (int t = 0; t < kTypes; ++t)
#pragma unroll
    for (int k = 0; k < K; ++k) acc[t][k] = 0.0;
  for (int base = 0; base < a.n_rec; base += 256) {
    __syncthreads();
    if (base + threadIdx.x < a.n_rec) tile[threadIdx.x] = a.rec[base + threadIdx.x];
    __syncthreads();
    const int cnt = min(256, a.n_rec - base);
    if (!live) continue;
    for (int j = 0; j < cnt; ++j) {
      const float4 rj = tile[j];
      // FP32 squared distance in a fixed order, each product and sum rounded
      // on its own: the inside-cutoff decisions depend on these exact bits
      const float d2 = d2_rounded(px - rj.x, py - rj.y, pz - rj.z);
      if (!(d2 < cmax2)) continue;
      const double ex = double(px) - double(rj.x), ey = double(py) - double(rj.y),
                   ez = double(pz) - double(rj.z);
      const double d = sqrt(ex * ex + ey * ey + ez * ez);
      const int tr = __float_as_int(rj.w) & 0xff;
#pragma unroll
      for (int t = 0; t < kTypes; ++t) {
        const TypePair tp = stab[t * kTypes + tr];
        double v[kMaxTerms];
        pair_terms_unweighted(a.preset, d2, d, tp.rsum64, tp.dclash2, tp.dclash64, tp.flags, v);
#pragma unroll
        for (int k = 0; k < K; ++k) acc[t][k] += v[k];
      }
    }
  }
  if (!live) return;
#pragma unroll
  for (int t = 0; t < kTypes; ++t) {
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      m += double(a.w[k]) * acc[t][k];
      if (a.G) a.G[((long long)t * K + k) * total + node] = float(acc[t][k]);
    }
    a.M[(long long)t * total + node] = float(m);
  }
}

hipError_t launch_map_build(const MapArgs& a, hipStream_t s) {
  const long long total = (long long)a.grid.dims[0] * a.grid.dims[1] * a.grid.dims[2];
  const unsigned blocks = unsigned((total + 255) / 256);
  if (a.n_terms == 3)
    hipLaunchKernelGGL(map_kernel<3>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(map_kernel<5>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ================================================================ map adjoint

// One workgroup per receptor atom: the nodes of the box around it that lie
// inside the 10 A cutoff (the same FP32 decisions as map_kernel), every
// ligand type, the chain rule in FP64.  Per atom: dL/dr written once (no
// atomics); dL/dtheta reduced in the workgroup, then 13 atomic adds.
__global__ void __launch_bounds__(256) map_adjoint_kernel(MapAdjArgs a) {
  __shared__ TypePair stab[kTypes * kTypes];
  __shared__ double red[256];
  if (threadIdx.x < kTypes * kTypes) stab[threadIdx.x] = a.tab[threadIdx.x];
  __syncthreads();
  const int i = blockIdx.x;
  const float4 ri = a.rec[i];
  const int u = __float_as_int(ri.w) & 0xff;
  const int nx = a.grid.dims[0], ny = a.grid.dims[1], nz = a.grid.dims[2];
  const long long nodes = (long long)nx * ny * nz;
  int lo[3], hi[3];
  const float rr[3] = {ri.x, ri.y, ri.z};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double o = a.grid.origin[c], h = a.grid.spacing;
    const int n = a.grid.dims[c];
    lo[c] = max(0, int(floor((double(rr[c]) - 10.0 - o) / h)) - 1);
    hi[c] = min(n - 1, int(ceil((double(rr[c]) + 10.0 - o) / h)) + 1);
  }
  const int bx = hi[0] - lo[0] + 1, by = hi[1] - lo[1] + 1, bz = hi[2] - lo[2] + 1;
  const long long nbox = (bx > 0 && by > 0 && bz > 0) ? (long long)bx * by * bz : 0;
  // accumulators: dL/dr (3), theta (13)
  double acc[3 + kMapTheta];
#pragma unroll
  for (int k = 0; k < 3 + kMapTheta; ++k) acc[k] = 0.0;
  constexpr double kSigL = 1.4142135623730951;   // sigma_long: 2 sigma^2 = 4
  constexpr double kSigL2 = 2.0, kSigL3 = 2.0 * 1.4142135623730951;
  constexpr double kSigH2 = 0.09, kSigH3 = 0.027;
  (void)kSigL;
  for (long long q = threadIdx.x; q < nbox; q += 256) {
    const int ix = lo[0] + int(q % bx), iy = lo[1] + int((q / bx) % by), iz = lo[2] + int(q / ((long long)bx * by));
    const float px = float(double(a.grid.origin[0]) + double(a.grid.spacing) * ix);
    const float py = float(double(a.grid.origin[1]) + double(a.grid.spacing) * iy);
    const float pz = float(double(a.grid.origin[2]) + double(a.grid.spacing) * iz);
    const float d2 = d2_rounded(px - ri.x, py - ri.y, pz - ri.z);
    if (!(d2 < 100.0f)) continue;
    const double ex = double(ri.x) - double(px), ey = double(ri.y) - double(py), ez = double(ri.z) - double(pz);
    const double d = sqrt(ex * ex + ey * ey + ez * ez);
    const long long node = ((long long)iz * ny + iy) * nx + ix;
    double dphi = 0.0;
    for (int t = 0; t < kTypes; ++t) {
      const TypePair tp = stab[t * kTypes + u];
      const float* lt = a.lam + (long long)(t * 3) * nodes + node;
      const double l0 = lt[0], l1 = lt[nodes], l2 = lt[2 * nodes];
      const bool hb = tp.flags & 1u;
      // E_long
      {
        const double x = d - tp.rsum64 - 3.0;
        const double g = exp(-0.25 * x * x);
        const double c = l0 * g * x / kSigL2;
        dphi += c;
        acc[3] -= c;
        acc[4] -= l0 * g * x * x / kSigL3;
        acc[3 + 5 + t] -= c;
        acc[3 + 5 + u] -= c;
      }
      // E_clash
      if (d2 < tp.dclash2) {
        if (d > 0.1) dphi -= l1 / d;
        const double ddc = l1 / tp.dclash64;
        if (hb) {
          acc[3 + 4] += ddc;
        } else {
          acc[3 + 5 + t] += ddc;
          acc[3 + 5 + u] += ddc;
        }
      }
      // E_Hbond
      if (hb && d2 < 3.4f * 3.4f) {
        const double x = d - 2.88;
        const double g = exp(-x * x / 0.18);
        const double c = l2 * g * x / kSigH2;
        dphi += c;
        acc[3 + 2] -= c;
        acc[3 + 3] -= l2 * g * x * x / kSigH3;
      }
    }
    if (d > 0.0) {
      acc[0] += dphi * ex / d;
      acc[1] += dphi * ey / d;
      acc[2] += dphi * ez / d;
    }
  }
  // workgroup reduction of the 16 accumulators
  for (int k = 0; k < 3 + kMapTheta; ++k) {
    red[threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (k < 3) {
        if (a.dLdxyz) a.dLdxyz[3 * i + k] += float(red[0]);
      } else if (a.dLdtheta && red[0] != 0.0) {
        atomicAdd(&a.dLdtheta[k - 3], red[0]);
      }
    }
    __syncthreads();
  }
}

hipError_t launch_map_adjoint(const MapAdjArgs& a, hipStream_t s) {
  if (a.n_rec <= 0) return hipSuccess;
  hipLaunchKernelGGL(map_adjoint_kernel, dim3(a.n_rec), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ================================================================ slabs

template <int LPP, int APL>
DK_INLINE GroupSlab make_slab(unsigned char* base) {
  constexpr int NA = LPP * APL;
  GroupSlab S;
  S.xs = reinterpret_cast<float4*>(base);
  S.fx = reinterpret_cast<double*>(base + 16 * NA);
  S.fy = S.fx + NA;
  S.fz = S.fy + NA;
  S.fb = reinterpret_cast<float4*>(S.fx);
  return S;
}
// coordinates (16 B per atom), then the larger of three FP64 force arrays
// (24 B per atom) and the force entries of the pass layout (2 * lanes + 1
// float4)
constexpr size_t slab_bytes(int lpp, int apl) {
  return size_t(lpp) * apl * 16 +
         (size_t(lpp) * apl * 24 > size_t(lpp) * 32 + 16 ? size_t(lpp) * apl * 24 : size_t(lpp) * 32 + 16);
}
// staged pair entries (8 bytes each), padded so the float4 slab that follows
// is aligned
constexpr size_t pair_bytes(int max_pairs) { return (size_t(max_pairs) * 8 + 15) / 16 * 16; }

size_t score_lds_bytes(int lpp, int apl, int max_pairs) {
  const int gpb = 64 / lpp;
  return size_t(gpb) * (pair_bytes(max_pairs) + slab_bytes(lpp, apl));
}

size_t sample_lds_bytes(int lpp, int apl, int block, int max_pairs) {
  const int gpb = block / lpp;
  return pair_bytes(max_pairs) + size_t(gpb) * slab_bytes(lpp, apl) + 16;
}

// E_MDN parameters of one ligand when the term is active for its pocket.
DK_INLINE MdnArg mdn_for(const LigandArrays& A, const LigDev& lg, const PocketDev& pk) {
  MdnArg m{nullptr, 0, 0};
  if (A.mdn && pk.mdn_res > 0 && pk.mdn_w != 0.f && A.mdn_res == pk.mdn_res) {
    m.par = A.mdn + size_t(lg.atom_off) * A.mdn_res * A.mdn_k;
    m.n_res = A.mdn_res;
    m.k = A.mdn_k;
  }
  return m;
}

// ================================================================ score

template <int LPP, int APL, int MODE>
__global__ void __launch_bounds__(64) score_kernel(ScoreArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int GPB = 64 / LPP;
  const int grp = threadIdx.x / LPP, r = threadIdx.x % LPP;
  const long long pose = (long long)blockIdx.x * GPB + grp;
  unsigned char* mine = smem + size_t(grp) * (pair_bytes(a.max_pairs) + slab_bytes(LPP, APL));
  PairRec* gp = reinterpret_cast<PairRec*>(mine);
  const GroupSlab S = make_slab<LPP, APL>(mine + pair_bytes(a.max_pairs));
  if (pose >= a.n_poses) return;
  const int lig = a.pose_lig[pose];
  if (lig < 0 || lig >= a.n_ligands) {
    if (r == 0) a.E[pose] = __int_as_float(0x7fc00000);
    return;
  }
  // single-launch kernels use the alternative (one atom per lane up to 64
  // atoms) pair layouts
  LigDev lg = a.L.ligs[lig];
  use_alt_layout(lg);
  const PocketDev pk = a.pockets[lg.pocket];
  LaneLig<APL> L;
  load_lane_lig<LPP, APL>(L, lg, a.L.ligs + lig, a.L.atoms, a.L.frags, a.L.tors, pk, r);
  for (int p = r; p < lg.n_stage; p += LPP) gp[p] = a.L.pairs[lg.pair_off + p];
  wave_sync();
  const float q = r < lg.n_dof ? a.q[pose * a.q_stride + r] : 0.f;
  float xo[APL][3], go[APL][3];
  const EvalOut o = eval_pose<LPP, APL, true, MODE>(L, q, pk, gp, S, r, xo, go, mdn_for(a.L, lg, pk));
  if (r == 0) a.E[pose] = o.E;
  if (a.dEdq && r < lg.n_dof) a.dEdq[pose * a.q_stride + r] = o.g;
  if (a.xyz) {
#pragma unroll
    for (int s = 0; s < APL; ++s) {
      const int atom = APL * r + s;
      if (atom < lg.n_atoms) {
        float* dst = a.xyz + pose * a.xyz_stride + 3 * L.aorig[s];
        dst[0] = xo[s][0];
        dst[1] = xo[s][1];
        dst[2] = xo[s][2];
      }
    }
  }
}

template <int MODE>
static hipError_t launch_score_t(const ScoreArgs& a, int lpp, int apl, unsigned blocks, size_t lds,
                                 hipStream_t s) {
  if (lpp == 16 && apl == 1)
    hipLaunchKernelGGL((score_kernel<16, 1, MODE>), dim3(blocks), dim3(64), lds, s, a);
  else if (lpp == 32 && apl == 1)
    hipLaunchKernelGGL((score_kernel<32, 1, MODE>), dim3(blocks), dim3(64), lds, s, a);
  else if (lpp == 64 && apl == 1)
    hipLaunchKernelGGL((score_kernel<64, 1, MODE>), dim3(blocks), dim3(64), lds, s, a);
  else
    hipLaunchKernelGGL((score_kernel<64, 2, MODE>), dim3(blocks), dim3(64), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_score(const ScoreArgs& a, int lpp, int apl, int mode, hipStream_t s) {
  const int gpb = 64 / lpp;
  const unsigned blocks = unsigned((a.n_poses + gpb - 1) / gpb);
  const size_t lds = score_lds_bytes(lpp, apl, a.max_pairs);
  if (blocks == 0) return hipSuccess;
  if (mode == kModeDirect) return launch_score_t<kModeDirect>(a, lpp, apl, blocks, lds, s);
  if (mode == kModeGridMdn) return launch_score_t<kModeGridMdn>(a, lpp, apl, blocks, lds, s);
  return launch_score_t<kModeGrid>(a, lpp, apl, blocks, lds, s);
}

// ================================================================ differentiable form

template <int LPP, int APL, int K, bool XIN>
__global__ void __launch_bounds__(64) terms_kernel(TermsArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int GPB = 64 / LPP;
  const int grp = threadIdx.x / LPP, r = threadIdx.x % LPP;
  const long long pose = (long long)blockIdx.x * GPB + grp;
  unsigned char* mine = smem + size_t(grp) * (pair_bytes(a.max_pairs) + slab_bytes(LPP, APL));
  PairRec* gp = reinterpret_cast<PairRec*>(mine);
  const GroupSlab S = make_slab<LPP, APL>(mine + pair_bytes(a.max_pairs));
  if (pose >= a.n_poses) return;
  const int lig = a.pose_lig[pose];
  if (lig < 0 || lig >= a.n_ligands) {
    if (r == 0 && a.E) a.E[pose] = __int_as_float(0x7fc00000);
    if (r == 0 && a.w_pocket) a.w_pocket[pose] = -1;
    return;
  }
  LigDev lg = a.L.ligs[lig];
  use_alt_layout(lg);
  const int pi = lg.pocket;
  const PocketDev pk = a.pockets[pi];
  LaneLig<APL> L;
  load_lane_lig<LPP, APL>(L, lg, a.L.ligs + lig, a.L.atoms, a.L.frags, a.L.tors, pk, r);
  float w[K];
#pragma unroll
  for (int k = 0; k < K; ++k) w[k] = a.w[pi * K + k];
  for (int p = r; p < lg.n_stage; p += LPP) gp[p] = a.L.pairs[lg.pair_off + p];
  wave_sync();
  float q = 0.f;
  float x[APL][3], g[APL][3], ek[K];
  Rigid rg{};
  if (XIN) {
#pragma unroll
    for (int s = 0; s < APL; ++s) {
      const int atom = APL * r + s;
      const float* src = a.xyz + pose * a.xyz_stride + 3 * L.aorig[s];
      x[s][0] = atom < lg.n_atoms ? src[0] : 0.f;
      x[s][1] = atom < lg.n_atoms ? src[1] : 0.f;
      x[s][2] = atom < lg.n_atoms ? src[2] : 0.f;
    }
  } else {
    q = r < lg.n_dof ? a.q[pose * a.q_stride + r] : 0.f;
  }
  const float dLdE = a.dLdE ? a.dLdE[pose] : 0.f;
  const bool det = a.acc_scale != nullptr;
  const float E = eval_terms<LPP, APL, K, XIN>(L, q, x, g, rg, a.G[pi], pk.grid, w, gp, S, r, dLdE,
                                               (a.dLdE && !det) ? a.dLdG[pi] : nullptr, ek,
                                               (a.dLdE && det) ? a.acc[pi] : nullptr,
                                               det ? a.acc_scale[pi] : 0.0);
  if (r == 0 && a.E) a.E[pose] = E;
  if (!a.dLdE) return;
  if (r == 0 && a.w_pose) {
#pragma unroll
    for (int k = 0; k < K; ++k) a.w_pose[pose * K + k] = dLdE * ek[k];
    a.w_pocket[pose] = pi;
  } else if (r == 0 && a.dLdw) {
#pragma unroll
    for (int k = 0; k < K; ++k) atomicAdd(&a.dLdw[pi * K + k], dLdE * ek[k]);
  }
  if (a.dLdx) {
#pragma unroll
    for (int s = 0; s < APL; ++s) {
      const int atom = APL * r + s;
      if (atom < lg.n_atoms) {
        float* d = a.dLdx + pose * a.xyz_stride + 3 * L.aorig[s];
        d[0] += dLdE * g[s][0];
        d[1] += dLdE * g[s][1];
        d[2] += dLdE * g[s][2];
      }
    }
  }
  if (!XIN && a.dLdq) {
    const float gq = chain_rule<LPP, APL>(L, rg, x, g, S, r);
    if (r < lg.n_dof) a.dLdq[pose * a.q_stride + r] += dLdE * gq;
  }
}

template <int K, bool XIN>
static hipError_t launch_terms_k(const TermsArgs& a, int lpp, int apl, unsigned blocks, size_t lds,
                                 hipStream_t s) {
  if (lpp == 16 && apl == 1)
    hipLaunchKernelGGL((terms_kernel<16, 1, K, XIN>), dim3(blocks), dim3(64), lds, s, a);
  else if (lpp == 32 && apl == 1)
    hipLaunchKernelGGL((terms_kernel<32, 1, K, XIN>), dim3(blocks), dim3(64), lds, s, a);
  else if (lpp == 64 && apl == 1)
    hipLaunchKernelGGL((terms_kernel<64, 1, K, XIN>), dim3(blocks), dim3(64), lds, s, a);
  else
    hipLaunchKernelGGL((terms_kernel<64, 2, K, XIN>), dim3(blocks), dim3(64), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_terms(const TermsArgs& a, int lpp, int apl, int K, hipStream_t s) {
  const int gpb = 64 / lpp;
  const unsigned blocks = unsigned((a.n_poses + gpb - 1) / gpb);
  const size_t lds = score_lds_bytes(lpp, apl, a.max_pairs);
  if (blocks == 0) return hipSuccess;
  const bool xin = a.xyz != nullptr;
  if (K == 3) return xin ? launch_terms_k<3, true>(a, lpp, apl, blocks, lds, s)
                         : launch_terms_k<3, false>(a, lpp, apl, blocks, lds, s);
  return xin ? launch_terms_k<5, true>(a, lpp, apl, blocks, lds, s)
             : launch_terms_k<5, false>(a, lpp, apl, blocks, lds, s);
}

// ================================================================ deterministic adjoint

// One workgroup: per pocket, the bound B = n_poses * max_p(|dLdE_p| N_p) *
// max_k |w_k| on any node's |dL/dG| (each atom's eight corner weights are
// non-negative and sum to one), and the fixed-point scale 2^(62 - e) with
// B <= 2^e.  Maxima do not depend on the order of evaluation.
__global__ void __launch_bounds__(256) adj_bound_kernel(AdjBoundArgs a) {
  __shared__ float red[kMaxDiffPockets][256];
  float m[kMaxDiffPockets];
#pragma unroll
  for (int k = 0; k < kMaxDiffPockets; ++k) m[k] = 0.f;
  for (long long p = threadIdx.x; p < a.n_poses; p += 256) {
    const int lig = a.pose_lig[p];
    if (lig < 0 || lig >= a.n_ligands) continue;
    const LigDev& lg = a.ligs[lig];
    float v = fabsf(a.dLdE[p]) * float(lg.n_atoms);
    if (!(v <= FLT_MAX)) v = INFINITY;  // NaN counts as unbounded
#pragma unroll
    for (int k = 0; k < kMaxDiffPockets; ++k)
      if (k == lg.pocket) m[k] = fmaxf(m[k], v);
  }
#pragma unroll
  for (int k = 0; k < kMaxDiffPockets; ++k) red[k][threadIdx.x] = m[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < kMaxDiffPockets; ++k) red[k][threadIdx.x] = fmaxf(red[k][threadIdx.x], red[k][threadIdx.x + w]);
    __syncthreads();
  }
  const int pi = threadIdx.x;
  if (pi < a.n_pockets) {
    float mw = 0.f;
    for (int k = 0; k < a.K; ++k) {
      float v = fabsf(a.w[pi * a.K + k]);
      if (!(v <= FLT_MAX)) v = INFINITY;
      mw = fmaxf(mw, v);
    }
    const double B = double(a.n_poses) * double(red[pi][0]) * double(mw);
    double scale = 1.0;
    if (!(B <= DBL_MAX)) {
      scale = 0.0;
    } else if (B > 0.0) {
      int ex = 0;
      (void)frexp(B, &ex);
      scale = ldexp(1.0, 62 - ex);
    }
    a.scale[pi] = scale;
  }
}

hipError_t launch_adj_bound(const AdjBoundArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(adj_bound_kernel, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

__global__ void adj_finalize_kernel(const unsigned long long* __restrict__ acc, const double* scale, long long n,
                                    float* __restrict__ dLdG) {
  const double sc = *scale;
  const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float v = sc > 0.0 ? float(double(static_cast<long long>(acc[i])) * inv) : __int_as_float(0x7fc00000);
    dLdG[i] += v;
  }
}

hipError_t launch_adj_finalize(const unsigned long long* acc, const double* scale, long long n, float* dLdG,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(adj_finalize_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, acc, scale, n, dLdG);
  return hipGetLastError();
}

// One workgroup per (pocket, term): thread t sums poses t, t + 256, ... in
// order, then a fixed tree over the workgroup.
__global__ void __launch_bounds__(256) adj_wreduce_kernel(const float* __restrict__ w_pose,
                                                          const int* __restrict__ w_pocket, long long n_poses,
                                                          int K, float* dLdw) {
  __shared__ float red[256];
  const int pi = blockIdx.x / K, k = blockIdx.x % K;
  float acc = 0.f;
  for (long long p = threadIdx.x; p < n_poses; p += 256)
    if (w_pocket[p] == pi) acc += w_pose[p * K + k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) dLdw[pi * K + k] += red[0];
}

hipError_t launch_adj_wreduce(const float* w_pose, const int* w_pocket, long long n_poses, int n_pockets, int K,
                              float* dLdw, hipStream_t s) {
  if (n_pockets * K <= 0) return hipSuccess;
  hipLaunchKernelGGL(adj_wreduce_kernel, dim3(unsigned(n_pockets * K)), dim3(256), 0, s, w_pose, w_pocket,
                     n_poses, K, dLdw);
  return hipGetLastError();
}

__global__ void zero_u64_kernel(unsigned long long* p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

hipError_t launch_zero_u64(unsigned long long* p, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(zero_u64_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// ================================================================ sampler

template <int APL>
DK_INLINE float wrap_clamp(float q, int r, const LaneLig<APL>& L) {
  if (r < 3) return fminf(fmaxf(q, L.lo), L.hi);
  return wrap_angle(q);
}

template <int LPP, int APL, int MODE>
DK_INLINE void run_traj(const SampleArgs& a, const LaneLig<APL>& L, const PocketDev& pk, const MdnArg& mdn,
                        const PairRec* pairs,
                        const GroupSlab& S, int lig, int traj, int r) {
  const size_t ti = size_t(lig) * a.n_traj + traj;
  const uint32_t k0 = uint32_t(lig), k1 = uint32_t(a.step_base[1]);
  const bool dof = r < L.n_dof;
  const int qs = a.q_stride;
  int nev = a.n_evals[ti];
  float* trow = nullptr;
  if (a.trace && lig % a.trace_stride == 0 && traj < a.trace_traj)
    trow = a.trace + (size_t(lig / a.trace_stride) * a.trace_traj + traj) * size_t(a.trace_cap) * (2 * qs + 1);
  auto record = [&](float qv, float gv, float Ev) {
    if (trow && nev < a.trace_cap) {
      float* row = trow + size_t(nev) * (2 * qs + 1);
      if (r < qs) {
        row[r] = dof ? qv : 0.f;
        row[qs + r] = dof ? gv : 0.f;
      }
      if (r == 0) row[2 * qs] = Ev;
    }
    ++nev;
  };
  if (a.init) {
    const uint4 w = philox4x32_10(make_uint4(uint32_t(traj), 0u, 0u, uint32_t(r >> 2)), k0, k1);
    const float q = dof ? L.lo + (L.hi - L.lo) * u01(pick4(w, r & 3)) : 0.f;
    const EvalOut o = eval_pose<LPP, APL, false, MODE>(L, q, pk, pairs, S, r, nullptr, nullptr, mdn);
    record(q, o.g, o.E);
    if (dof) {
      a.q_cur[ti * qs + r] = q;
      a.q_best[ti * qs + r] = q;
    }
    if (r == 0) {
      a.E_cur[ti] = o.E;
      a.E_best[ti] = o.E;
      a.n_evals[ti] = nev;
    }
    return;
  }
  float q = dof ? a.q_cur[ti * qs + r] : 0.f;
  float qb = dof ? a.q_best[ti * qs + r] : 0.f;
  float Ecur = a.E_cur[ti], Ebest = a.E_best[ti];
  const int base = *a.step_base + a.step_off;
  for (int s = base + 1; s <= base + a.step_count; ++s) {
    const uint4 w = philox4x32_10(make_uint4(uint32_t(traj), uint32_t(s), 1u, 0u), k0, k1);
    const int j = int(__umulhi(w.x, uint32_t(L.n_dof)));
    float qn = q;
    if (r == j) qn = L.lo + (L.hi - L.lo) * u01(w.y);
    float E;
    if (a.local_opt != DOCK_LOCAL_LINESEARCH) {
      // n_local gradient evaluations with a first-order update after each
      // (Adam by default; the Table S5 alternatives otherwise), then the
      // energy of the refined pose: one evaluation site, n_local + 1 calls
      float m = 0.f, v = 0.f, b1t = 1.f, b2t = 1.f;
      for (int t = 0;; ++t) {
        const EvalOut o = eval_pose<LPP, APL, false, MODE>(L, qn, pk, pairs, S, r, nullptr, nullptr, mdn);
        record(qn, o.g, o.E);
        E = o.E;
        if (t == a.n_local) break;
        const float g = o.g;
        // square roots and quotients on the hardware units (about 1 ulp;
        // the IEEE-exact sequences cost ~12 instructions each)
        float step;
        if (a.local_opt == DOCK_LOCAL_SGD) {
          step = a.lr * g;
        } else if (a.local_opt == DOCK_LOCAL_RMSPROP) {
          v = a.rms_alpha * v + (1.f - a.rms_alpha) * g * g;
          step = a.lr * g * rcp_hw(sqrt_hw(v) + a.eps);
        } else if (a.local_opt == DOCK_LOCAL_ADAGRAD) {
          v += g * g;
          step = a.lr * g * rcp_hw(sqrt_hw(v) + a.eps);
        } else {
          if (a.local_opt == DOCK_LOCAL_ADAMW) qn *= 1.f - a.lr * a.weight_decay;
          m = a.b1 * m + (1.f - a.b1) * g;
          v = a.b2 * v + (1.f - a.b2) * g * g;
          b1t *= a.b1;
          b2t *= a.b2;
          const float mh = m * rcp_hw(1.f - b1t), vh = v * rcp_hw(1.f - b2t);
          step = a.lr * mh * rcp_hw(sqrt_hw(vh) + a.eps);
        }
        if (dof) qn = wrap_clamp(qn - step, r, L);
      }
    } else {
      // Armijo line search as a loop over trial poses (one evaluation site):
      // the first call scores the perturbed pose; each search tries
      // alpha = 1, 1/2, ..., 2^-10 along -g/|g|; a failed search ends the
      // refinement
      float g = 0.f, d = 0.f, slope = 0.f, alpha = 1.f;
      float qtry = qn;
      int done_steps = 0, halvings = 0;
      bool first = true;
      E = 0.f;
      for (;;) {
        const EvalOut o = eval_pose<LPP, APL, false, MODE>(L, qtry, pk, pairs, S, r, nullptr, nullptr, mdn);
        record(qtry, o.g, o.E);
        if (first) {
          E = o.E;
          g = o.g;
          first = false;
        } else if (o.E <= E + 1e-4f * alpha * slope) {
          qn = qtry;
          E = o.E;
          g = o.g;
          ++done_steps;
        } else {
          if (++halvings > 10) break;
          alpha *= 0.5f;
          qtry = dof ? wrap_clamp(qn + alpha * d, r, L) : 0.f;
          continue;
        }
        if (done_steps >= a.n_local) break;
        const float gn = sqrtf(group_sum<LPP>(dof ? g * g : 0.f));
        if (!(gn > 0.f)) break;
        d = dof ? -g / gn : 0.f;
        slope = -gn;
        alpha = 1.f;
        halvings = 0;
        qtry = dof ? wrap_clamp(qn + d, r, L) : 0.f;
      }
    }
    const float u = u01(w.z);
    const bool acc = u < expf(-a.mc_beta * (E - Ecur));
    if (acc) {
      q = qn;
      Ecur = E;
    }
    if (E < Ebest) {
      qb = qn;
      Ebest = E;
    }
  }
  if (dof) {
    a.q_cur[ti * qs + r] = q;
    a.q_best[ti * qs + r] = qb;
  }
  if (r == 0) {
    a.E_cur[ti] = Ecur;
    a.E_best[ti] = Ebest;
    a.n_evals[ti] = nev;
  }
}

// Three waves per SIMD (168 VGPRs).  With two atoms per lane the step loop
// needs more and spills a few registers to scratch (served from L2, outside
// the pair-pass loop); two waves per SIMD without spills measured slower.
template <int LPP, int APL, int BLOCK, int MODE>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(3))) sample_kernel(SampleArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int GPB = BLOCK / LPP;
  const int grp = threadIdx.x / LPP, r = threadIdx.x % LPP;
  PairRec* sp = reinterpret_cast<PairRec*>(smem);
  unsigned char* slabs = smem + pair_bytes(a.max_pairs);
  const GroupSlab S = make_slab<LPP, APL>(slabs + size_t(grp) * slab_bytes(LPP, APL));
  int* s_item = reinterpret_cast<int*>(slabs + size_t(GPB) * slab_bytes(LPP, APL));
  int taken = 0;
  // persistent: partitions in turn from the block's own (b mod n_part); a
  // partition is left for good once its counter passes its size, so every
  // block exits after at most n_part empty pops
  const int home = a.queue ? int(blockIdx.x % unsigned(a.n_part)) : 0;
  int tried = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      int it = a.n_items;
      if (a.queue) {
        while (tried < a.n_part) {
          int q = home + tried;
          if (q >= a.n_part) q -= a.n_part;
          const int lo = a.part_off[q], n = a.part_off[q + 1] - lo;
          const int k = n > 0 ? atomicAdd(a.queue + q, 1) : n;
          if (k < n) {
            it = lo + k;
            break;
          }
          ++tried;
        }
      } else {
        it = taken == 0 ? int(blockIdx.x) : a.n_items;
      }
      *s_item = it;
    }
    __syncthreads();
    const int item = *s_item;
    __syncthreads();
    if (item >= a.n_items) break;
    ++taken;
    const int2 wi = a.items[item];
    const int lig = wi.x;
    // one atom per lane: the alternative layout (the primary one for every
    // ligand not laid out with two atoms per lane)
    LigDev lg = a.L.ligs[lig];
    if (APL == 1) use_alt_layout(lg);
    for (int p = threadIdx.x; p < lg.n_stage; p += BLOCK) sp[p] = a.L.pairs[lg.pair_off + p];
    __syncthreads();
    const int traj = wi.y + grp;
    if (traj < a.n_traj) {
      const PocketDev pk = a.pockets[lg.pocket];
      LaneLig<APL> L;
      load_lane_lig<LPP, APL>(L, lg, a.L.ligs + lig, a.L.atoms, a.L.frags, a.L.tors, pk, r);
      run_traj<LPP, APL, MODE>(a, L, pk, mdn_for(a.L, lg, pk), sp, S, lig, traj, r);
    }
    __syncthreads();
  }
}

template <int LPP, int APL, int BLOCK, int MODE>
static hipError_t launch_sample_t(const SampleArgs& a, int grid, hipStream_t s) {
  const size_t lds = sample_lds_bytes(LPP, APL, BLOCK, a.max_pairs);
  hipLaunchKernelGGL((sample_kernel<LPP, APL, BLOCK, MODE>), dim3(grid), dim3(BLOCK), lds, s, a);
  return hipGetLastError();
}

#define DOCK_SAMPLE_CASES(X)                                                                      \
  X(16, 1, 64) X(32, 1, 64) X(64, 1, 64) X(32, 2, 64) X(64, 2, 64) X(16, 1, 128) X(32, 1, 128)    \
      X(64, 1, 128) X(32, 2, 128) X(64, 2, 128) X(16, 1, 256) X(32, 1, 256) X(64, 1, 256)          \
          X(32, 2, 256) X(64, 2, 256)

hipError_t launch_sample(const SampleArgs& a, int lpp, int apl, int grid, int block, int mode,
                         hipStream_t s) {
  if (grid <= 0) return hipSuccess;
#define X(L, A, B)                                                                     \
  if (lpp == L && apl == A && block == B) {                                            \
    if (mode == kModeDirect) return launch_sample_t<L, A, B, kModeDirect>(a, grid, s); \
    if (mode == kModeGridMdn) return launch_sample_t<L, A, B, kModeGridMdn>(a, grid, s); \
    return launch_sample_t<L, A, B, kModeGrid>(a, grid, s);                            \
  }
  DOCK_SAMPLE_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

template <int L, int A, int B>
static int blocks_per_cu(int mode, size_t lds) {
  int n = 0;
  hipError_t e;
  if (mode == kModeDirect)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sample_kernel<L, A, B, kModeDirect>, B, lds);
  else if (mode == kModeGridMdn)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sample_kernel<L, A, B, kModeGridMdn>, B, lds);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sample_kernel<L, A, B, kModeGrid>, B, lds);
  if (e != hipSuccess) n = 1;
  return n > 0 ? n : 1;
}

int sample_max_blocks_per_cu(int lpp, int apl, int block, int mode, size_t lds) {
#define X(L, A, B) \
  if (lpp == L && apl == A && block == B) return blocks_per_cu<L, A, B>(mode, lds);
  DOCK_SAMPLE_CASES(X)
#undef X
  return 1;
}

// ================================================================ best poses

__global__ void __launch_bounds__(64) best_kernel(BestArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int LPP = 64, APL = 2;
  const int lig = blockIdx.x, r = threadIdx.x;
  float* kE = reinterpret_cast<float*>(smem);
  int* kI = reinterpret_cast<int*>(kE + a.t_pad);
  float4* kept = reinterpret_cast<float4*>(smem + (size_t(a.t_pad) * 8 + 15) / 16 * 16);  // [top_n][kMaxAtoms]
  const LigDev lg = a.L.ligs[lig];
  PocketDev none;
  none.preset = DOCK_PRESET_TRIDS;
  none.n_terms = 0;
  LaneLig<APL> L;
  load_lane_lig<LPP, APL>(L, lg, a.L.ligs + lig, a.L.atoms, a.L.frags, a.L.tors, none, r);
  const int T = a.n_traj;
  for (int i = r; i < a.t_pad; i += 64) {
    float e = i < T ? a.E_best[size_t(lig) * T + i] : INFINITY;
    if (!(e < INFINITY)) e = INFINITY;  // NaN and +inf rank last
    kE[i] = e;
    kI[i] = i < T ? i : 0x7fffffff;
  }
  wave_sync();
  for (int k = 2; k <= a.t_pad; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = r; i < a.t_pad; i += 64) {
        const int l = i ^ j;
        if (l > i) {
          const float ei = kE[i], el = kE[l];
          const int ii = kI[i], il = kI[l];
          const bool gt = ei > el || (ei == el && ii > il);
          const bool up = (i & k) == 0;
          if (gt == up) {
            kE[i] = el; kE[l] = ei;
            kI[i] = il; kI[l] = ii;
          }
        }
      }
      wave_sync();
    }
  }
  int n_kept = 0;
  const float inv_n = 1.0f / float(lg.n_atoms);
  for (int c = 0; c < T && n_kept < a.top_n; ++c) {
    const float E = kE[c];
    if (!(E < INFINITY)) break;
    const int t = kI[c];
    const float q = r < lg.n_dof ? a.q_best[(size_t(lig) * T + t) * a.q_stride + r] : 0.f;
    float x[APL][3];
    fk_place_shfl<LPP, APL>(L, q, r, x);
    bool dup = false;
    for (int k = 0; k < n_kept && !dup; ++k) {
      float acc = 0.f;
#pragma unroll
      for (int s = 0; s < APL; ++s) {
        const int atom = APL * r + s;
        if (atom < lg.n_atoms) {
          const float4 y = kept[k * kMaxAtoms + atom];
          const float dx = x[s][0] - y.x, dy = x[s][1] - y.y, dz = x[s][2] - y.z;
          acc += dx * dx + dy * dy + dz * dz;
        }
      }
      dup = sqrtf(group_sum<64>(acc) * inv_n) < a.rmsd_cut;
    }
    if (!dup) {
      const size_t o = size_t(lig) * a.top_n + n_kept;
#pragma unroll
      for (int s = 0; s < APL; ++s) {
        const int atom = APL * r + s;
        if (atom < lg.n_atoms) {
          kept[n_kept * kMaxAtoms + atom] = make_float4(x[s][0], x[s][1], x[s][2], 0.f);
          if (a.xyz_out) {
            float* dst = a.xyz_out + o * a.xyz_stride + 3 * L.aorig[s];
            dst[0] = x[s][0];
            dst[1] = x[s][1];
            dst[2] = x[s][2];
          }
        }
      }
      if (r == 0) {
        if (a.E_out) a.E_out[o] = E;
        if (a.E_screen) a.E_screen[o] = E / (1.0f + a.w_tor * float(lg.n_tors));
        if (a.idx_out) a.idx_out[o] = t;
      }
      if (a.q_out && r < a.q_stride) a.q_out[o * a.q_stride + r] = r < lg.n_dof ? q : 0.f;
      ++n_kept;
    }
    wave_sync();
  }
  for (int k = n_kept; k < a.top_n; ++k) {
    const size_t o = size_t(lig) * a.top_n + k;
    if (r == 0) {
      if (a.E_out) a.E_out[o] = INFINITY;
      if (a.E_screen) a.E_screen[o] = INFINITY;
      if (a.idx_out) a.idx_out[o] = -1;
    }
    if (a.q_out && r < a.q_stride) a.q_out[o * a.q_stride + r] = 0.f;
  }
  if (r == 0 && a.n_out) a.n_out[lig] = n_kept;
}

hipError_t launch_best(const BestArgs& a, hipStream_t s) {
  const size_t lds = (size_t(a.t_pad) * 8 + 15) / 16 * 16 + size_t(a.top_n) * kMaxAtoms * 16;
  if (a.n_ligands <= 0) return hipSuccess;
  hipLaunchKernelGGL(best_kernel, dim3(a.n_ligands), dim3(64), lds, s, a);
  return hipGetLastError();
}

// ================================================================ screening rank

// Total order on (score, index): the score's bits mapped to an unsigned key
// that sorts like the float (-0.0 as +0.0, every NaN after +inf), the
// ligand index breaking ties.
DK_INLINE unsigned long long rank_key(float v, int idx) {
  uint32_t u = __float_as_uint(v);
  if (v != v) u = 0xffffffffu;
  else if (u == 0x80000000u) u = 0u;
  if (u != 0xffffffffu) u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return (static_cast<unsigned long long>(u) << 32) | static_cast<uint32_t>(idx);
}

__global__ void __launch_bounds__(256) rank_kernel(RankArgs a) {
  __shared__ unsigned long long key[kRankBlock];
  __shared__ float val[kRankBlock];
  const long long base = (long long)blockIdx.x * kRankBlock;
  for (int t = threadIdx.x; t < kRankBlock; t += 256) {
    const long long e = base + t;
    if (e < a.n) {
      const float v = a.idx ? a.score[e] : a.score[e * a.stride];
      const int id = a.idx ? a.idx[e] : int(e);
      // an empty slot of an earlier pass (index -1) stays empty
      key[t] = id < 0 ? ~0ull : rank_key(v, id);
      val[t] = v;
    } else {
      key[t] = ~0ull;
      val[t] = __int_as_float(0x7f800000);
    }
  }
  __syncthreads();
  // bitonic sort of kRankBlock keys (values follow their key)
  for (int size = 2; size <= kRankBlock; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < kRankBlock / 2; t += 256) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const unsigned long long kl = key[lo], kh = key[hi];
        if ((kl > kh) == up) {
          key[lo] = kh;
          key[hi] = kl;
          const float vl = val[lo];
          val[lo] = val[hi];
          val[hi] = vl;
        }
      }
      __syncthreads();
    }
  }
  const int keep = a.k < kRankBlock ? a.k : kRankBlock;
  for (int t = threadIdx.x; t < keep; t += 256) {
    const unsigned long long kv = key[t];
    const bool none = kv == ~0ull;
    a.out_score[(long long)blockIdx.x * keep + t] = none ? __int_as_float(0x7f800000) : val[t];
    a.out_idx[(long long)blockIdx.x * keep + t] = none ? -1 : int(uint32_t(kv));
  }
}

hipError_t launch_rank(const RankArgs& a, hipStream_t s) {
  const long long nb = (a.n + kRankBlock - 1) / kRankBlock;
  const unsigned blocks = unsigned(nb > 0 ? nb : 1);
  hipLaunchKernelGGL(rank_kernel, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ================================================================ Philox dump

__global__ void philox_kernel(const uint4* ctr, uint32_t k0, uint32_t k1, long long n, uint4* out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = philox4x32_10(ctr[i], k0, k1);
}

hipError_t launch_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, long long n, uint32_t* out,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(philox_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const uint4*>(ctr), k0, k1, n, reinterpret_cast<uint4*>(out));
  return hipGetLastError();
}

// ================================================================ small helpers

__global__ void fill_int_kernel(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void add_int_kernel(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p += v;
}

hipError_t launch_fill_int(int* p, int n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
__global__ void fill_u32_kernel(uint32_t* p, long long n, uint32_t v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
hipError_t launch_fill_u32(uint32_t* p, long long n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(fill_u32_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_add_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(add_int_kernel, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

}  // namespace dock
