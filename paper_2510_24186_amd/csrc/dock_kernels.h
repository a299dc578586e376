// Kernel argument blocks and launchers (host <-> device interface of libdock).
#pragma once

#include "dock_internal.h"

namespace dock {

struct PairRec;

struct LigandArrays {
  const LigDev* ligs;
  const float4* atoms;   // DFS order; w = bits(type | frag << 8 | caller index << 16)
  const FragDev* frags;
  const TorsDev* tors;
  const PairRec* pairs;
  // E_MDN mixture parameters, float4 (pi, mu, log2(e) / (2 sigma^2),
  // 1 / sigma^2) per [atom (DFS, global)][residue][gaussian]; null if none
  const float4* mdn;
  int mdn_res, mdn_k;
};

struct ScoreArgs {
  LigandArrays L;
  const PocketDev* pockets;
  int n_ligands, n_pockets;
  long long n_poses;
  const int* pose_lig;
  const float* q;
  int q_stride;
  float* E;
  float* dEdq;
  float* xyz;
  int xyz_stride;
  int max_pairs;
};

constexpr int kMaxDiffPockets = 16;

struct TermsArgs {
  LigandArrays L;
  const PocketDev* pockets;  // grid geometry per pocket
  int n_ligands, n_pockets;
  long long n_poses;
  const int* pose_lig;
  const float* q;            // pose DOFs (coordinates mode: null)
  int q_stride;
  const float* xyz;          // world coordinates, caller atom order (DOF mode: null)
  int xyz_stride;
  const float* G[kMaxDiffPockets];   // per-term maps per pocket
  const float* w;                    // device [n_pockets * K]
  float* E;
  const float* dLdE;                 // null: forward only
  float* dLdG[kMaxDiffPockets];
  float* dLdw;
  float* dLdq;
  float* dLdx;
  int max_pairs;
  // deterministic adjoint (null otherwise): dL/dG into 64-bit fixed-point
  // accumulators acc[pocket] (layout of dLdG) at scale acc_scale[pocket];
  // dL/dw as per-pose contributions w_pose [n_poses * K] and the pose's
  // pocket w_pocket [n_poses] (-1: invalid ligand), reduced afterwards
  unsigned long long* acc[kMaxDiffPockets];
  const double* acc_scale;
  float* w_pose;
  int* w_pocket;
};

// Deterministic adjoint helpers.
struct AdjBoundArgs {
  const LigDev* ligs;
  int n_ligands, n_pockets, K;
  long long n_poses;
  const int* pose_lig;
  const float* dLdE;
  const float* w;       // [n_pockets * K]
  double* scale;        // out [n_pockets]: 2^(62 - e), 0 for a non-finite bound
};
hipError_t launch_adj_bound(const AdjBoundArgs& a, hipStream_t s);
// dLdG[i] += acc[i] / scale (NaN where scale = 0), i < n
hipError_t launch_adj_finalize(const unsigned long long* acc, const double* scale, long long n, float* dLdG,
                               hipStream_t s);
// dLdw[pi * K + k] += sum over poses p with w_pocket[p] == pi of w_pose[p * K + k],
// in a fixed order
hipError_t launch_adj_wreduce(const float* w_pose, const int* w_pocket, long long n_poses, int n_pockets, int K,
                              float* dLdw, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, long long n, hipStream_t s);

struct SampleArgs {
  LigandArrays L;
  const PocketDev* pockets;
  const int2* items;      // (ligand, first trajectory)
  int n_items;
  int* queue;             // persistent work counters (one per partition), or null:
                          // item = blockIdx.x
  const int* part_off;    // n_part + 1 item bounds of the partitions
  int n_part;             // block b takes partition b mod n_part first, then the others
  const int* step_base;   // device: [0] MC steps already taken, [1] the seed
  int step_off;           // this launch covers steps base+off+1 .. base+off+count
  int step_count;
  int init;               // draw initial poses and score them instead of stepping
  int n_traj, q_stride;
  int n_local, local_opt;
  float lr, b1, b2, eps, mc_beta, rms_alpha, weight_decay;
  float* q_cur;
  float* E_cur;
  float* q_best;
  float* E_best;
  int* n_evals;
  float* trace;
  int trace_cap;
  int trace_stride, trace_traj;  // logged: ligands l % stride == 0, trajectories < trace_traj
  int max_pairs;
};

struct BestArgs {
  LigandArrays L;
  int n_ligands, n_traj, q_stride;
  const float* E_best;
  const float* q_best;
  int top_n;
  float rmsd_cut, w_tor;
  float* E_out;
  float* E_screen;
  float* q_out;
  int* idx_out;
  float* xyz_out;
  int xyz_stride;
  int* n_out;
  int t_pad;
};

struct MapArgs {
  const float4* rec;  // xyz, w = bits(type)
  int n_rec;
  GridDev grid;
  int preset, n_terms;
  float w[kMaxTerms];
  TypePair tab[kTypes * kTypes];
  float* G;  // [8][K][nodes] or null
  float* M;  // [8][nodes]
};

// Adjoint of the TRIDS map build: dL/d(receptor xyz) and dL/dtheta for
// theta = (mu_long, sigma_long, mu_hb, sigma_hb, d_clash_hb, R_0..R_7).
constexpr int kMapTheta = 5 + kTypes;
struct MapAdjArgs {
  const float4* rec;   // xyz, w = bits(type), caller order
  int n_rec;
  GridDev grid;
  TypePair tab[kTypes * kTypes];
  const float* lam;    // dL/dG [8][3][nodes]
  float* dLdxyz;       // [n_rec * 3], +=
  double* dLdtheta;    // [kMapTheta], +=
};
hipError_t launch_map_adjoint(const MapAdjArgs& a, hipStream_t s);

// LDS bytes a sampler block of `block` threads needs.
size_t sample_lds_bytes(int lpp, int apl, int block, int max_pairs);
size_t score_lds_bytes(int lpp, int apl, int max_pairs);

hipError_t launch_map_build(const MapArgs& a, hipStream_t s);
// mode: 0 grid maps, 1 direct pair sums, 2 grid maps + E_MDN
hipError_t launch_score(const ScoreArgs& a, int lpp, int apl, int mode, hipStream_t s);
hipError_t launch_sample(const SampleArgs& a, int lpp, int apl, int grid, int block, int mode,
                         hipStream_t s);
hipError_t launch_best(const BestArgs& a, hipStream_t s);

// Screening rank: one pass reduces every block of kRankBlock (score, index)
// entries to its k smallest.
constexpr int kRankBlock = 2048;
struct RankArgs {
  const float* score;  // first pass: strided ligand scores; later: packed
  const int* idx;      // null on the first pass (index = position)
  long long n;
  int stride;
  int k;
  float* out_score;
  int* out_idx;
};
hipError_t launch_rank(const RankArgs& a, hipStream_t s);
hipError_t launch_terms(const TermsArgs& a, int lpp, int apl, int K, hipStream_t s);
hipError_t launch_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, long long n, uint32_t* out,
                         hipStream_t s);
hipError_t launch_fill_int(int* p, int n, int v, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, long long n, uint32_t v, hipStream_t s);
hipError_t launch_add_int(int* p, int v, hipStream_t s);
int sample_max_blocks_per_cu(int lpp, int apl, int block, int mode, size_t lds);

}  // namespace dock
