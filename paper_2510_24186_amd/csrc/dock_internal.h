// Internal layout shared by the host half (ligand preparation, planning,
// ABI) and the device half (HIP kernels) of libdock.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/dock.h"

namespace dock {

constexpr int kTypes = DOCK_N_TYPES;
constexpr int kMaxAtoms = DOCK_MAX_ATOMS;
constexpr int kMaxTors = DOCK_MAX_TORS;
constexpr int kMaxDof = 6 + DOCK_MAX_TORS;
constexpr int kMaxTerms = DOCK_MAX_TERMS;

// Where one layout of a ligand's pair records sits in the packed array, and
// its shape (see LigDev).
struct PairLayout {
  int pair_off, n_prec, n_stage;
  int n_pass, pass_w, pull_cap, pass_apl;
  int pad;
};

// Per-ligand record, device resident.  Atoms are stored in fragment
// depth-first pre-order so that every torsion's moving subtree is one
// contiguous atom range (the chain rule sums over ranges).
struct alignas(16) LigDev {
  int n_atoms, n_tors, n_frags, n_pairs;
  int atom_off, pair_off, frag_off, tors_off;
  int pocket, fk_rounds, n_dof, n_prec;   // n_prec: device pair records (with empty slots)
  float c0[3];
  float box_min[3];
  float box_max[3];
  int n_pass, pass_w, pull_cap;           // pass layout (n_pass = 0: pairs are strided, forces by atomics)
  int pass_apl;                           // atoms per lane of the pass layout (pull words per pass = apl * w)
  int n_stage;                            // 8-byte entries to stage: pair records (+ pull words)
  // The fields above describe the primary pair layout (the lane
  // configuration of large batched runs).  `alt` is the layout with one atom
  // per lane up to 64 atoms, for launches that hold few poses of a ligand
  // (plain form, the single-launch kernels, small batches); it equals the
  // primary one where that already has one atom per lane.
  PairLayout alt;
};

// Switches a copy of a ligand record to its alternative pair layout.
__host__ __device__ inline void use_alt_layout(LigDev& g) {
  g.pair_off = g.alt.pair_off;
  g.n_prec = g.alt.n_prec;
  g.n_stage = g.alt.n_stage;
  g.n_pass = g.alt.n_pass;
  g.pass_w = g.alt.pass_w;
  g.pull_cap = g.alt.pull_cap;
  g.pass_apl = g.alt.pass_apl;
}

// Fragment record (DFS numbering).  Root: parent = -1, dof = -1.
// A child turns about the input-frame axis through xb with unit direction u.
// Atom coordinates and pivots are stored relative to the root centroid c0.
struct alignas(16) FragDev {
  float u[3];
  float xb[3];
  int parent;
  int dof;
};

// Torsion record, indexed by torsion k (DOF 6 + k): its moving atoms are the
// DFS range [sub_begin, sub_end); a, b are the axis atoms (DFS numbering).
struct alignas(16) TorsDev {
  int sub_begin, sub_end, a, b;
};

// Term constants for one (type_i, type_j) pair.  The FP32 copies decide
// cutoffs and serve the FP32 pair terms; the FP64 copies serve the map build.
struct alignas(16) TypePair {
  float rsum;     // R_i + R_j, rounded once from FP64
  float dclash;   // d_clash (2.6 for donor/acceptor pairs, else rsum)
  float dclash2;  // fl32(dclash)^2 in FP32
  uint32_t flags; // bit0 donor/acceptor pair, bit1 both hydrophobic
  double rsum64;
  double dclash64;
};

// Grid geometry of one pocket.
struct GridDev {
  float origin[3];
  float spacing, inv_spacing;
  int dims[3];
  float hi[3];
};

struct PocketDev {
  GridDev grid;
  const float* M;   // combined maps [8][nz][ny][nx]
  const float* G;   // per-term maps [8][K][nz][ny][nx] (may be null)
  int preset, n_terms;
  float w[kMaxTerms];
  // direct pair mode: receptor atoms sorted by cell (w = type bits), cell
  // offsets [ncells + 1], per (ligand type, receptor type) radius sum and
  // flags (x = rsum, y = flags bits)
  int inter_mode;
  const float4* rec;
  const int* cell_start;
  const float2* tp;
  float cell_origin[3];
  float inv_cell;
  int cell_dims[3];
  // E_MDN residue geometry (mdn_res = 0: no term): receptor atoms sorted by
  // residue, [begin, end) per residue, and per cell of a fine lattice over
  // the receptor box grown by the 5 A cutoff the residues that come within
  // 5 A of the cell
  int mdn_res;
  float mdn_w;
  const float4* res_xyz;
  const int2* res_range;
  const int* mcell_start;
  const int* mcell_res;
  float mcell_origin[3];
  float inv_mcell;
  int mcell_dims[3];
};

constexpr float kMdnCutoff = 5.0f;
constexpr float kMdnCell = 1.5f;

// Host build of the E_MDN residue geometry.
struct MdnGeometry {
  std::vector<float4> res_xyz;
  std::vector<int2> res_range;
  std::vector<int> cell_start, cell_res;
  float origin[3];
  int dims[3];
  int n_res = 0;
};
int build_mdn_geometry(int n_atoms, const float* xyz, const int32_t* residue, MdnGeometry& g, std::string& err);

// ---------------------------------------------------------------- host side

struct LigandHost {
  int n_atoms = 0, n_tors = 0, n_frags = 0, root = 0, height = 0, pocket = 0;
  double c0[3] = {0, 0, 0};
  float box_min[3] = {0, 0, 0}, box_max[3] = {0, 0, 0};
  std::vector<float> x0;               // [N*3] input coordinates (caller order)
  std::vector<uint8_t> type;           // caller order
  std::vector<int> atom_frag;          // caller order, fragment ids by lowest atom
  std::vector<int> frag_parent;        // [F]
  std::vector<int> bfs;                // [F]
  std::vector<int> tors_frag, tors_a, tors_b;  // [n_t]
  std::vector<int> pair_i, pair_j;     // caller order, lexicographic
  // packing (DFS order)
  std::vector<int> dfs_atom;           // new atom index -> caller atom index
  std::vector<int> atom_new;           // caller atom index -> new index
  std::vector<int> dfs_frag;           // new fragment id -> caller fragment id
  std::vector<int> frag_new;           // caller fragment id -> new id
};

// Builds the topology of one ligand; returns DOCK_OK or an error code with
// a message in `err`.
int prepare_ligand(int n, const uint8_t* element, const uint8_t* n_h, const float* xyz,
                   int n_bonds, const int32_t* bonds, const uint8_t* rotatable,
                   const float* box_min, const float* box_max, LigandHost& out, std::string& err);

void type_pair_table(int preset, TypePair table[kTypes * kTypes]);

// Intra-pair passes for groups whose lanes each own `apl` (1 or 2) atoms.  A
// pass is `width` slots (one per lane); slot s of pass k holds pair
// (slot_i, slot_j)[k * width + s], or -1 for an empty slot.  Every pair is in
// exactly one slot (in either orientation), and within a pass no atom is the
// first endpoint of more than cap / 2 slots nor the second endpoint of more
// than cap / 2.  Each pass the lane of slot s stores the pair force f (on its
// first endpoint) at entry s; entry `width` holds zero.
// pulls[k * n_pull + a] (n_pull = apl * width) names, byte by byte, the
// entries atom a adds (bytes 0 .. cap/2 - 1: slots where it is the first
// endpoint) and subtracts (bytes cap/2 .. cap - 1: slots where it is the
// second); unused bytes name the zero entry.  Plain stores and gathers: no
// LDS atomics.
constexpr int kMaxPull = 8;
// Staged bytes above which a ligand of more than 64 atoms keeps its strided
// pair list (8-byte records) instead of the pass layout: what a 256-thread
// sampler block of four 64-lane groups (5 KiB of slab each) can add to stay
// within 64 KiB of LDS.  The largest layouts of 65-70-atom ligands with
// ~2,100 pairs stage ~41 KiB.
constexpr size_t kPassStageBytes = 43 * 1024;
struct PassPlan {
  int n_pass = 0, cap = 0, n_pull = 0;
  std::vector<int> slot_i, slot_j;
  std::vector<uint64_t> pulls;
};
PassPlan schedule_passes(int n_atoms, const std::vector<int>& pi, const std::vector<int>& pj, int width,
                         int apl = 1);

void preset_weights(int preset, float* w, int* K);

}  // namespace dock
