/*
 * dock.h -- C ABI of the MI355X docking hot path (libdock.so).
 *
 * The library evaluates the TRIDS physics scoring function (arXiv
 * 2510.24186, Methods, "Scoring functions": E_long, E_clash, E_Hbond and
 * their weighted sum E_dock, without the learned MDN term) and its gradient
 * with respect to each pose's translation, rotation and torsion DOFs
 * (Methods, "Conformation sampling"), and drives many independent Metropolis
 * Monte Carlo + local-gradient trajectories per ligand (Fig. 2).  Receptor
 * terms are tabulated on per-ligand-type grid maps; ligand-internal pairs are
 * summed directly.
 *
 * Conventions shared by every call
 *  - Every call returns DOCK_OK (0) or a negative dock_status.  On error no
 *    output buffer is modified and dock_last_error() (thread-local) holds a
 *    message.  No C++ exception crosses the ABI.
 *  - "host" pointers are read during the call and copied; "device" pointers
 *    are HIP device memory owned by the caller (e.g. torch tensor storage).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *    enqueued asynchronously on it unless stated otherwise.
 *  - Handles are immutable after creation (runs excepted): calls that only
 *    read them do not race on them.  Use of the library from several host
 *    threads at once has not been verified, and the sampler does not
 *    support it (dock_sample).
 *  - Poses: q = (Tx, Ty, Tz, alpha, beta, gamma, theta_0 .. theta_{n_t-1}),
 *    row-major with a caller-chosen row stride q_stride >= 6 + n_t.  T is
 *    where the root fragment's centroid lands; R = Rz(alpha) Ry(beta)
 *    Rx(gamma) turns about it; theta_k are torsion deltas from the input
 *    pose.  Angles are radians; energies are in the score's units.
 */
#ifndef DOCK_H
#define DOCK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DOCK_ABI_VERSION 2
#define DOCK_MAX_ATOMS 128
#define DOCK_MAX_TORS 32
#define DOCK_N_TYPES 8
#define DOCK_MAX_TERMS 5

typedef enum {
  DOCK_OK = 0,
  DOCK_E_ARG = -1,      /* invalid argument, size or handle */
  DOCK_E_TOPOLOGY = -2, /* disconnected ligand, rotatable ring bond, bad bond */
  DOCK_E_LIMIT = -3,    /* N > DOCK_MAX_ATOMS, n_t > DOCK_MAX_TORS, LDS budget */
  DOCK_E_OOM = -4,      /* device or host allocation failed */
  DOCK_E_HIP = -5       /* a HIP runtime call failed */
} dock_status;

enum { DOCK_PRESET_TRIDS = 0, DOCK_PRESET_VINA = 1 };
/* Local refinement rules: Adam (the paper's choice, Methods), an Armijo line
 * search, and the alternatives the paper compares in Table S5. */
enum {
  DOCK_LOCAL_ADAM = 0,
  DOCK_LOCAL_LINESEARCH = 1,
  DOCK_LOCAL_SGD = 2,
  DOCK_LOCAL_RMSPROP = 3,
  DOCK_LOCAL_ADAGRAD = 4,
  DOCK_LOCAL_ADAMW = 5
};
enum { DOCK_FORM_PLAIN = 0, DOCK_FORM_BATCHED = 1 };
enum { DOCK_INTER_GRID = 0, DOCK_INTER_DIRECT = 1 };

typedef struct dock_pocket_s* dock_pocket_t;
typedef struct dock_ligands_s* dock_ligands_t;
typedef struct dock_run_s* dock_run_t;

/* ------------------------------------------------------------------------
 * Pocket: receptor atoms -> grid maps (Methods, E_long / E_clash / E_Hbond;
 * Discussion item 4: only pairs inside a cutoff are summed).
 *
 * G[t][k][node] = sum over receptor atoms i inside term k's cutoff of
 * phi_k(|node - r_i|; t, type_i); the combined map M[t] = sum_k w_k G[t][k].
 * Node (ix, iy, iz) sits at origin + spacing * (ix, iy, iz); layout
 * [t][k][iz][iy][ix] (x fastest).  The inside-cutoff test uses the FP32
 * squared distance ((dx*dx + dy*dy) + dz*dz) against fl32(c)^2, evaluated
 * without contraction; the terms and their sums are evaluated in FP64 and
 * stored as FP32.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t n_atoms;        /* receptor atoms, >= 0 */
  const float* xyz;       /* host [n_atoms * 3] */
  const uint8_t* type;    /* host [n_atoms], 0..7 (C_H C_P N_P N_D N_A O_A O_DA Cl_H) */
  float origin[3];        /* first node */
  float spacing;          /* > 0, Angstrom */
  int32_t dims[3];        /* nx, ny, nz, each in [2, 1024] */
  int32_t preset;         /* DOCK_PRESET_TRIDS (K = 3) or DOCK_PRESET_VINA (K = 5) */
  const float* weights;   /* host [K] or NULL for the preset's weights
                             (TRIDS 0.2 / 10 / 0.6, Methods E_dock) */
  int32_t keep_per_term;  /* nonzero: also keep G (needed by the adjoint) */
  int32_t inter_mode;     /* DOCK_INTER_GRID: receptor terms from the grid maps
                             (+ 10 |x - clamp(x)|_1 outside the map box);
                             DOCK_INTER_DIRECT: summed pair by pair over the
                             receptor atoms inside the cutoffs, found through a
                             cell list of half-cutoff cells (the paper's cutoff
                             pair kernel, Discussion item 4); no maps, no box
                             term, not usable by the differentiable form */
  const int32_t* residue; /* host [n_atoms] residue index per receptor atom
                             (0 .. n_res - 1, every index used) or NULL: the
                             residue geometry of the E_MDN term */
  float mdn_weight;       /* w_MDN (Methods E_dock: 1.0) */
} dock_pocket_desc;

/* E_MDN term (Methods, "Scoring functions"): for residue i and ligand atom
 * j, d_ij = the smallest distance from the atom to the residue's atoms,
 * P(d) = sum_k pi_k exp(-(d - mu_k)^2 / (2 sigma_k^2)), and
 * E_MDN = -sum over d_ij < 5 A of P(d_ij); E_dock adds mdn_weight * E_MDN.
 * The term is active in grid mode when the pocket has residues, mdn_weight
 * is nonzero and the ligands carry mixture parameters for as many residues
 * (dock_ligands_set_mdn); the gradient goes through d_ij at the nearest
 * atom (lowest index on ties).  The network that predicts the parameters is
 * not part of the library. */

/* Builds the maps on `stream`; the returned handle owns them.  The call
 * returns after enqueueing; the maps are ready when the stream reaches it. */
int dock_load_pocket(const dock_pocket_desc* desc, void* stream, dock_pocket_t* out);

/* Builds the maps of an existing grid-mode handle again, in place, on
 * `stream` (same receptor, grid and weights; kernels only, no allocation):
 * for a step that redoes the whole path, map build included.  Work that
 * reads the maps on other streams must be ordered against it by the caller.
 * Direct-mode handles have no maps: DOCK_OK, nothing enqueued. */
int dock_pocket_rebuild(dock_pocket_t p, void* stream);

/* Device pointer to the combined maps M [8][nz][ny][nx] (per_term = 0) or to
 * G [8][K][nz][ny][nx] (per_term = 1, only if kept).  Owned by the handle. */
int dock_pocket_maps(dock_pocket_t p, int32_t per_term, float** dev_ptr, int64_t* n_floats);
/* Copies the maps of dock_pocket_maps into `dst` (device, n_floats) on `stream`. */
int dock_pocket_copy_maps(dock_pocket_t p, int32_t per_term, float* dst, void* stream);
int dock_pocket_terms(dock_pocket_t p, int32_t* preset, int32_t* n_terms, float* weights /* host [K] */);
/* Frees the handle and its maps.  Returns DOCK_E_ARG (and frees nothing)
 * while a run created with this pocket is alive: free the run first. */
int dock_free_pocket(dock_pocket_t p);

/* ------------------------------------------------------------------------
 * Ligands: typing, torsion tree and intra-ligand pair list, on the host.
 *
 * Typing: C -> C_P if bonded to N/O else C_H; N -> N_D if it carries H, else
 * N_A if <= 2 heavy neighbours, else N_P; O -> O_DA if it carries H else O_A;
 * Cl -> Cl_H.  Fragments: components after removing rotatable bonds (ids by
 * lowest atom).  Root: the fragment of smallest tree height (lowest id on
 * ties); torsion k = k-th non-root fragment in breadth-first order (children
 * by id), axis a_k (parent side) -> b_k.  Pairs: atoms in different
 * fragments >= 4 bonds apart.  Box: bounds of the input pose unless given.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t n_ligands;           /* >= 1 */
  const int32_t* atom_off;     /* host [n_ligands + 1] */
  const uint8_t* element;      /* host [total atoms]: 0 C, 1 N, 2 O, 3 Cl */
  const uint8_t* n_h;          /* host [total atoms], implicit hydrogens */
  const float* xyz;            /* host [total atoms * 3], input pose */
  const int32_t* bond_off;     /* host [n_ligands + 1] */
  const int32_t* bonds;        /* host [total bonds * 2], ligand-local indices */
  const uint8_t* rotatable;    /* host [total bonds] */
  const float* box_min;        /* host [n_ligands * 3] or NULL */
  const float* box_max;        /* host [n_ligands * 3] or NULL */
  const int32_t* pocket_index; /* host [n_ligands] or NULL (all 0) */
  int32_t host_only;           /* nonzero: build topology only, no device upload
                                  (such a handle serves dock_ligand_* queries) */
} dock_ligand_desc;

/* Prepares the ligands on the host, one ligand per task on OMP_NUM_THREADS
 * threads (default: the hardware's, at most 64; the result does not depend
 * on the count), then uploads the packed arrays with synchronous copies.
 * On a failing ligand returns its code with the lowest failing index named
 * in dock_last_error(). */
int dock_load_ligands(const dock_ligand_desc* desc, void* stream, dock_ligands_t* out);

typedef struct {
  int32_t n_atoms, n_tors, n_frags, n_pairs, root, height, pocket;
  float c0[3];                 /* root-fragment centroid (FP64 mean, stored FP32) */
  float box_min[3], box_max[3];
  /* device layout of the pair records for large batched runs: passes of
   * pass_lanes slots (0 passes: pairs strided over the lanes), atoms per
   * lane, entries gathered per atom and pass, and the bytes staged in LDS
   * per work item */
  int32_t n_pass, pass_lanes, pass_apl, pull_cap, stage_bytes;
} dock_ligand_info_t;

int dock_ligand_info(dock_ligands_t L, int32_t lig, dock_ligand_info_t* info);
/* Integer topology in the caller's atom numbering (host outputs, nullable):
 * type [N], atom_frag [N], frag_parent [F] (-1 root), tors_frag [n_t],
 * tors_atoms [n_t * 2] (a_k, b_k), pairs [n_pairs * 2], bfs [F]. */
/* Mixture parameters of the E_MDN term for every ligand atom and residue:
 * params host [total_atoms][n_res][n_gauss][3] = (pi, mu, sigma), atoms in
 * the caller's order (dock_ligand_desc), sigma > 0, 1 <= n_gauss <= 16.
 * Copied; replaces earlier parameters.  n_res must match the pockets the
 * ligands are scored against. */
int dock_ligands_set_mdn(dock_ligands_t L, int32_t n_res, int32_t n_gauss, const float* params);

int dock_ligand_topology(dock_ligands_t L, int32_t lig, uint8_t* type, int32_t* atom_frag,
                         int32_t* frag_parent, int32_t* tors_frag, int32_t* tors_atoms,
                         int32_t* pairs, int32_t* bfs);
int dock_ligands_count(dock_ligands_t L, int32_t* n_ligands, int32_t* max_atoms,
                       int32_t* max_tors, int64_t* total_atoms);
/* Returns DOCK_E_ARG (and frees nothing) while a run over L is alive. */
int dock_free_ligands(dock_ligands_t L);

/* ------------------------------------------------------------------------
 * Score and gradient of arbitrary poses (teacher input, no sampling).
 * E = sum_i trilerp(M[t_i], x_i) + 10 |x_i - clamp(x_i)|_1 + E_intra, and
 * dE/dq by the chain rule (Discussion item 3).
 *   pose_lig  device [n_poses] int32 ligand of each pose
 *   q         device [n_poses * q_stride]
 *   E         device [n_poses]
 *   dEdq      device [n_poses * q_stride] or NULL (entries >= 6 + n_t untouched)
 *   xyz_out   device [n_poses * xyz_stride] or NULL: world coordinates in the
 *             caller's atom order, xyz_stride >= 3 * max_atoms
 * Each ligand's pocket is pockets[pocket_index].
 * ---------------------------------------------------------------------- */
int dock_score_grad(const dock_pocket_t* pockets, int32_t n_pockets, dock_ligands_t L,
                    int64_t n_poses, const int32_t* pose_lig, const float* q, int32_t q_stride,
                    float* E, float* dEdq, float* xyz_out, int32_t xyz_stride, void* stream);

/* ------------------------------------------------------------------------
 * Differentiable form.  The score is linear in the per-term maps and the
 * weights (Methods, E_dock: a weighted sum of pairwise terms):
 *   E = sum_k w_k (sum_i trilerp(G[t_i][k], x_i) + sum_pairs phi_k(r_ij)) + E_out
 * dock_score_terms evaluates it with caller-supplied maps and weights;
 * dock_score_adjoint ACCUMULATES (+=) the gradients of L = sum_p dLdE[p] E_p
 *   dL/dG[t][k][node]  trilinear corner weights x w_k x dLdE,
 *   dL/dw_k            dLdE x (per-term map sum + per-term pair sum),
 *   dL/dx              dLdE x dE/dx (caller atom order), and
 *   dL/dq              dLdE x dE/dq (DOF mode only),
 * recomputing the forward kinematics from q instead of storing coordinates.
 * Poses are given either as DOFs (q, q_stride; xyz = NULL) or as world
 * coordinates (xyz, xyz_stride >= 3 * max atoms, caller atom order; q = NULL).
 *   G      host array [n_pockets] of device pointers to [8][K][nz][ny][nx];
 *          a NULL entry uses the pocket's kept per-term maps
 *   w      device [n_pockets * K]
 *   dLdG   host array [n_pockets] of device pointers (entries nullable) or NULL
 *   dLdw   device [n_pockets * K] or NULL;  dLdq, dLdx device or NULL
 * All pockets of a call share one preset; n_pockets <= 16.
 *   deterministic  0: dL/dG and dL/dw by float atomics (summation order, and
 *                     so the last bits, vary from call to call);
 *                  1: bitwise repeatable.  dL/dG is summed as 64-bit
 *                     integers: every corner contribution is rounded once to
 *                     a multiple of 2^(e - 62), where 2^e bounds any node's
 *                     sum (n_poses x max_p |dLdE_p| N_p x max_k |w_k|, per
 *                     pocket), so the sum is exact and order-free; then it is
 *                     converted and added to dLdG.  dL/dw is reduced over the
 *                     poses in a fixed order.  Scratch (8 bytes per dL/dG
 *                     entry, 4 (K + 1) bytes per pose) is allocated and
 *                     released on the stream.  Non-finite dLdE or w make
 *                     that pocket's dL/dG NaN.
 * Ligand-internal pair forces are summed as fixed point in either mode, so
 * E, dL/dq and dL/dx never depend on timing.
 * ---------------------------------------------------------------------- */
int dock_score_terms(const dock_pocket_t* pockets, int32_t n_pockets, dock_ligands_t L,
                     int64_t n_poses, const int32_t* pose_lig, const float* q, int32_t q_stride,
                     const float* xyz, int32_t xyz_stride, const float* const* G, const float* w,
                     float* E, void* stream);
int dock_score_adjoint(const dock_pocket_t* pockets, int32_t n_pockets, dock_ligands_t L,
                       int64_t n_poses, const int32_t* pose_lig, const float* q, int32_t q_stride,
                       const float* xyz, int32_t xyz_stride, const float* const* G, const float* w,
                       const float* dLdE, float* const* dLdG, float* dLdw, float* dLdq, float* dLdx,
                       int32_t deterministic, void* stream);

/* ------------------------------------------------------------------------
 * Sampling (Methods, "Conformation sampling"; Fig. 2).  Each trajectory
 * starts from random DOFs, then each MC step resamples one scalar DOF
 * uniformly over its range, refines with n_local local steps (Adam, lr 0.1,
 * moments reset per MC step; or Armijo line search) and accepts iff
 * u < exp(-mc_beta * dE).  Randoms: Philox4x32-10 with key (ligand, seed)
 * and counter (trajectory, step, purpose, block).
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t n_traj;           /* trajectories per ligand, >= 1 */
  int32_t n_steps;          /* MC steps, >= 0 */
  int32_t n_local;          /* local steps per MC step, >= 0 */
  int32_t local_opt;        /* DOCK_LOCAL_*: Adam (lr, beta1, beta2, eps), line search,
                               SGD (lr), RMSprop (lr, rms_alpha, eps), AdaGrad (lr, eps),
                               AdamW (Adam + weight_decay); state resets every MC step */
  float lr, beta1, beta2, eps;
  float mc_beta;            /* 0.069 */
  uint32_t seed;
  int32_t form;             /* DOCK_FORM_PLAIN: one launch per ligand;
                               DOCK_FORM_BATCHED: ragged-packed persistent launches */
  int32_t use_graph;        /* batched: replay the launch sequence as a hipGraph */
  int32_t steps_per_launch; /* 0: all steps in one launch per bucket */
  int32_t record_trace;     /* store q, E, dE/dq of every evaluation (tests) */
  int32_t lanes_per_pose;   /* 0: planner choice; else 16, 32 or 64: a wider group
                               for ligands laid out one atom per lane (ligands with
                               two atoms per lane keep their width) */
  float rms_alpha;          /* RMSprop smoothing (0.99) */
  float weight_decay;       /* AdamW decoupled weight decay (0.01) */
  int32_t trace_lig_stride; /* record_trace: log ligands l with l % stride == 0
                               (0 or 1: every ligand) */
  int32_t trace_traj;       /* record_trace: log trajectories t < trace_traj of those
                               ligands (0: all) */
} dock_sample_params;

void dock_sample_params_default(dock_sample_params* p);

/* Creates a run, draws the initial poses, scores them and advances every
 * trajectory by p->n_steps MC steps.  The run owns its state buffers.
 * In the batched form the lane buckets run in groups, one per occupancy
 * class (blocks per CU) of the buckets whose grid fills the device, highest
 * first, each group after the previous one (smaller buckets join the first);
 * within a group the first bucket runs on `stream` and the others on side
 * streams forked from `stream` and joined back into it.  The library keeps
 * a pool of side streams per device for the life of the process, shared by
 * all runs.  Runs are created, advanced, restarted and freed from one host
 * thread at a time: with use_graph = 1 (the default) the first MC-step
 * phase of a run is captured as a graph through the shared side streams,
 * and runs used from several threads at once are not supported.
 * A run's ligands of 33-64 atoms are laid out two atoms per lane when its
 * trajectories of such ligands fill at least two waves per wave slot of the
 * device (two poses per wavefront), else one atom per lane. */
int dock_sample(const dock_pocket_t* pockets, int32_t n_pockets, dock_ligands_t L,
                const dock_sample_params* p, void* stream, dock_run_t* out);
/* Autotuner.  For every lane configuration that L's ligands fall into
 * (group width 16/32/64 lanes, 1-2 atoms per lane), times `trial_steps` MC
 * steps of the batched sampler with p's settings for each candidate: blocks
 * of 64, 128 or 256 threads (trajectories per workgroup = block / width) and
 * the natural or the next wider group width.  The fastest is kept in a
 * process-wide cache keyed by (GPU architecture, configuration) that
 * dock_sample consults when lanes_per_pose == 0.  Random streams depend on
 * (ligand, trajectory, step) only, so tuning never changes which numbers a
 * trajectory draws.  Synchronizes `stream`. */
int dock_autotune(const dock_pocket_t* pockets, int32_t n_pockets, dock_ligands_t L,
                  const dock_sample_params* p, int32_t trial_steps, void* stream);
/* The cache as JSON text into buf (host, cap bytes, NUL-terminated);
 * *needed (nullable) receives the size required. */
int dock_autotune_report(char* buf, int32_t cap, int32_t* needed);
int dock_autotune_clear(void);
/* Puts one entry into the cache (as dock_autotune_report lists them), for
 * restoring a cache saved from an earlier process: for natural
 * configuration (lanes, atoms_per_lane) on architecture `arch`, run groups
 * of chosen_lanes lanes in blocks of `block` threads.  DOCK_E_ARG unless
 * lanes is 16/32/64, atoms_per_lane 1/2, chosen_lanes the natural width
 * (or twice it, at most 64, with one atom per lane) and block 64/128/256
 * holds at least one group. */
int dock_autotune_set(const char* arch, int32_t lanes, int32_t atoms_per_lane, int32_t chosen_lanes,
                      int32_t block, float trial_ms);

/* Advances every trajectory by n_steps more MC steps (resume). */
int dock_run_advance(dock_run_t r, int32_t n_steps, void* stream);
/* Starts the run over with a new seed: every trajectory redraws its initial
 * pose and takes the run's n_steps MC steps again, in the run's own buffers
 * with its plan and launches, exactly as dock_sample with that seed would.
 * Enqueues kernels only (no allocation, no host synchronisation, no memset):
 * repeated docking of the same ligand set without per-call setup. */
int dock_run_restart(dock_run_t r, uint32_t seed, void* stream);

typedef struct {
  int32_t n_ligands, n_traj, q_stride, step;
  float* q_cur;       /* device [n_ligands * n_traj * q_stride] */
  float* E_cur;       /* device [n_ligands * n_traj] */
  float* q_best;      /* device [n_ligands * n_traj * q_stride] */
  float* E_best;      /* device [n_ligands * n_traj] */
  int32_t* n_evals;   /* device [n_ligands * n_traj], evaluations so far */
  float* trace;       /* device, record_trace only: per logged trajectory
                         [trace_cap][2 * q_stride + 1] rows (q, dE/dq, E);
                         trajectory t of ligand l (l % trace_lig_stride == 0,
                         t < trace_traj) is block (l / trace_lig_stride) *
                         trace_traj + t */
  int32_t trace_cap;  /* rows per trajectory */
  int32_t trace_lig_stride, trace_traj;  /* as applied (>= 1) */
  int32_t n_trace;    /* logged trajectories */
} dock_run_view;

int dock_run_view_get(dock_run_t r, dock_run_view* v);
/* Copies the run's state into caller device buffers laid out as in
 * dock_run_view (each nullable) on `stream`.  Pose slots past a ligand's
 * n_dof are zero (or what dock_run_set_state last put there). */
int dock_run_copy_state(dock_run_t r, float* q_cur, float* E_cur, float* q_best, float* E_best,
                        int32_t* n_evals, float* trace, void* stream);
/* Replaces the trajectory state (checkpoint restore).  Device inputs laid out
 * as in dock_run_view; `step` is the number of MC steps already taken. */
int dock_run_set_state(dock_run_t r, const float* q_cur, const float* E_cur, const float* q_best,
                       const float* E_best, int32_t step, void* stream);
/* Device time (ms) of the sampler launches of the last dock_sample /
 * dock_run_advance call, measured with HIP events on the run's stream
 * (blocks until they complete). */
int dock_run_kernel_ms(dock_run_t r, float* ms);
/* Per-launch record of the last dock_sample / dock_run_advance call.
 * Durations come from HIP events recorded around each sampler launch on the
 * run's stream (not available when the launches were replayed as a graph:
 * ms = -1 then).  bucket: index of the lane configuration (see dock_run_plan). */
typedef struct {
  int32_t bucket, lanes_per_pose, atoms_per_lane, block, grid, n_items, init, step_count;
  float ms;
} dock_launch_stat;
int dock_run_launch_stats(dock_run_t r, dock_launch_stat* out, int32_t cap, int32_t* n);
/* Lane configuration chosen for each ligand: lig_bucket [n_ligands] (host,
 * nullable); bucket_lanes / bucket_apl [n_buckets] (host, nullable). */
int dock_run_plan(dock_run_t r, int32_t* lig_bucket, int32_t* bucket_lanes, int32_t* bucket_apl,
                  int32_t* n_buckets);
int dock_free_run(dock_run_t r);

/* ------------------------------------------------------------------------
 * Best poses (Methods, "Conformation sampling": rank, cluster, top N;
 * E_screen = E / (1 + w_tor N_tor), Methods E_screen).  Per ligand, the
 * n_traj candidates (E_best, q_best) are ranked by E (ties: lower
 * trajectory), then greedily kept unless their heavy-atom RMSD (atom order,
 * no superposition) to a kept pose is below rmsd_cluster, up to top_n.
 * Outputs are device arrays [n_ligands * top_n (* q_stride | * xyz_stride)];
 * unused slots get E = +inf and idx = -1.
 * ---------------------------------------------------------------------- */
int dock_best_poses(dock_ligands_t L, int32_t n_traj, const float* E_best, const float* q_best,
                    int32_t q_stride, int32_t top_n, float rmsd_cluster, float w_tor,
                    float* E_out, float* E_screen, float* q_out, int32_t* idx_out,
                    float* xyz_out, int32_t xyz_stride, int32_t* n_out, void* stream);

/* Adjoint of the grid-map build for the TRIDS terms (Methods, E_long,
 * E_clash, E_Hbond): with lam = dL/dG for the per-term maps (device float
 * [8][3][nz][ny][nx], the layout dock_pocket_copy_maps returns per term),
 * accumulates (+=)
 *   dLdxyz   [n_atoms * 3] device float, caller atom order: dL/d receptor xyz
 *   dLdtheta [DOCK_MAP_THETA] device double: dL/d(mu_long, sigma_long, mu_hb,
 *            sigma_hb, d_clash_hb, R_0 .. R_7) at the library's constants
 *            (3, sqrt 2, 2.88, 0.3, 2.6, the type radii)
 * (either may be null).  Cutoff decisions are the map build's; the fixed
 * cutoffs (10 A, 3.4 A) are not differentiated.  Grid-mode TRIDS pockets
 * only (DOCK_E_ARG otherwise).  Asynchronous on the stream. */
#define DOCK_MAP_THETA 13
int dock_pocket_map_adjoint(dock_pocket_t p, const float* dLdG, float* dLdxyz, double* dLdtheta,
                            void* stream);

/* Screening rank across ligands (Methods, E_screen: virtual screening
 * ranks compounds by it).  scores: device, one score per ligand at
 * scores[i * stride] (for instance a ligand's best E_screen, column 0 of
 * dock_best_poses' E_screen with stride = top_n), n ligands.  Writes the
 * top_k lowest (1 <= top_k <= 1024) to score_out / lig_out (device
 * [top_k]) in ascending order; equal scores rank by lower ligand index,
 * -0.0 equals +0.0, NaN ranks after +inf; slots beyond n get +inf and -1.
 * Allocates its scratch on the stream (stream-ordered) and returns at once. */
int dock_screen_rank(const float* scores, int64_t n, int32_t stride, int32_t top_k, float* score_out,
                     int32_t* lig_out, void* stream);

/* dock_screen_rank without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, ordering and outputs.
 * The intermediate passes run in a static device array of
 * 4 * DOCK_NOALLOC_RANK_ENTRIES * 4 bytes (4 MiB) that each GPU the library
 * runs on holds until the process ends; the call needs
 * ceil(n / 2048) * top_k <= DOCK_NOALLOC_RANK_ENTRIES when n > 2048 and
 * returns DOCK_E_LIMIT otherwise (e.g. top_k = 1024 allows n up to 524,288,
 * top_k = 16 up to 2^31 - 2).  Every call on one GPU shares that array:
 * calls that overlap on one GPU (other streams, other threads) race and
 * give wrong results; calls ordered on one stream are safe.  The first call
 * on a device looks up the array's address there (no allocation). */
#define DOCK_NOALLOC_RANK_ENTRIES 262144
int dock_screen_rank_noalloc(const float* scores, int64_t n, int32_t stride, int32_t top_k,
                             float* score_out, int32_t* lig_out, void* stream);

/* Raw Philox4x32-10 blocks from the sampler's generator (Salmon et al.,
 * SC'11): out[4i..4i+3] = Philox(counter = counters[4i..4i+3], key = (k0, k1)).
 * counters, out: device [n * 4] uint32.  For checking the random stream. */
int dock_philox(const uint32_t* counters, uint32_t k0, uint32_t k1, int64_t n, uint32_t* out,
                void* stream);

/* Utilities */
const char* dock_last_error(void);
int dock_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DOCK_H */
