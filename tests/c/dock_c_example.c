/* A C consumer of libdock: reads a small docking problem from a binary file,
 * scores the given poses with their gradients, runs the batched sampler,
 * keeps the best poses, and writes the results to a binary file.  Device
 * memory comes from the HIP runtime; every library call takes plain
 * pointers.  The tests build it with gcc -std=c99 and compare its output
 * with the Python binding's on the same inputs.
 *
 *   dock_c_example IN OUT
 *
 * IN (little endian):
 *   int32  n_rec, preset, nx, ny, nz, n_w
 *   f32    origin[3], spacing, weights[n_w]
 *   f32    rec_xyz[n_rec * 3];  u8 rec_type[n_rec]
 *   int32  n_lig, n_atoms, n_bonds
 *   int32  atom_off[n_lig + 1];  u8 element[n_atoms], n_h[n_atoms]
 *   f32    xyz[n_atoms * 3]
 *   int32  bond_off[n_lig + 1], bonds[2 * n_bonds];  u8 rotatable[n_bonds]
 *   int32  n_poses, q_stride;  int32 pose_lig[n_poses];  f32 q[n_poses * q_stride]
 *   int32  n_traj, n_steps, seed, top_n
 * OUT:
 *   f32    E[n_poses], dEdq[n_poses * q_stride], E_best[n_lig * n_traj],
 *          best_E[n_lig * top_n];  int32 best_idx[n_lig * top_n], best_n[n_lig]
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "dock.h"

static FILE* g_in;

static void die(const char* what, const char* detail) {
  fprintf(stderr, "dock_c_example: %s: %s\n", what, detail);
  exit(1);
}
#define DOCK(call)                                     \
  do {                                                 \
    if ((call) != DOCK_OK) die(#call, dock_last_error()); \
  } while (0)
#define HIP(call)                                                     \
  do {                                                                \
    hipError_t e_ = (call);                                           \
    if (e_ != hipSuccess) die(#call, hipGetErrorString(e_));          \
  } while (0)

static void* read_n(size_t elem, size_t n) {
  void* p = malloc(elem * (n ? n : 1));
  if (!p) die("malloc", "out of memory");
  if (n && fread(p, elem, n, g_in) != n) die("read", "input file too short");
  return p;
}
static int32_t read_i32(void) {
  int32_t v;
  if (fread(&v, 4, 1, g_in) != 1) die("read", "input file too short");
  return v;
}
static void* to_device(const void* host, size_t bytes) {
  void* d = NULL;
  HIP(hipMalloc(&d, bytes ? bytes : 4));
  if (bytes) HIP(hipMemcpy(d, host, bytes, hipMemcpyHostToDevice));
  return d;
}
static void write_device(FILE* f, const void* dev, size_t bytes) {
  void* h = malloc(bytes ? bytes : 1);
  if (!h) die("malloc", "out of memory");
  if (bytes) HIP(hipMemcpy(h, dev, bytes, hipMemcpyDeviceToHost));
  if (bytes && fwrite(h, 1, bytes, f) != bytes) die("write", "output file");
  free(h);
}

int main(int argc, char** argv) {
  if (argc != 3) die("usage", "dock_c_example IN OUT");
  g_in = fopen(argv[1], "rb");
  if (!g_in) die("open", argv[1]);

  /* ---- pocket: maps built on the default stream from host arrays */
  dock_pocket_desc pd = {0};
  pd.n_atoms = read_i32();
  pd.preset = read_i32();
  for (int k = 0; k < 3; ++k) pd.dims[k] = read_i32();
  const int32_t n_w = read_i32();
  float* head = (float*)read_n(4, 4);
  for (int k = 0; k < 3; ++k) pd.origin[k] = head[k];
  pd.spacing = head[3];
  float* weights = (float*)read_n(4, (size_t)n_w);
  float* rec_xyz = (float*)read_n(4, (size_t)pd.n_atoms * 3);
  uint8_t* rec_type = (uint8_t*)read_n(1, (size_t)pd.n_atoms);
  pd.xyz = rec_xyz;
  pd.type = rec_type;
  pd.weights = n_w > 0 ? weights : NULL;
  pd.inter_mode = DOCK_INTER_GRID;
  pd.mdn_weight = 1.0f;
  dock_pocket_t pocket = NULL;
  DOCK(dock_load_pocket(&pd, NULL, &pocket));

  /* ---- ligands: typing, torsion tree and pair lists on the host */
  dock_ligand_desc ld = {0};
  ld.n_ligands = read_i32();
  const int32_t n_atoms = read_i32(), n_bonds = read_i32();
  int32_t* atom_off = (int32_t*)read_n(4, (size_t)ld.n_ligands + 1);
  uint8_t* element = (uint8_t*)read_n(1, (size_t)n_atoms);
  uint8_t* n_h = (uint8_t*)read_n(1, (size_t)n_atoms);
  float* xyz = (float*)read_n(4, (size_t)n_atoms * 3);
  int32_t* bond_off = (int32_t*)read_n(4, (size_t)ld.n_ligands + 1);
  int32_t* bonds = (int32_t*)read_n(4, (size_t)n_bonds * 2);
  uint8_t* rotatable = (uint8_t*)read_n(1, (size_t)n_bonds);
  ld.atom_off = atom_off;
  ld.element = element;
  ld.n_h = n_h;
  ld.xyz = xyz;
  ld.bond_off = bond_off;
  ld.bonds = bonds;
  ld.rotatable = rotatable;
  dock_ligands_t lig = NULL;
  DOCK(dock_load_ligands(&ld, NULL, &lig));
  int32_t n_lig = 0, max_atoms = 0, max_tors = 0;
  int64_t total_atoms = 0;
  DOCK(dock_ligands_count(lig, &n_lig, &max_atoms, &max_tors, &total_atoms));

  /* ---- score and gradient of the given poses */
  const int32_t n_poses = read_i32(), q_stride = read_i32();
  if (q_stride < 6 + max_tors) die("input", "q_stride below 6 + max torsions");
  int32_t* pose_lig = (int32_t*)read_n(4, (size_t)n_poses);
  float* q = (float*)read_n(4, (size_t)n_poses * q_stride);
  int32_t* d_pose_lig = (int32_t*)to_device(pose_lig, (size_t)n_poses * 4);
  float* d_q = (float*)to_device(q, (size_t)n_poses * q_stride * 4);
  float *d_E = NULL, *d_g = NULL;
  HIP(hipMalloc((void**)&d_E, (size_t)(n_poses ? n_poses : 1) * 4));
  HIP(hipMalloc((void**)&d_g, (size_t)(n_poses ? n_poses : 1) * q_stride * 4));
  HIP(hipMemset(d_g, 0, (size_t)(n_poses ? n_poses : 1) * q_stride * 4));
  DOCK(dock_score_grad(&pocket, 1, lig, n_poses, d_pose_lig, d_q, q_stride, d_E, d_g, NULL, 0, NULL));

  /* ---- sampler (batched form) and best poses */
  dock_sample_params sp;
  dock_sample_params_default(&sp);
  sp.n_traj = read_i32();
  sp.n_steps = read_i32();
  sp.seed = (uint32_t)read_i32();
  const int32_t top_n = read_i32();
  sp.form = DOCK_FORM_BATCHED;
  dock_run_t run = NULL;
  DOCK(dock_sample(&pocket, 1, lig, &sp, NULL, &run));
  dock_run_view v;
  DOCK(dock_run_view_get(run, &v));
  const size_t nb = (size_t)n_lig * top_n;
  float *d_bE = NULL, *d_bS = NULL, *d_bq = NULL;
  int32_t *d_bi = NULL, *d_bn = NULL;
  HIP(hipMalloc((void**)&d_bE, nb * 4));
  HIP(hipMalloc((void**)&d_bS, nb * 4));
  HIP(hipMalloc((void**)&d_bq, nb * v.q_stride * 4));
  HIP(hipMalloc((void**)&d_bi, nb * 4));
  HIP(hipMalloc((void**)&d_bn, (size_t)n_lig * 4));
  DOCK(dock_best_poses(lig, v.n_traj, v.E_best, v.q_best, v.q_stride, top_n, 1.0f, 0.01f, d_bE, d_bS, d_bq,
                       d_bi, NULL, 0, d_bn, NULL));
  HIP(hipDeviceSynchronize());

  FILE* out = fopen(argv[2], "wb");
  if (!out) die("open", argv[2]);
  write_device(out, d_E, (size_t)n_poses * 4);
  write_device(out, d_g, (size_t)n_poses * q_stride * 4);
  write_device(out, v.E_best, (size_t)n_lig * v.n_traj * 4);
  write_device(out, d_bE, nb * 4);
  write_device(out, d_bi, nb * 4);
  write_device(out, d_bn, (size_t)n_lig * 4);
  fclose(out);

  DOCK(dock_free_run(run));
  DOCK(dock_free_ligands(lig));
  DOCK(dock_free_pocket(pocket));
  hipFree(d_pose_lig);
  hipFree(d_q);
  hipFree(d_E);
  hipFree(d_g);
  hipFree(d_bE);
  hipFree(d_bS);
  hipFree(d_bq);
  hipFree(d_bi);
  hipFree(d_bn);
  fclose(g_in);
  free(head);
  free(weights);
  free(rec_xyz);
  free(rec_type);
  free(atom_off);
  free(element);
  free(n_h);
  free(xyz);
  free(bond_off);
  free(bonds);
  free(rotatable);
  free(pose_lig);
  free(q);
  printf("dock_c_example: %d poses scored, %d ligands x %d trajectories sampled\n", n_poses, n_lig, v.n_traj);
  return 0;
}
