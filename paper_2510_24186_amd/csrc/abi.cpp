// C ABI of libdock: argument validation, handle ownership, device upload,
// the sampling planner (lane configuration per ligand, ragged packing into
// work items, persistent launches, hipGraph replay) and the launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "dock_device.h"
#include "dock_internal.h"
#include "dock_kernels.h"

using namespace dock;

// ---------------------------------------------------------------- errors

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// Status of an exception caught at an entry point (every exported function
// with a body is a function-try-block, so none escapes into C callers): a
// failed host allocation is DOCK_E_OOM, a size the standard containers
// refuse is DOCK_E_ARG.  Called only from a catch handler.
static int exception_status() noexcept {
  int code = DOCK_E_ARG;
  const char* what = "unknown exception";
  try {
    throw;
  } catch (const std::bad_alloc&) {
    code = DOCK_E_OOM;
    what = "host allocation failed";
  } catch (const std::exception& e) {
    what = e.what();
  } catch (...) {
  }
  try {
    g_err = what;
  } catch (...) {
    g_err.clear();
  }
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(e_ == hipErrorOutOfMemory ? DOCK_E_OOM : DOCK_E_HIP,                  \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                   \
  } while (0)

template <class T>
static hipError_t dev_alloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
}

template <class T>
static void dev_free(T*& p) {
  if (p) (void)hipFree(const_cast<void*>(reinterpret_cast<const void*>(p)));
  p = nullptr;
}

// ---------------------------------------------------------------- handles

struct dock_pocket_s {
  PocketDev dev{};   // host copy of the device descriptor
  std::atomic<int> n_runs{0};  // live runs reading this pocket's device tables
  MapArgs build{};   // the map build's arguments (grid mode), for dock_pocket_rebuild
  int n_rec = 0;
  float4* d_rec = nullptr;
  float* d_M = nullptr;
  float* d_G = nullptr;
  float4* d_sorted = nullptr;   // direct mode
  int* d_cells = nullptr;
  float2* d_tp = nullptr;
  float4* d_res_xyz = nullptr;  // E_MDN residue geometry
  int2* d_res_range = nullptr;
  int* d_mcell_start = nullptr;
  int* d_mcell_res = nullptr;
};

static void free_pocket_device(dock_pocket_s* p) {
  dev_free(p->d_rec);
  dev_free(p->d_M);
  dev_free(p->d_G);
  dev_free(p->d_sorted);
  dev_free(p->d_cells);
  dev_free(p->d_tp);
  dev_free(p->d_res_xyz);
  dev_free(p->d_res_range);
  dev_free(p->d_mcell_start);
  dev_free(p->d_mcell_res);
}

struct dock_ligands_s {
  std::atomic<int> n_runs{0};  // live runs reading these device arrays
  std::vector<LigandHost> host;
  std::vector<LigDev> h_ligs;
  int n = 0, max_atoms = 0, max_tors = 0, max_pairs = 0, max_frags = 0;
  int max_alt_pairs = 0;  // largest staged alternative layout
  long long total_atoms = 0;
  bool host_only = false;
  LigDev* d_ligs = nullptr;
  float4* d_atoms = nullptr;
  FragDev* d_frags = nullptr;
  TorsDev* d_tors = nullptr;
  PairRec* d_pairs = nullptr;
  float4* d_mdn = nullptr;   // E_MDN mixture parameters (see LigandArrays)
  int mdn_res = 0, mdn_k = 0;
  LigandArrays arrays() const {
    return LigandArrays{d_ligs, d_atoms, d_frags, d_tors, d_pairs, d_mdn, mdn_res, mdn_k};
  }
};

// Device tables of PocketDev, cached per ordered list of pocket handles.
static std::mutex g_tab_mu;
static std::map<std::vector<dock_pocket_t>, PocketDev*> g_tables;

static int pocket_table(const dock_pocket_t* pockets, int n, const PocketDev** out) {
  std::vector<dock_pocket_t> key(pockets, pockets + n);
  std::lock_guard<std::mutex> lk(g_tab_mu);
  auto it = g_tables.find(key);
  if (it != g_tables.end()) {
    *out = it->second;
    return DOCK_OK;
  }
  std::vector<PocketDev> h(n);
  for (int i = 0; i < n; ++i) h[i] = pockets[i]->dev;
  PocketDev* d = nullptr;
  HIP_TRY(dev_alloc(&d, size_t(n)));
  hipError_t e = hipMemcpy(d, h.data(), sizeof(PocketDev) * n, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    dev_free(d);
    return fail(DOCK_E_HIP, std::string("pocket table upload: ") + hipGetErrorString(e));
  }
  g_tables[key] = d;
  *out = d;
  return DOCK_OK;
}

static void drop_tables_with(dock_pocket_t p) {
  std::lock_guard<std::mutex> lk(g_tab_mu);
  for (auto it = g_tables.begin(); it != g_tables.end();) {
    if (std::find(it->first.begin(), it->first.end(), p) != it->first.end()) {
      (void)hipDeviceSynchronize();
      dev_free(it->second);
      it = g_tables.erase(it);
    } else {
      ++it;
    }
  }
}

// ---------------------------------------------------------------- lane plan

// Wavefronts one CU holds with the sampler's register budget (3 per SIMD).
constexpr int kWavesPerCu = 12;

struct LaneCfg {
  int lpp, apl;
};

// Smallest group that gives every DOF, fragment and atom a lane: one atom per
// lane up to 32 atoms; two per lane above 64, and from 33 to 64 atoms when
// the DOFs and fragments fit 32 lanes (two poses per wavefront then share the
// per-pose work: FK transforms, scans, optimiser updates).
static LaneCfg lane_cfg(const LigDev& lg, int force_lpp, bool one_per_lane = false) {
  LaneCfg c;
  const bool mid = !one_per_lane && lg.n_atoms > 32 && lg.n_atoms <= 64 && lg.n_dof <= 32 &&
                   lg.n_frags <= 32;
  c.apl = (lg.n_atoms > 64 || mid) ? 2 : 1;
  const int need = std::max({(lg.n_atoms + c.apl - 1) / c.apl, lg.n_dof, lg.n_frags});
  c.lpp = need <= 16 ? 16 : (need <= 32 ? 32 : 64);
  if (lg.n_atoms > 64) c.lpp = 64;
  if (force_lpp > c.lpp && c.apl == 1) c.lpp = force_lpp;
  return c;
}

// One lane configuration wide enough for every ligand of a handle (the score
// and differentiable kernels launch one grid).
// These kernels run on the ligands' alternative (one atom per lane up to 64
// atoms) layouts: a launch holds few poses of each ligand.
static LaneCfg wide_cfg(const dock_ligands_s* L) {
  LaneCfg w{16, 1};
  for (const LigDev& g : L->h_ligs) {
    const LaneCfg c = lane_cfg(g, 0, true);
    w.lpp = std::max(w.lpp, c.lpp);
    w.apl = std::max(w.apl, c.apl);
  }
  if (w.apl == 2) w.lpp = 64;
  return w;
}

// Autotuner choices per natural lane configuration (lpp, apl): the group
// width and block size that measured fastest, process-wide, per device arch.
struct TuneChoice {
  int lpp, block;
  float ms;
};
static std::mutex g_tune_mu;
static std::map<std::tuple<std::string, int, int>, TuneChoice> g_tune;

static std::string device_arch() {
  static std::mutex mu;
  static std::map<int, std::string> names;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  std::lock_guard<std::mutex> lk(mu);
  auto it = names.find(dev);
  if (it != names.end()) return it->second;
  hipDeviceProp_t prop;
  std::string name = hipGetDeviceProperties(&prop, dev) == hipSuccess ? std::string(prop.gcnArchName) : "unknown";
  names[dev] = name;
  return name;
}

// Runs f(i) for i in [0, n) on up to OMP_NUM_THREADS (else the hardware's)
// host threads, at most 64.  f must not throw.
template <class F>
static void parallel_for(int n, F&& f) {
  int nt = int(std::thread::hardware_concurrency());
  if (const char* v = std::getenv("OMP_NUM_THREADS")) nt = std::atoi(v);
  nt = std::max(1, std::min({nt, 64, (n + 63) / 64}));
  std::atomic<int> next(0);
  auto work = [&] {
    for (int i; (i = next.fetch_add(1)) < n;) f(i);
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (std::thread& t : pool) t.join();
}

extern "C" {

const char* dock_last_error(void) { return g_err.c_str(); }
int dock_abi_version(void) { return DOCK_ABI_VERSION; }

// ================================================================ pocket

int dock_load_pocket(const dock_pocket_desc* d, void* stream, dock_pocket_t* out) try {
  if (!d || !out) return fail(DOCK_E_ARG, "null argument");
  if (d->n_atoms < 0 || (d->n_atoms > 0 && (!d->xyz || !d->type)))
    return fail(DOCK_E_ARG, "bad receptor arrays");
  if (d->preset != DOCK_PRESET_TRIDS && d->preset != DOCK_PRESET_VINA)
    return fail(DOCK_E_ARG, "unknown preset");
  if (d->inter_mode != DOCK_INTER_GRID && d->inter_mode != DOCK_INTER_DIRECT)
    return fail(DOCK_E_ARG, "unknown inter_mode");
  if (d->inter_mode == DOCK_INTER_DIRECT && d->keep_per_term)
    return fail(DOCK_E_ARG, "per-term maps need inter_mode DOCK_INTER_GRID");
  if (!(d->spacing > 0.f) || !std::isfinite(d->spacing)) return fail(DOCK_E_ARG, "bad spacing");
  for (int c = 0; c < 3; ++c) {
    if (d->dims[c] < 2 || d->dims[c] > 1024) return fail(DOCK_E_ARG, "grid dims must be in [2, 1024]");
    if (!std::isfinite(d->origin[c])) return fail(DOCK_E_ARG, "bad origin");
  }
  for (int i = 0; i < d->n_atoms; ++i) {
    if (d->type[i] >= kTypes) return fail(DOCK_E_ARG, "receptor type out of range");
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(d->xyz[3 * i + c])) return fail(DOCK_E_ARG, "non-finite receptor coordinate");
  }
  const long long nodes = (long long)d->dims[0] * d->dims[1] * d->dims[2];
  dock_pocket_s* p = new (std::nothrow) dock_pocket_s;
  if (!p) return fail(DOCK_E_OOM, "host allocation");
  PocketDev& pd = p->dev;
  int K = 0;
  preset_weights(d->preset, pd.w, &K);
  if (d->weights)
    for (int k = 0; k < K; ++k) {
      if (!std::isfinite(d->weights[k])) {
        delete p;
        return fail(DOCK_E_ARG, "non-finite weight");
      }
      pd.w[k] = d->weights[k];
    }
  for (int k = K; k < kMaxTerms; ++k) pd.w[k] = 0.f;
  pd.preset = d->preset;
  pd.n_terms = K;
  for (int c = 0; c < 3; ++c) {
    pd.grid.origin[c] = d->origin[c];
    pd.grid.dims[c] = d->dims[c];
    pd.grid.hi[c] = float(double(d->origin[c]) + double(d->spacing) * (d->dims[c] - 1));
  }
  pd.grid.spacing = d->spacing;
  pd.grid.inv_spacing = 1.0f / d->spacing;
  p->n_rec = d->n_atoms;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<float4> rec(std::max(1, d->n_atoms));
  for (int i = 0; i < d->n_atoms; ++i) {
    int bits = d->type[i];
    rec[i] = make_float4(d->xyz[3 * i], d->xyz[3 * i + 1], d->xyz[3 * i + 2], 0.f);
    std::memcpy(&rec[i].w, &bits, 4);
  }
  auto cleanup = [&](int code, const std::string& m) {
    free_pocket_device(p);
    delete p;
    return fail(code, m);
  };
  pd.inter_mode = d->inter_mode;
  // E_MDN residue geometry
  pd.mdn_res = 0;
  pd.mdn_w = 0.f;
  if (d->residue && d->n_atoms > 0) {
    if (!std::isfinite(d->mdn_weight)) return cleanup(DOCK_E_ARG, "non-finite mdn_weight");
    MdnGeometry mg;
    std::string err;
    const int rc = build_mdn_geometry(d->n_atoms, d->xyz, d->residue, mg, err);
    if (rc != DOCK_OK) return cleanup(rc, err);
    hipError_t e = dev_alloc(&p->d_res_xyz, mg.res_xyz.size());
    if (e == hipSuccess) e = dev_alloc(&p->d_res_range, mg.res_range.size());
    if (e == hipSuccess) e = dev_alloc(&p->d_mcell_start, mg.cell_start.size());
    if (e == hipSuccess) e = dev_alloc(&p->d_mcell_res, std::max<size_t>(1, mg.cell_res.size()));
    if (e != hipSuccess) return cleanup(DOCK_E_OOM, std::string("residue geometry allocation: ") + hipGetErrorString(e));
    e = hipMemcpy(p->d_res_xyz, mg.res_xyz.data(), sizeof(float4) * mg.res_xyz.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(p->d_res_range, mg.res_range.data(), sizeof(int2) * mg.res_range.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(p->d_mcell_start, mg.cell_start.data(), sizeof(int) * mg.cell_start.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !mg.cell_res.empty())
      e = hipMemcpy(p->d_mcell_res, mg.cell_res.data(), sizeof(int) * mg.cell_res.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return cleanup(DOCK_E_HIP, std::string("residue geometry upload: ") + hipGetErrorString(e));
    pd.mdn_res = mg.n_res;
    pd.mdn_w = d->mdn_weight;
    pd.res_xyz = p->d_res_xyz;
    pd.res_range = p->d_res_range;
    pd.mcell_start = p->d_mcell_start;
    pd.mcell_res = p->d_mcell_res;
    for (int c = 0; c < 3; ++c) {
      pd.mcell_origin[c] = mg.origin[c];
      pd.mcell_dims[c] = mg.dims[c];
    }
    pd.inv_mcell = 1.0f / kMdnCell;
  }
  if (d->inter_mode == DOCK_INTER_DIRECT) {
    // cell list: cells of half the largest cutoff over the receptor's bounds
    const double cell = (d->preset == DOCK_PRESET_TRIDS ? 10.0 : 8.0) / 2.0;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
      lo[c] = hi[c] = d->n_atoms ? d->xyz[c] : 0.0;
      for (int i = 1; i < d->n_atoms; ++i) {
        lo[c] = std::min(lo[c], double(d->xyz[3 * i + c]));
        hi[c] = std::max(hi[c], double(d->xyz[3 * i + c]));
      }
      pd.cell_origin[c] = float(lo[c]);
      pd.cell_dims[c] = std::max(1, int(std::floor((hi[c] - double(pd.cell_origin[c])) / cell)) + 1);
    }
    pd.inv_cell = float(1.0 / cell);
    const size_t ncell = size_t(pd.cell_dims[0]) * pd.cell_dims[1] * pd.cell_dims[2];
    if (ncell > (size_t(1) << 26)) return cleanup(DOCK_E_LIMIT, "receptor too extended for the cell list");
    std::vector<int> cidx(d->n_atoms), start(ncell + 1, 0);
    for (int i = 0; i < d->n_atoms; ++i) {
      int ic[3];
      for (int c = 0; c < 3; ++c) {
        const float u = (d->xyz[3 * i + c] - pd.cell_origin[c]) * pd.inv_cell;
        ic[c] = std::min(std::max(int(std::floor(u)), 0), pd.cell_dims[c] - 1);
      }
      cidx[i] = (ic[2] * pd.cell_dims[1] + ic[1]) * pd.cell_dims[0] + ic[0];
      start[cidx[i] + 1]++;
    }
    for (size_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    std::vector<float4> sorted(std::max(1, d->n_atoms));
    std::vector<int> fill(start.begin(), start.end() - 1);
    for (int i = 0; i < d->n_atoms; ++i) sorted[fill[cidx[i]]++] = rec[i];
    TypePair tab[kTypes * kTypes];
    type_pair_table(d->preset, tab);
    std::vector<float2> tp(kTypes * kTypes);
    for (int k = 0; k < kTypes * kTypes; ++k) {
      tp[k].x = tab[k].rsum;
      std::memcpy(&tp[k].y, &tab[k].flags, 4);
    }
    hipError_t e = dev_alloc(&p->d_sorted, sorted.size());
    if (e == hipSuccess) e = dev_alloc(&p->d_cells, start.size());
    if (e == hipSuccess) e = dev_alloc(&p->d_tp, tp.size());
    if (e != hipSuccess) return cleanup(DOCK_E_OOM, std::string("cell list allocation: ") + hipGetErrorString(e));
    e = hipMemcpy(p->d_sorted, sorted.data(), sizeof(float4) * sorted.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_cells, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_tp, tp.data(), sizeof(float2) * tp.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return cleanup(DOCK_E_HIP, std::string("cell list upload: ") + hipGetErrorString(e));
    pd.rec = p->d_sorted;
    pd.cell_start = p->d_cells;
    pd.tp = p->d_tp;
    pd.M = nullptr;
    pd.G = nullptr;
    *out = p;
    return DOCK_OK;
  }
  hipError_t e = dev_alloc(&p->d_rec, rec.size());
  if (e == hipSuccess) e = dev_alloc(&p->d_M, size_t(kTypes) * nodes);
  if (e == hipSuccess && d->keep_per_term) e = dev_alloc(&p->d_G, size_t(kTypes) * K * nodes);
  if (e != hipSuccess) return cleanup(DOCK_E_OOM, std::string("map allocation: ") + hipGetErrorString(e));
  e = hipMemcpy(p->d_rec, rec.data(), sizeof(float4) * rec.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return cleanup(DOCK_E_HIP, std::string("receptor upload: ") + hipGetErrorString(e));
  MapArgs a{};
  a.rec = p->d_rec;
  a.n_rec = d->n_atoms;
  a.grid = pd.grid;
  a.preset = d->preset;
  a.n_terms = K;
  for (int k = 0; k < kMaxTerms; ++k) a.w[k] = pd.w[k];
  type_pair_table(d->preset, a.tab);
  a.G = p->d_G;
  a.M = p->d_M;
  p->build = a;
  e = launch_map_build(a, s);
  if (e != hipSuccess) return cleanup(DOCK_E_HIP, std::string("map build: ") + hipGetErrorString(e));
  pd.M = p->d_M;
  pd.G = p->d_G;
  *out = p;
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_pocket_rebuild(dock_pocket_t p, void* stream) try {
  if (!p) return fail(DOCK_E_ARG, "null pocket");
  if (p->dev.inter_mode != DOCK_INTER_GRID) return DOCK_OK;  // direct mode: no maps
  HIP_TRY(launch_map_build(p->build, reinterpret_cast<hipStream_t>(stream)));
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_pocket_maps(dock_pocket_t p, int32_t per_term, float** dev_ptr, int64_t* n_floats) try {
  if (!p || !dev_ptr) return fail(DOCK_E_ARG, "null argument");
  if (p->dev.inter_mode == DOCK_INTER_DIRECT) return fail(DOCK_E_ARG, "a direct-mode pocket has no maps");
  const long long nodes = (long long)p->dev.grid.dims[0] * p->dev.grid.dims[1] * p->dev.grid.dims[2];
  if (per_term) {
    if (!p->d_G) return fail(DOCK_E_ARG, "per-term maps were not kept");
    *dev_ptr = p->d_G;
    if (n_floats) *n_floats = (long long)kTypes * p->dev.n_terms * nodes;
  } else {
    *dev_ptr = p->d_M;
    if (n_floats) *n_floats = (long long)kTypes * nodes;
  }
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_pocket_copy_maps(dock_pocket_t p, int32_t per_term, float* dst, void* stream) try {
  float* src = nullptr;
  int64_t n = 0;
  int rc = dock_pocket_maps(p, per_term, &src, &n);
  if (rc) return rc;
  if (!dst) return fail(DOCK_E_ARG, "null destination");
  HIP_TRY(hipMemcpyAsync(dst, src, size_t(n) * sizeof(float), hipMemcpyDeviceToDevice,
                         reinterpret_cast<hipStream_t>(stream)));
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_pocket_terms(dock_pocket_t p, int32_t* preset, int32_t* n_terms, float* weights) try {
  if (!p) return fail(DOCK_E_ARG, "null pocket");
  if (preset) *preset = p->dev.preset;
  if (n_terms) *n_terms = p->dev.n_terms;
  if (weights)
    for (int k = 0; k < p->dev.n_terms; ++k) weights[k] = p->dev.w[k];
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_free_pocket(dock_pocket_t p) try {
  if (!p) return DOCK_OK;
  if (p->n_runs.load() > 0)
    return fail(DOCK_E_ARG, "pocket is still used by " + std::to_string(p->n_runs.load()) +
                                " live run(s): free the runs first");
  drop_tables_with(p);
  (void)hipDeviceSynchronize();
  free_pocket_device(p);
  delete p;
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

// ================================================================ ligands

static void free_ligand_device(dock_ligands_s* L) {
  dev_free(L->d_ligs);
  dev_free(L->d_atoms);
  dev_free(L->d_frags);
  dev_free(L->d_tors);
  dev_free(L->d_pairs);
  dev_free(L->d_mdn);
}

static int bit_length(int v) {
  int b = 0;
  while (v > 0) {
    ++b;
    v >>= 1;
  }
  return b;
}

// Device records of one prepared ligand, with offsets into its own arrays
// (the merge in dock_load_ligands shifts them into the packed arrays).
struct PackedLigand {
  LigDev g;
  std::vector<float4> atoms;
  std::vector<FragDev> frags;
  std::vector<TorsDev> tors;
  std::vector<PairRec> pairs;
};

static void pack_ligand(const LigandHost& H, const TypePair* tab, PackedLigand& P) {
  std::vector<float4>& atoms = P.atoms;
  std::vector<FragDev>& frags = P.frags;
  std::vector<TorsDev>& tors = P.tors;
  std::vector<PairRec>& pairs = P.pairs;
  LigDev& g = P.g;
  std::memset(&g, 0, sizeof g);
  g.n_atoms = H.n_atoms;
  g.n_tors = H.n_tors;
  g.n_frags = H.n_frags;
  g.n_pairs = int(H.pair_i.size());
  g.atom_off = int(atoms.size());
  g.pair_off = int(pairs.size());
  g.frag_off = int(frags.size());
  g.tors_off = int(tors.size());
  g.pocket = H.pocket;
  g.n_dof = 6 + H.n_tors;
  g.fk_rounds = bit_length(H.height);
  for (int c = 0; c < 3; ++c) {
    g.c0[c] = float(H.c0[c]);
    g.box_min[c] = H.box_min[c];
    g.box_max[c] = H.box_max[c];
  }
  // coordinates relative to the root centroid c0 (FP64 difference, rounded
  // once): the rotation then acts on vectors of ligand size, not on
  // absolute positions, which keeps FP32 forward kinematics accurate
  for (int na = 0; na < H.n_atoms; ++na) {
    const int a = H.dfs_atom[na];
    const int bits = int(H.type[a]) | (H.frag_new[H.atom_frag[a]] << 8) | (a << 16);
    float4 v = make_float4(float(double(H.x0[3 * a]) - H.c0[0]), float(double(H.x0[3 * a + 1]) - H.c0[1]),
                           float(double(H.x0[3 * a + 2]) - H.c0[2]), 0.f);
    std::memcpy(&v.w, &bits, 4);
    atoms.push_back(v);
  }
  std::vector<int> frag_tors(H.n_frags, -1);
  for (int k = 0; k < H.n_tors; ++k) frag_tors[H.tors_frag[k]] = k;
  for (int nf = 0; nf < H.n_frags; ++nf) {
    const int f = H.dfs_frag[nf];
    FragDev fd{};
    if (H.frag_parent[f] < 0) {
      fd.parent = -1;
      fd.dof = -1;
    } else {
      const int k = frag_tors[f];
      const int a = H.tors_a[k], b = H.tors_b[k];
      double u[3], n2 = 0;
      for (int c = 0; c < 3; ++c) {
        u[c] = double(H.x0[3 * b + c]) - double(H.x0[3 * a + c]);
        n2 += u[c] * u[c];
      }
      const double inv = 1.0 / std::sqrt(n2);
      for (int c = 0; c < 3; ++c) {
        fd.u[c] = float(u[c] * inv);
        fd.xb[c] = float(double(H.x0[3 * b + c]) - H.c0[c]);
      }
      fd.parent = H.frag_new[H.frag_parent[f]];
      fd.dof = 6 + k;
    }
    frags.push_back(fd);
  }
  // torsion k moves the DFS subtree of its child fragment: a contiguous range
  std::vector<int> first(H.n_frags, 0), last(H.n_frags, 0);  // atom range per new frag id
  {
    std::vector<int> start(H.n_frags, -1), stop(H.n_frags, -1);
    for (int na = 0; na < H.n_atoms; ++na) {
      const int nf = H.frag_new[H.atom_frag[H.dfs_atom[na]]];
      if (start[nf] < 0) start[nf] = na;
      stop[nf] = na + 1;
    }
    // subtree end = max stop over the DFS subtree; in pre-order the subtree
    // of nf is nf .. nf + size - 1
    std::vector<int> size(H.n_frags, 1);
    for (int nf = H.n_frags - 1; nf >= 1; --nf) {
      const int par = frags[g.frag_off + nf].parent;
      size[par] += size[nf];
    }
    for (int nf = 0; nf < H.n_frags; ++nf) {
      first[nf] = start[nf];
      last[nf] = stop[nf + size[nf] - 1];
    }
  }
  for (int k = 0; k < H.n_tors; ++k) {
    const int nf = H.frag_new[H.tors_frag[k]];
    TorsDev t{};
    t.sub_begin = first[nf];
    t.sub_end = last[nf];
    t.a = H.atom_new[H.tors_a[k]];
    t.b = H.atom_new[H.tors_b[k]];
    tors.push_back(t);
  }
  // device pair records: with one atom per lane, passes of one group's
  // width whose forces are gathered per atom (no LDS atomics); with two
  // atoms per lane, the caller's order, strided over the lanes
  std::vector<int> pi_new(H.pair_i.size()), pj_new(H.pair_j.size());
  for (size_t p = 0; p < H.pair_i.size(); ++p) {
    pi_new[p] = H.atom_new[H.pair_i[p]];
    pj_new[p] = H.atom_new[H.pair_j[p]];
  }
  auto record = [&](int i0, int j0) {
    PairRec pr{};
    if (i0 < 0) {
      pr.w = kPairEmpty;
      pr.rsum = kEmptyRsum;
      return pr;
    }
    const int ti = H.type[H.dfs_atom[i0]], tj = H.type[H.dfs_atom[j0]];
    const TypePair& tp = tab[ti * kTypes + tj];
    pr.w = uint32_t(i0) | (uint32_t(j0) << 8) | (uint32_t(ti) << 16) | (uint32_t(tj) << 20) |
           (tp.flags << 24);
    pr.rsum = tp.rsum;
    return pr;
  };
  auto bits = [](float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
  };
  // one pair layout for a lane configuration, appended to `pairs`
  auto emit_layout = [&](const LaneCfg& lc) {
    PairLayout lay{};
    lay.pair_off = int(pairs.size());
    PassPlan plan;
    if (!pi_new.empty()) plan = schedule_passes(H.n_atoms, pi_new, pj_new, lc.lpp, lc.apl);
    // the pass layout stages 2 entries per slot and apl * cap pull bytes
    // per lane and pass; with two atoms per lane above 64 atoms it is kept
    // only where it fits the LDS budget
    const size_t pull_bytes = size_t(plan.n_pass) * lc.lpp * lc.apl * plan.cap;
    const size_t pass_entries = plan.slot_i.size() * 2 + pull_bytes / sizeof(PairRec) + 1;
    if (plan.n_pass > 0 &&
        (H.n_atoms <= 64 || pass_entries * sizeof(PairRec) <= kPassStageBytes)) {
      lay.n_pass = plan.n_pass;
      lay.pass_w = lc.lpp;
      lay.pass_apl = lc.apl;
      lay.pull_cap = plan.cap;
      // 16-byte slot records (pair word, radius sum, d_clash^2 as the
      // device squares it, log2 d_clash), then the pull bytes
      for (size_t s = 0; s < plan.slot_i.size(); ++s) {
        const int i0 = plan.slot_i[s], j0 = plan.slot_j[s];
        pairs.push_back(record(i0, j0));
        PairRec cl{};
        if (i0 >= 0) {
          const TypePair& tp = tab[H.type[H.dfs_atom[i0]] * kTypes + H.type[H.dfs_atom[j0]]];
          // negated for a donor/acceptor pair: the kernel tests
          // |d_clash^2| for the clash term and the sign for the
          // hydrogen-bond term
          cl.w = bits((tp.flags & 1u) ? -tp.dclash2 : tp.dclash2);
          cl.rsum = float(std::log2(double(tp.dclash)));
        }
        pairs.push_back(cl);
      }
      // pull bytes per (pass, lane): the lane's atoms one after the other,
      // the first `cap` bytes of each atom's pull list
      std::vector<uint8_t> pb(pull_bytes);
      const int per_lane = lc.apl * plan.cap;
      for (int ps = 0; ps < plan.n_pass; ++ps)
        for (int ln = 0; ln < lc.lpp; ++ln)
          for (int sa = 0; sa < lc.apl; ++sa) {
            const uint64_t w = plan.pulls[size_t(ps) * plan.n_pull + lc.apl * ln + sa];
            for (int b = 0; b < plan.cap; ++b)
              pb[(size_t(ps) * lc.lpp + ln) * per_lane + sa * plan.cap + b] = uint8_t(w >> (8 * b));
          }
      for (size_t o = 0; o < pb.size(); o += sizeof(PairRec)) {
        PairRec pw;
        std::memcpy(&pw, pb.data() + o, sizeof(PairRec));
        pairs.push_back(pw);
      }
      // padding: the kernel reads each 4-byte pull word with its successor
      pairs.push_back(PairRec{});
      lay.n_prec = int(plan.slot_i.size());
    } else {
      for (size_t p = 0; p < pi_new.size(); ++p) pairs.push_back(record(pi_new[p], pj_new[p]));
      lay.n_prec = int(pi_new.size());
    }
    lay.n_stage = int(pairs.size()) - lay.pair_off;
    return lay;
  };
  const LaneCfg lc = lane_cfg(g, 0), la = lane_cfg(g, 0, true);
  const PairLayout prim = emit_layout(lc);
  g.pair_off = prim.pair_off;
  g.n_prec = prim.n_prec;
  g.n_pass = prim.n_pass;
  g.pass_w = prim.pass_w;
  g.pull_cap = prim.pull_cap;
  g.pass_apl = prim.pass_apl;
  g.alt = (la.lpp == lc.lpp && la.apl == lc.apl) ? prim : emit_layout(la);
  g.n_stage = prim.n_stage;
}

int dock_load_ligands(const dock_ligand_desc* d, void* stream, dock_ligands_t* out) try {
  (void)stream;
  if (!d || !out) return fail(DOCK_E_ARG, "null argument");
  if (d->n_ligands < 1) return fail(DOCK_E_ARG, "n_ligands must be >= 1");
  if (!d->atom_off || !d->element || !d->n_h || !d->xyz || !d->bond_off)
    return fail(DOCK_E_ARG, "null ligand array");
  if (d->atom_off[0] != 0 || d->bond_off[0] != 0) return fail(DOCK_E_ARG, "offsets must start at 0");
  for (int i = 0; i < d->n_ligands; ++i)
    if (d->atom_off[i + 1] < d->atom_off[i] || d->bond_off[i + 1] < d->bond_off[i])
      return fail(DOCK_E_ARG, "offsets must be non-decreasing");
  if (d->bond_off[d->n_ligands] > 0 && (!d->bonds || !d->rotatable))
    return fail(DOCK_E_ARG, "null bond arrays");
  dock_ligands_s* L = new (std::nothrow) dock_ligands_s;
  if (!L) return fail(DOCK_E_OOM, "host allocation");
  L->n = d->n_ligands;
  L->host_only = d->host_only != 0;
  L->host.resize(L->n);
  // typing, fragments, torsion tree and pair list of every ligand, in
  // parallel; the first failing ligand (in order) is reported
  std::vector<int> prep_rc(L->n, DOCK_OK);
  std::vector<std::string> prep_err(L->n);
  parallel_for(L->n, [&](int i) {
    const int a0 = d->atom_off[i], b0 = d->bond_off[i];
    const int n = d->atom_off[i + 1] - a0, nb = d->bond_off[i + 1] - b0;
    try {
      prep_rc[i] = prepare_ligand(n, d->element + a0, d->n_h + a0, d->xyz + 3 * size_t(a0), nb,
                                  nb ? d->bonds + 2 * size_t(b0) : nullptr, nb ? d->rotatable + b0 : nullptr,
                                  d->box_min ? d->box_min + 3 * size_t(i) : nullptr,
                                  d->box_max ? d->box_max + 3 * size_t(i) : nullptr, L->host[i], prep_err[i]);
    } catch (const std::bad_alloc&) {
      prep_rc[i] = DOCK_E_OOM;
      prep_err[i] = "host allocation failed";
    } catch (...) {
      prep_rc[i] = DOCK_E_ARG;
      prep_err[i] = "preparation failed";
    }
  });
  for (int i = 0; i < L->n; ++i) {
    if (prep_rc[i] != DOCK_OK) {
      const int rc = prep_rc[i];
      const std::string msg = "ligand " + std::to_string(i) + ": " + prep_err[i];
      delete L;
      return fail(rc, msg);
    }
    L->host[i].pocket = d->pocket_index ? d->pocket_index[i] : 0;
    if (L->host[i].pocket < 0) {
      delete L;
      return fail(DOCK_E_ARG, "negative pocket index");
    }
  }
  // pack (DFS atom order): each ligand's records on its own, in parallel,
  // then concatenated in ligand order with the offsets shifted
  TypePair tab[kTypes * kTypes];
  type_pair_table(DOCK_PRESET_TRIDS, tab);
  std::vector<PackedLigand> packed(L->n);
  std::vector<int> pack_rc(L->n, DOCK_OK);
  parallel_for(L->n, [&](int i) {
    try {
      std::memset(&packed[i].g, 0, sizeof(LigDev));
      pack_ligand(L->host[i], tab, packed[i]);
    } catch (const std::bad_alloc&) {
      pack_rc[i] = DOCK_E_OOM;
    } catch (...) {
      pack_rc[i] = DOCK_E_ARG;
    }
  });
  for (int i = 0; i < L->n; ++i)
    if (pack_rc[i] != DOCK_OK) {
      delete L;
      return fail(pack_rc[i], "ligand " + std::to_string(i) + ": packing failed");
    }
  std::vector<float4> atoms;
  std::vector<FragDev> frags;
  std::vector<TorsDev> tors;
  std::vector<PairRec> pairs;
  L->h_ligs.resize(L->n);
  for (int i = 0; i < L->n; ++i) {
    PackedLigand& P = packed[i];
    LigDev& g = L->h_ligs[i];
    g = P.g;
    g.atom_off += int(atoms.size());
    g.frag_off += int(frags.size());
    g.tors_off += int(tors.size());
    g.pair_off += int(pairs.size());
    g.alt.pair_off += int(pairs.size());
    atoms.insert(atoms.end(), P.atoms.begin(), P.atoms.end());
    frags.insert(frags.end(), P.frags.begin(), P.frags.end());
    tors.insert(tors.end(), P.tors.begin(), P.tors.end());
    pairs.insert(pairs.end(), P.pairs.begin(), P.pairs.end());
    P = PackedLigand{};
    const LigandHost& H = L->host[i];
    L->max_atoms = std::max(L->max_atoms, H.n_atoms);
    L->max_tors = std::max(L->max_tors, H.n_tors);
    L->max_pairs = std::max({L->max_pairs, g.n_stage, g.alt.n_stage});
    L->max_alt_pairs = std::max(L->max_alt_pairs, g.alt.n_stage);
    L->max_frags = std::max(L->max_frags, H.n_frags);
    L->total_atoms += H.n_atoms;
  }
  if (!L->host_only) {
    hipError_t e = dev_alloc(&L->d_ligs, L->h_ligs.size());
    if (e == hipSuccess) e = dev_alloc(&L->d_atoms, atoms.size());
    if (e == hipSuccess) e = dev_alloc(&L->d_frags, frags.size());
    if (e == hipSuccess) e = dev_alloc(&L->d_tors, tors.size());
    if (e == hipSuccess) e = dev_alloc(&L->d_pairs, pairs.size());
    if (e == hipSuccess && !L->h_ligs.empty())
      e = hipMemcpy(L->d_ligs, L->h_ligs.data(), sizeof(LigDev) * L->h_ligs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !atoms.empty())
      e = hipMemcpy(L->d_atoms, atoms.data(), sizeof(float4) * atoms.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !frags.empty())
      e = hipMemcpy(L->d_frags, frags.data(), sizeof(FragDev) * frags.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !tors.empty())
      e = hipMemcpy(L->d_tors, tors.data(), sizeof(TorsDev) * tors.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !pairs.empty())
      e = hipMemcpy(L->d_pairs, pairs.data(), sizeof(PairRec) * pairs.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      free_ligand_device(L);
      delete L;
      return fail(e == hipErrorOutOfMemory ? DOCK_E_OOM : DOCK_E_HIP,
                  std::string("ligand upload: ") + hipGetErrorString(e));
    }
  }
  *out = L;
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_ligand_info(dock_ligands_t L, int32_t lig, dock_ligand_info_t* info) try {
  if (!L || !info) return fail(DOCK_E_ARG, "null argument");
  if (lig < 0 || lig >= L->n) return fail(DOCK_E_ARG, "ligand index out of range");
  const LigandHost& H = L->host[lig];
  info->n_atoms = H.n_atoms;
  info->n_tors = H.n_tors;
  info->n_frags = H.n_frags;
  info->n_pairs = int(H.pair_i.size());
  info->root = H.root;
  info->height = H.height;
  info->pocket = H.pocket;
  for (int c = 0; c < 3; ++c) {
    info->c0[c] = float(H.c0[c]);
    info->box_min[c] = H.box_min[c];
    info->box_max[c] = H.box_max[c];
  }
  const LigDev& g = L->h_ligs[lig];
  info->n_pass = g.n_pass;
  info->pass_lanes = g.pass_w;
  info->pass_apl = g.pass_apl;
  info->pull_cap = g.pull_cap;
  info->stage_bytes = g.n_stage * int(sizeof(PairRec));
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_ligand_topology(dock_ligands_t L, int32_t lig, uint8_t* type, int32_t* atom_frag,
                         int32_t* frag_parent, int32_t* tors_frag, int32_t* tors_atoms, int32_t* pairs,
                         int32_t* bfs) try {
  if (!L) return fail(DOCK_E_ARG, "null argument");
  if (lig < 0 || lig >= L->n) return fail(DOCK_E_ARG, "ligand index out of range");
  const LigandHost& H = L->host[lig];
  if (type) std::copy(H.type.begin(), H.type.end(), type);
  if (atom_frag) std::copy(H.atom_frag.begin(), H.atom_frag.end(), atom_frag);
  if (frag_parent) std::copy(H.frag_parent.begin(), H.frag_parent.end(), frag_parent);
  if (tors_frag) std::copy(H.tors_frag.begin(), H.tors_frag.end(), tors_frag);
  if (tors_atoms)
    for (int k = 0; k < H.n_tors; ++k) {
      tors_atoms[2 * k] = H.tors_a[k];
      tors_atoms[2 * k + 1] = H.tors_b[k];
    }
  if (pairs)
    for (size_t p = 0; p < H.pair_i.size(); ++p) {
      pairs[2 * p] = H.pair_i[p];
      pairs[2 * p + 1] = H.pair_j[p];
    }
  if (bfs) std::copy(H.bfs.begin(), H.bfs.end(), bfs);
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_ligands_set_mdn(dock_ligands_t L, int32_t n_res, int32_t n_gauss, const float* params) try {
  if (!L || !params) return fail(DOCK_E_ARG, "null argument");
  if (L->host_only) return fail(DOCK_E_ARG, "ligand handle was loaded host_only");
  if (n_res < 1 || n_gauss < 1 || n_gauss > 16) return fail(DOCK_E_ARG, "n_res >= 1 and 1 <= n_gauss <= 16");
  const size_t per_atom = size_t(n_res) * n_gauss;
  if (size_t(L->total_atoms) * per_atom > (size_t(1) << 31)) return fail(DOCK_E_LIMIT, "mixture table too large");
  std::vector<float4> tab(size_t(L->total_atoms) * per_atom);
  constexpr double kLog2e = 1.4426950408889634;
  for (int l = 0; l < L->n; ++l) {
    const LigandHost& H = L->host[l];
    const LigDev& g = L->h_ligs[l];
    for (int na = 0; na < H.n_atoms; ++na) {
      const size_t src = (size_t(g.atom_off) + size_t(H.dfs_atom[na])) * per_atom;
      const size_t dst = (size_t(g.atom_off) + size_t(na)) * per_atom;
      for (size_t q = 0; q < per_atom; ++q) {
        const double pi = params[3 * (src + q)], mu = params[3 * (src + q) + 1], sig = params[3 * (src + q) + 2];
        if (!std::isfinite(pi) || !std::isfinite(mu) || !(sig > 0.0) || !std::isfinite(sig))
          return fail(DOCK_E_ARG, "mixture parameters must be finite with sigma > 0");
        tab[dst + q] = make_float4(float(pi), float(mu), float(kLog2e / (2.0 * sig * sig)), float(1.0 / (sig * sig)));
      }
    }
  }
  float4* d = nullptr;
  hipError_t e = dev_alloc(&d, std::max<size_t>(1, tab.size()));
  if (e == hipSuccess && !tab.empty()) e = hipMemcpy(d, tab.data(), sizeof(float4) * tab.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    dev_free(d);
    return fail(DOCK_E_HIP, std::string("mixture table upload: ") + hipGetErrorString(e));
  }
  (void)hipDeviceSynchronize();
  dev_free(L->d_mdn);
  L->d_mdn = d;
  L->mdn_res = n_res;
  L->mdn_k = n_gauss;
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_ligands_count(dock_ligands_t L, int32_t* n_ligands, int32_t* max_atoms, int32_t* max_tors,
                       int64_t* total_atoms) try {
  if (!L) return fail(DOCK_E_ARG, "null argument");
  if (n_ligands) *n_ligands = L->n;
  if (max_atoms) *max_atoms = L->max_atoms;
  if (max_tors) *max_tors = L->max_tors;
  if (total_atoms) *total_atoms = L->total_atoms;
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_free_ligands(dock_ligands_t L) try {
  if (!L) return DOCK_OK;
  if (L->n_runs.load() > 0)
    return fail(DOCK_E_ARG, "ligand handle is still used by " + std::to_string(L->n_runs.load()) +
                                " live run(s): free the runs first");
  if (!L->host_only) (void)hipDeviceSynchronize();
  free_ligand_device(L);
  delete L;
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

// ================================================================ score

static int check_pockets(const dock_pocket_t* pockets, int n_pockets, dock_ligands_t L) {
  if (!pockets || n_pockets < 1) return fail(DOCK_E_ARG, "no pockets");
  for (int i = 0; i < n_pockets; ++i)
    if (!pockets[i]) return fail(DOCK_E_ARG, "null pocket handle");
  for (int i = 1; i < n_pockets; ++i)
    if (pockets[i]->dev.inter_mode != pockets[0]->dev.inter_mode)
      return fail(DOCK_E_ARG, "pockets of one call must share inter_mode");
  for (int i = 0; i < L->n; ++i)
    if (L->host[i].pocket >= n_pockets) return fail(DOCK_E_ARG, "ligand pocket index out of range");
  if (L->host_only) return fail(DOCK_E_ARG, "ligand handle was loaded host_only");
  for (int i = 0; i < n_pockets; ++i) {
    const PocketDev& pd = pockets[i]->dev;
    if (pd.mdn_res > 0 && pd.mdn_w != 0.f && L->d_mdn && L->mdn_res != pd.mdn_res)
      return fail(DOCK_E_ARG, "E_MDN parameters cover a different number of residues than the pocket");
  }
  return DOCK_OK;
}

// Kernel mode of a call: direct pair sums, grid maps with the E_MDN term
// (some pocket has residues and a weight, and the ligands carry mixture
// parameters), or grid maps only.
static int eval_mode(const dock_pocket_t* pockets, int n_pockets, dock_ligands_t L) {
  if (pockets[0]->dev.inter_mode == DOCK_INTER_DIRECT) return kModeDirect;
  if (L->d_mdn)
    for (int i = 0; i < n_pockets; ++i)
      if (pockets[i]->dev.mdn_res > 0 && pockets[i]->dev.mdn_w != 0.f) return kModeGridMdn;
  return kModeGrid;
}

int dock_score_grad(const dock_pocket_t* pockets, int32_t n_pockets, dock_ligands_t L, int64_t n_poses,
                    const int32_t* pose_lig, const float* q, int32_t q_stride, float* E, float* dEdq,
                    float* xyz_out, int32_t xyz_stride, void* stream) try {
  if (!L) return fail(DOCK_E_ARG, "null ligands");
  int rc = check_pockets(pockets, n_pockets, L);
  if (rc) return rc;
  if (n_poses < 0) return fail(DOCK_E_ARG, "negative n_poses");
  if (n_poses == 0) return DOCK_OK;
  if (!pose_lig || !q || !E) return fail(DOCK_E_ARG, "null pose array");
  if (q_stride < 6 + L->max_tors) return fail(DOCK_E_ARG, "q_stride < 6 + max torsions");
  if (xyz_out && xyz_stride < 3 * L->max_atoms) return fail(DOCK_E_ARG, "xyz_stride < 3 * max atoms");
  const PocketDev* tab = nullptr;
  rc = pocket_table(pockets, n_pockets, &tab);
  if (rc) return rc;
  const LaneCfg wc = wide_cfg(L);
  const int lpp = wc.lpp, apl = wc.apl;
  if (score_lds_bytes(lpp, apl, L->max_alt_pairs) > 64 * 1024)
    return fail(DOCK_E_LIMIT, "pair list too long for the LDS budget");
  ScoreArgs a{};
  a.L = L->arrays();
  a.pockets = tab;
  a.n_ligands = L->n;
  a.n_pockets = n_pockets;
  a.n_poses = n_poses;
  a.pose_lig = pose_lig;
  a.q = q;
  a.q_stride = q_stride;
  a.E = E;
  a.dEdq = dEdq;
  a.xyz = xyz_out;
  a.xyz_stride = xyz_stride;
  a.max_pairs = L->max_alt_pairs;
  HIP_TRY(launch_score(a, lpp, apl, eval_mode(pockets, n_pockets, L),
                       reinterpret_cast<hipStream_t>(stream)));
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

// ================================================================ differentiable form

static int terms_call(const dock_pocket_t* pockets, int32_t n_pockets, dock_ligands_t L, int64_t n_poses,
                      const int32_t* pose_lig, const float* q, int32_t q_stride, const float* xyz,
                      int32_t xyz_stride, const float* const* G, const float* w, float* E,
                      const float* dLdE, float* const* dLdG, float* dLdw, float* dLdq, float* dLdx,
                      int deterministic, void* stream) {
  if (!L) return fail(DOCK_E_ARG, "null ligands");
  int rc = check_pockets(pockets, n_pockets, L);
  if (rc) return rc;
  if (n_pockets > kMaxDiffPockets) return fail(DOCK_E_LIMIT, "more than 16 pockets in one differentiable call");
  const int K = pockets[0]->dev.n_terms;
  for (int i = 1; i < n_pockets; ++i)
    if (pockets[i]->dev.n_terms != K) return fail(DOCK_E_ARG, "pockets of one call must share a preset");
  if (n_poses < 0) return fail(DOCK_E_ARG, "negative n_poses");
  if (n_poses == 0) return DOCK_OK;
  if (!pose_lig || !w) return fail(DOCK_E_ARG, "null pose_lig or weights");
  if ((q == nullptr) == (xyz == nullptr)) return fail(DOCK_E_ARG, "give exactly one of q and xyz");
  if (q && q_stride < 6 + L->max_tors) return fail(DOCK_E_ARG, "q_stride < 6 + max torsions");
  if ((xyz || dLdx) && xyz_stride < 3 * L->max_atoms) return fail(DOCK_E_ARG, "xyz_stride < 3 * max atoms");
  if (xyz && dLdq) return fail(DOCK_E_ARG, "dLdq needs poses given as DOFs");
  if (dLdq && q_stride < 6 + L->max_tors) return fail(DOCK_E_ARG, "q_stride < 6 + max torsions");
  const PocketDev* tab = nullptr;
  rc = pocket_table(pockets, n_pockets, &tab);
  if (rc) return rc;
  TermsArgs a{};
  for (int i = 0; i < n_pockets; ++i) {
    if (pockets[i]->dev.inter_mode != DOCK_INTER_GRID)
      return fail(DOCK_E_ARG, "the differentiable form needs grid-mode pockets");
    const float* gi = (G && G[i]) ? G[i] : pockets[i]->d_G;
    if (!gi) return fail(DOCK_E_ARG, "no per-term maps for pocket " + std::to_string(i));
    a.G[i] = gi;
    a.dLdG[i] = dLdG ? dLdG[i] : nullptr;
  }
  const LaneCfg wc = wide_cfg(L);
  const int lpp = wc.lpp, apl = wc.apl;
  if (score_lds_bytes(lpp, apl, L->max_alt_pairs) > 64 * 1024)
    return fail(DOCK_E_LIMIT, "pair list too long for the LDS budget");
  a.L = L->arrays();
  a.pockets = tab;
  a.n_ligands = L->n;
  a.n_pockets = n_pockets;
  a.n_poses = n_poses;
  a.pose_lig = pose_lig;
  a.q = q;
  a.q_stride = q_stride;
  a.xyz = xyz;
  a.xyz_stride = xyz_stride;
  a.w = w;
  a.E = E;
  a.dLdE = dLdE;
  a.dLdw = dLdw;
  a.dLdq = dLdq;
  a.dLdx = dLdx;
  a.max_pairs = L->max_alt_pairs;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (!(dLdE && deterministic)) {
    HIP_TRY(launch_terms(a, lpp, apl, K, s));
    return DOCK_OK;
  }
  // Deterministic adjoint: dL/dG summed as 64-bit integers (fixed point at a
  // per-pocket power-of-two scale from a bound on every node's sum), dL/dw as
  // per-pose contributions reduced in a fixed order.  Scratch is allocated on
  // the stream and released after the last kernel that reads it.
  long long off[kMaxDiffPockets + 1] = {0};
  for (int i = 0; i < n_pockets; ++i) {
    const GridDev& gd = pockets[i]->dev.grid;
    const long long n = a.dLdG[i] ? (long long)kTypes * K * gd.dims[0] * gd.dims[1] * gd.dims[2] : 0;
    off[i + 1] = off[i] + n;
  }
  unsigned long long* acc = nullptr;
  double* scale = nullptr;
  float* w_pose = nullptr;
  int* w_pocket = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&scale), sizeof(double) * kMaxDiffPockets, s);
  if (e == hipSuccess && off[n_pockets] > 0)
    e = hipMallocAsync(reinterpret_cast<void**>(&acc), sizeof(unsigned long long) * off[n_pockets], s);
  if (e == hipSuccess && dLdw) {
    e = hipMallocAsync(reinterpret_cast<void**>(&w_pose), sizeof(float) * size_t(n_poses) * K, s);
    if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&w_pocket), sizeof(int) * size_t(n_poses), s);
  }
  if (e == hipSuccess && acc) e = launch_zero_u64(acc, off[n_pockets], s);
  if (e == hipSuccess) {
    AdjBoundArgs b{};
    b.ligs = L->d_ligs;
    b.n_ligands = L->n;
    b.n_pockets = n_pockets;
    b.K = K;
    b.n_poses = n_poses;
    b.pose_lig = pose_lig;
    b.dLdE = dLdE;
    b.w = w;
    b.scale = scale;
    e = launch_adj_bound(b, s);
  }
  if (e == hipSuccess) {
    for (int i = 0; i < n_pockets; ++i) a.acc[i] = a.dLdG[i] ? acc + off[i] : nullptr;
    a.acc_scale = scale;
    a.w_pose = w_pose;
    a.w_pocket = w_pocket;
    a.dLdw = dLdw;
    e = launch_terms(a, lpp, apl, K, s);
  }
  for (int i = 0; i < n_pockets && e == hipSuccess; ++i)
    if (a.dLdG[i]) e = launch_adj_finalize(acc + off[i], scale + i, off[i + 1] - off[i], a.dLdG[i], s);
  if (e == hipSuccess && dLdw) e = launch_adj_wreduce(w_pose, w_pocket, n_poses, n_pockets, K, dLdw, s);
  for (void* p : {static_cast<void*>(acc), static_cast<void*>(scale), static_cast<void*>(w_pose),
                  static_cast<void*>(w_pocket)})
    if (p) (void)hipFreeAsync(p, s);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? DOCK_E_OOM : DOCK_E_HIP,
                std::string("deterministic adjoint: ") + hipGetErrorString(e));
  return DOCK_OK;
}

int dock_score_terms(const dock_pocket_t* pockets, int32_t n_pockets, dock_ligands_t L, int64_t n_poses,
                     const int32_t* pose_lig, const float* q, int32_t q_stride, const float* xyz,
                     int32_t xyz_stride, const float* const* G, const float* w, float* E, void* stream) try {
  if (!E) return fail(DOCK_E_ARG, "null E");
  return terms_call(pockets, n_pockets, L, n_poses, pose_lig, q, q_stride, xyz, xyz_stride, G, w, E, nullptr,
                    nullptr, nullptr, nullptr, nullptr, 0, stream);
} catch (...) {
  return exception_status();
}

int dock_score_adjoint(const dock_pocket_t* pockets, int32_t n_pockets, dock_ligands_t L, int64_t n_poses,
                       const int32_t* pose_lig, const float* q, int32_t q_stride, const float* xyz,
                       int32_t xyz_stride, const float* const* G, const float* w, const float* dLdE,
                       float* const* dLdG, float* dLdw, float* dLdq, float* dLdx, int32_t deterministic,
                       void* stream) try {
  if (!dLdE) return fail(DOCK_E_ARG, "null dLdE");
  if (deterministic != 0 && deterministic != 1) return fail(DOCK_E_ARG, "deterministic must be 0 or 1");
  return terms_call(pockets, n_pockets, L, n_poses, pose_lig, q, q_stride, xyz, xyz_stride, G, w, nullptr, dLdE,
                    dLdG, dLdw, dLdq, dLdx, deterministic, stream);
} catch (...) {
  return exception_status();
}

// ================================================================ sampling

void dock_sample_params_default(dock_sample_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->n_traj = 64;
  p->n_steps = 100;
  p->n_local = 10;
  p->local_opt = DOCK_LOCAL_ADAM;
  p->lr = 0.1f;
  p->beta1 = 0.9f;
  p->beta2 = 0.999f;
  p->eps = 1e-8f;
  p->mc_beta = 0.069f;
  p->seed = 0;
  p->form = DOCK_FORM_BATCHED;
  p->use_graph = 1;
  p->steps_per_launch = 0;
  p->record_trace = 0;
  p->lanes_per_pose = 0;
  p->rms_alpha = 0.99f;
  p->weight_decay = 0.01f;
}

struct Bucket {
  int lpp = 0, apl = 0, block = 256, max_pairs = 0;
  int alt = 0;                     // ligands use their alternative pair layout
  int per_cu = 0;                  // blocks per CU its ligands' LDS allows
  int item_off = 0, n_items = 0;   // batched: this bucket's items
  int grid = 0;                    // batched: persistent grid
  int part_base = 0;               // batched: offset of its partition bounds in d_part
  std::vector<int> ligs;
};

struct dock_run_s {
  dock_ligands_t L = nullptr;
  std::vector<dock_pocket_t> pockets;  // distinct handles, each counted in its n_runs
  bool holds_refs = false;
  const PocketDev* table = nullptr;
  int mode = kModeGrid;             // kernel mode (eval_mode)
  dock_sample_params p{};
  int n_lig = 0, T = 0, q_stride = 0, step = 0, trace_cap = 0;
  int trace_stride = 1, trace_tt = 0, n_trace = 0;  // logged ligands / trajectories
  float *q_cur = nullptr, *E_cur = nullptr, *q_best = nullptr, *E_best = nullptr, *trace = nullptr;
  int* n_evals = nullptr;
  int* d_step = nullptr;   // device: [0] MC steps taken, [1] seed (read by the kernels, so
                            // graph replays follow dock_run_restart)
  int2* d_items = nullptr;
  int* d_queue = nullptr;
  int n_queue = 0;
  int n_part = 1;                   // batched: item partitions per bucket (one per XCD for
                                    // several pockets), each with its own queue counter
  int* d_part = nullptr;            // per bucket: n_part + 1 item bounds
  std::vector<Bucket> buckets;
  // plain form: per ligand (bucket index, first item, item count)
  std::vector<int> lig_bucket, lig_item_off, lig_n_items;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_steps = -1;
  // per-launch timing of the last call (eager launches only)
  struct Launch {
    dock_launch_stat st;
    hipEvent_t a, b;
  };
  std::vector<Launch> launches;
  std::vector<hipEvent_t> event_pool;
  size_t events_used = 0;
  bool recording = false;
  // batched form: the buckets run in groups, one per occupancy class (blocks
  // per CU) of the buckets that fill the chip, highest first; buckets too
  // small to fill it join the first group.  The buckets of a group run
  // concurrently: the first on the caller's stream, the k-th on side[k - 1],
  // forked from and joined back into the caller's stream, so a bucket too
  // small to fill the chip and the tail of a large one overlap.  A group
  // starts when the one before it has ended: blocks of kernels of different
  // occupancy classes sharing a CU lower the waves it holds.  The side
  // streams belong to the device's process-wide pool (side_streams).
  std::vector<std::vector<int>> occ_groups;
  std::vector<hipStream_t> side;
  std::vector<std::vector<hipEvent_t>> join;  // [group][side stream]
  std::vector<hipEvent_t> fork;               // [group]
};

// Side streams of the batched form, shared by every run on a device and kept
// until the process ends.  The runtime hands each new stream a hardware
// queue; streams created and destroyed with each run were at times handed the
// queue of the caller's stream (or of another side stream), and the buckets
// on it then ran one after the other.  Created once, the pool's streams keep
// their queues.  Runs enqueued from several host threads at once share these
// streams: eager launches stay ordered by the fork and join events, but
// capturing graphs from several threads at once is not supported.
static int side_streams(size_t n, std::vector<hipStream_t>* out) {
  static std::mutex mu;
  static std::map<int, std::vector<hipStream_t>> pool;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(DOCK_E_HIP, std::string("bucket streams: ") + hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(mu);
  std::vector<hipStream_t>& v = pool[dev];
  while (v.size() < n) {
    hipStream_t q = nullptr;
    e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(DOCK_E_HIP, std::string("bucket streams: ") + hipGetErrorString(e));
    v.push_back(q);
  }
  out->assign(v.begin(), v.begin() + n);
  return DOCK_OK;
}

static hipEvent_t pool_event(dock_run_s* r) {
  if (r->events_used == r->event_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    r->event_pool.push_back(e);
  }
  return r->event_pool[r->events_used++];
}

// Launch one sampler grid, bracketed by events when recording.
static hipError_t timed_launch(dock_run_s* r, const SampleArgs& a, int bucket, int lpp, int apl, int grid,
                               int block, hipStream_t s) {
  hipEvent_t ea = nullptr, eb = nullptr;
  if (r->recording) {
    ea = pool_event(r);
    eb = pool_event(r);
    if (ea) (void)hipEventRecord(ea, s);
  }
  hipError_t e = launch_sample(a, lpp, apl, grid, block, r->mode, s);
  if (r->recording && ea && eb) {
    (void)hipEventRecord(eb, s);
    dock_run_s::Launch L;
    L.st.bucket = bucket;
    L.st.lanes_per_pose = lpp;
    L.st.atoms_per_lane = apl;
    L.st.block = block;
    L.st.grid = grid;
    L.st.n_items = a.n_items;
    L.st.init = a.init;
    L.st.step_count = a.step_count;
    L.st.ms = -1.f;
    L.a = ea;
    L.b = eb;
    r->launches.push_back(L);
  }
  return e;
}

static void free_run(dock_run_s* r) {
  if (r->holds_refs) {
    for (dock_pocket_t p : r->pockets) p->n_runs.fetch_sub(1);
    r->L->n_runs.fetch_sub(1);
  }
  for (hipEvent_t e : r->event_pool) (void)hipEventDestroy(e);
  for (const auto& jg : r->join)
    for (hipEvent_t e : jg) (void)hipEventDestroy(e);
  for (hipEvent_t e : r->fork)
    if (e) (void)hipEventDestroy(e);
  if (r->gexec) (void)hipGraphExecDestroy(r->gexec);
  if (r->graph) (void)hipGraphDestroy(r->graph);
  if (r->ev0) (void)hipEventDestroy(r->ev0);
  if (r->ev1) (void)hipEventDestroy(r->ev1);
  dev_free(r->q_cur);
  dev_free(r->E_cur);
  dev_free(r->q_best);
  dev_free(r->E_best);
  dev_free(r->trace);
  dev_free(r->n_evals);
  dev_free(r->d_step);
  dev_free(r->d_items);
  dev_free(r->d_queue);
  dev_free(r->d_part);
  delete r;
}

static SampleArgs base_args(const dock_run_s* r) {
  SampleArgs a{};
  a.L = r->L->arrays();
  a.pockets = r->table;
  a.step_base = r->d_step;
  a.n_traj = r->T;
  a.q_stride = r->q_stride;
  a.n_local = r->p.n_local;
  a.local_opt = r->p.local_opt;
  a.lr = r->p.lr;
  a.b1 = r->p.beta1;
  a.b2 = r->p.beta2;
  a.eps = r->p.eps;
  a.mc_beta = r->p.mc_beta;
  a.rms_alpha = r->p.rms_alpha;
  a.weight_decay = r->p.weight_decay;
  a.q_cur = r->q_cur;
  a.E_cur = r->E_cur;
  a.q_best = r->q_best;
  a.E_best = r->E_best;
  a.n_evals = r->n_evals;
  a.trace = r->trace;
  a.trace_cap = r->trace_cap;
  a.trace_stride = r->trace_stride;
  a.trace_traj = r->trace_tt;
  return a;
}

// Enqueue the launches of one phase: init (steps = 0) or `steps` MC steps.
static hipError_t enqueue_phase(dock_run_s* r, bool init, int steps, hipStream_t s) {
  const int chunk = (init || r->p.steps_per_launch <= 0) ? std::max(steps, 1)
                                                          : r->p.steps_per_launch;
  const int n_chunks = init ? 1 : (steps + chunk - 1) / chunk;
  hipError_t e = hipSuccess;
  const int nb = int(r->buckets.size()), np = r->n_part;
  auto chunk_args = [&](int c) {
    SampleArgs a = base_args(r);
    a.init = init ? 1 : 0;
    a.step_off = init ? 0 : c * chunk;
    a.step_count = init ? 0 : std::min(chunk, steps - c * chunk);
    return a;
  };
  if (r->p.form == DOCK_FORM_BATCHED) {
    const int need = n_chunks * nb * np;
    if (need > r->n_queue) return hipErrorInvalidValue;
    e = launch_fill_int(r->d_queue, need, 0, s);
    if (e != hipSuccess) return e;
    // occupancy classes one after the other; within one, the buckets run
    // concurrently, each through all of its chunks on its own stream
    for (size_t gi = 0; gi < r->occ_groups.size(); ++gi) {
      const std::vector<int>& P = r->occ_groups[gi];
      if (P.size() > 1) {
        if ((e = hipEventRecord(r->fork[gi], s)) != hipSuccess) return e;
        for (size_t k = 1; k < P.size(); ++k)
          if ((e = hipStreamWaitEvent(r->side[k - 1], r->fork[gi], 0)) != hipSuccess) return e;
      }
      for (int c = 0; c < n_chunks; ++c) {
        SampleArgs a = chunk_args(c);
        for (size_t k = 0; k < P.size(); ++k) {
          const int b = P[k];
          const Bucket& B = r->buckets[b];
          a.items = r->d_items + B.item_off;
          a.n_items = B.n_items;
          a.queue = r->d_queue + (c * nb + b) * np;
          a.part_off = r->d_part + B.part_base;
          a.n_part = np;
          a.max_pairs = B.max_pairs;
          e = timed_launch(r, a, b, B.lpp, B.apl, B.grid, B.block, k == 0 ? s : r->side[k - 1]);
          if (e != hipSuccess) return e;
        }
      }
      if (P.size() > 1)
        for (size_t k = 1; k < P.size(); ++k) {
          if ((e = hipEventRecord(r->join[gi][k - 1], r->side[k - 1])) != hipSuccess) return e;
          if ((e = hipStreamWaitEvent(s, r->join[gi][k - 1], 0)) != hipSuccess) return e;
        }
    }
  } else {
    for (int c = 0; c < n_chunks; ++c) {
      SampleArgs a = chunk_args(c);
      for (int l = 0; l < r->n_lig; ++l) {
        const Bucket& B = r->buckets[r->lig_bucket[l]];
        a.items = r->d_items + r->lig_item_off[l];
        a.n_items = r->lig_n_items[l];
        a.queue = nullptr;
        a.part_off = nullptr;
        a.n_part = 1;
        a.max_pairs = B.alt ? r->L->h_ligs[l].alt.n_stage : r->L->h_ligs[l].n_stage;
        e = timed_launch(r, a, r->lig_bucket[l], B.lpp, B.apl, r->lig_n_items[l], B.block, s);
        if (e != hipSuccess) return e;
      }
    }
  }
  if (!init) e = launch_add_int(r->d_step, steps, s);
  return e;
}

static int run_phase(dock_run_s* r, bool init, int steps, hipStream_t s) {
  if (!init && steps == 0) return DOCK_OK;
  if (!init && r->p.use_graph && r->p.form == DOCK_FORM_BATCHED) {
    if (r->graph_steps != steps) {
      if (r->gexec) (void)hipGraphExecDestroy(r->gexec);
      if (r->graph) (void)hipGraphDestroy(r->graph);
      r->gexec = nullptr;
      r->graph = nullptr;
      r->graph_steps = -1;
      hipStream_t cs = nullptr;
      HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        const bool rec = r->recording;
        r->recording = false;
        hipError_t e2 = enqueue_phase(r, false, steps, cs);
        r->recording = rec;
        e = hipStreamEndCapture(cs, &r->graph);
        if (e2 != hipSuccess) e = e2;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&r->gexec, r->graph, nullptr, nullptr, 0);
      (void)hipStreamDestroy(cs);
      if (e != hipSuccess) return fail(DOCK_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
      r->graph_steps = steps;
    }
    HIP_TRY(hipGraphLaunch(r->gexec, s));
  } else {
    HIP_TRY(enqueue_phase(r, init, steps, s));
  }
  if (!init) r->step += steps;
  return DOCK_OK;
}

// Runs phases between the run's two timing events.
static int timed_phases(dock_run_s* r, bool init, int steps, hipStream_t s) {
  r->launches.clear();
  r->events_used = 0;
  r->recording = true;
  HIP_TRY(hipEventRecord(r->ev0, s));
  int rc = DOCK_OK;
  if (init) rc = run_phase(r, true, 0, s);
  if (rc == DOCK_OK) rc = run_phase(r, false, steps, s);
  if (rc != DOCK_OK) return rc;
  HIP_TRY(hipEventRecord(r->ev1, s));
  r->timed = true;
  return DOCK_OK;
}

static int check_params(const dock_sample_params* p) {
  if (!p) return fail(DOCK_E_ARG, "null params");
  if (p->n_traj < 1 || p->n_steps < 0 || p->n_local < 0) return fail(DOCK_E_ARG, "bad counts");
  if (p->local_opt < DOCK_LOCAL_ADAM || p->local_opt > DOCK_LOCAL_ADAMW)
    return fail(DOCK_E_ARG, "unknown local_opt");
  if (p->form != DOCK_FORM_PLAIN && p->form != DOCK_FORM_BATCHED) return fail(DOCK_E_ARG, "unknown form");
  if (p->lanes_per_pose != 0 && p->lanes_per_pose != 16 && p->lanes_per_pose != 32 && p->lanes_per_pose != 64)
    return fail(DOCK_E_ARG, "lanes_per_pose must be 0, 16, 32 or 64");
  if (!(std::isfinite(p->lr) && std::isfinite(p->beta1) && std::isfinite(p->beta2) &&
        std::isfinite(p->eps) && std::isfinite(p->mc_beta) && std::isfinite(p->rms_alpha) &&
        std::isfinite(p->weight_decay)))
    return fail(DOCK_E_ARG, "non-finite sampler constant");
  if (p->steps_per_launch < 0) return fail(DOCK_E_ARG, "negative steps_per_launch");
  if (p->trace_lig_stride < 0 || p->trace_traj < 0) return fail(DOCK_E_ARG, "negative trace selection");
  return DOCK_OK;
}

// Plan overrides used by the autotuner: a forced (lpp, block) for one natural
// lane configuration, and the subset of ligands that get work items.
struct PlanOverride {
  int nat_lpp = 0, nat_apl = 0, lpp = 0, block = 0;
  const std::vector<char>* subset = nullptr;
  int one_per_lane = -1;  // >= 0: the full run's layout decision (trials on a subset)
};

// The layout decision of create_run: ligands of 33-64 atoms go two atoms per
// lane when their trajectories fill at least two waves per wave slot of the
// device with two poses per wavefront.
static bool run_one_per_lane(const dock_ligands_s* L, int T, int n_cu, const std::vector<char>* subset) {
  long long mid_traj = 0;
  for (int l = 0; l < L->n; ++l) {
    if (subset && !(*subset)[l]) continue;
    const LigDev& g = L->h_ligs[l];
    if (g.n_atoms <= 64 && lane_cfg(g, 0).apl == 2) mid_traj += T;
  }
  return mid_traj / 2 < 2LL * kWavesPerCu * n_cu;
}

static int device_cu_count() {
  int dev = 0, n_cu = 256;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) n_cu = 256;
  return n_cu;
}

static int create_run(const dock_pocket_t* pockets, int32_t n_pockets, dock_ligands_t L,
                      const dock_sample_params* p, void* stream, dock_run_t* out, const PlanOverride* ov) {
  if (!L || !out) return fail(DOCK_E_ARG, "null argument");
  int rc = check_pockets(pockets, n_pockets, L);
  if (rc) return rc;
  rc = check_params(p);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  dock_run_s* r = new (std::nothrow) dock_run_s;
  if (!r) return fail(DOCK_E_OOM, "host allocation");
  r->L = L;
  r->pockets.assign(pockets, pockets + n_pockets);
  std::sort(r->pockets.begin(), r->pockets.end());
  r->pockets.erase(std::unique(r->pockets.begin(), r->pockets.end()), r->pockets.end());
  // the run reads the pockets' tables and the ligands' arrays until it is
  // freed: dock_free_pocket / dock_free_ligands refuse while it lives
  for (dock_pocket_t pk : r->pockets) pk->n_runs.fetch_add(1);
  L->n_runs.fetch_add(1);
  r->holds_refs = true;
  r->mode = eval_mode(pockets, n_pockets, L);
  r->p = *p;
  r->n_lig = L->n;
  r->T = p->n_traj;
  r->q_stride = 6 + L->max_tors;
  r->stream = s;
  auto bail = [&](int code, const std::string& m) {
    free_run(r);
    return fail(code, m);
  };
  rc = pocket_table(pockets, n_pockets, &r->table);
  if (rc) {
    std::string m = g_err;
    free_run(r);
    return fail(rc, m);
  }
  // ---- plan: lane configuration per ligand, buckets, work items
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int n_cu = device_cu_count();
  int n_xcc = 8;
  if (hipDeviceGetAttribute(&n_xcc, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || n_xcc < 1) n_xcc = 1;
  // several pockets: the items of each bucket are split into one partition
  // per XCD (pocket p -> partition p mod n_xcc), which blocks on that XCD
  // (block b runs on XCD b mod n_xcc) take first, so that an XCD's L2 holds
  // the maps of a few pockets instead of all of them; a block whose
  // partition is empty takes from the others in turn
  r->n_part = (p->form == DOCK_FORM_BATCHED && n_pockets > 1) ? std::min(n_xcc, 64) : 1;
  std::map<std::tuple<int, int, int, int>, int> bidx;
  std::map<std::tuple<int, int, int, int>, int> occ;  // (lpp, apl, block, LDS / 256) -> blocks per CU
  r->lig_bucket.resize(r->n_lig);
  const std::string arch = device_arch();
  // Two atoms per lane (ligands of 33-64 atoms) pays when the run fills the
  // chip many times over; a smaller run keeps one atom per lane, which gives
  // it twice the wavefronts.  The choice depends on the ligand set and the
  // trajectory count only, so every form of the run evaluates alike.
  const bool one_per_lane = (ov && ov->one_per_lane >= 0) ? ov->one_per_lane != 0
                                                            : run_one_per_lane(L, r->T, n_cu, ov ? ov->subset : nullptr);
  for (int l = 0; l < r->n_lig; ++l) {
    LaneCfg c = lane_cfg(L->h_ligs[l], p->lanes_per_pose, one_per_lane);
    int block = 256;
    if (ov && ov->lpp) {
      if (c.lpp == ov->nat_lpp && c.apl == ov->nat_apl) {
        c.lpp = ov->lpp;
        block = ov->block;
      }
    } else if (p->lanes_per_pose == 0) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto t = g_tune.find(std::make_tuple(arch, c.lpp, c.apl));
      if (t != g_tune.end()) {
        c.lpp = t->second.lpp;
        block = t->second.block;
      }
    }
    // ligands whose staged pair records lower the blocks per CU go to a
    // bucket of their own, so that one large ligand does not lower the
    // occupancy of every launch of its lane configuration
    const LigDev& gl0 = L->h_ligs[l];
    const int stage = c.apl == 1 ? gl0.alt.n_stage : gl0.n_stage;
    const size_t lds_l = sample_lds_bytes(c.lpp, c.apl, block, stage);
    int per_cu = 0;
    if (p->form == DOCK_FORM_BATCHED && lds_l <= 64 * 1024) {
      const auto ok = std::make_tuple(c.lpp, c.apl, block, int((lds_l + 255) / 256));
      auto oi = occ.find(ok);
      if (oi == occ.end())
        oi = occ.emplace(ok, sample_max_blocks_per_cu(c.lpp, c.apl, block, r->mode, (lds_l + 255) / 256 * 256)).first;
      per_cu = oi->second;
    }
    auto key = std::make_tuple(c.lpp, c.apl, block, per_cu);
    auto it = bidx.find(key);
    if (it == bidx.end()) {
      Bucket B;
      B.lpp = c.lpp;
      B.apl = c.apl;
      B.block = block;
      B.per_cu = per_cu;
      // the kernels with one atom per lane read the alternative layout (the
      // primary one for every ligand not laid out with two atoms per lane)
      B.alt = c.apl == 1 ? 1 : 0;
      it = bidx.emplace(key, int(r->buckets.size())).first;
      r->buckets.push_back(B);
    }
    Bucket& B = r->buckets[it->second];
    B.ligs.push_back(l);
    const LigDev& gl = L->h_ligs[l];
    B.max_pairs = std::max(B.max_pairs, B.alt ? gl.alt.n_stage : gl.n_stage);
    r->lig_bucket[l] = it->second;
  }
  std::vector<int2> items;
  std::vector<int> part_bounds;  // batched: per bucket n_part + 1 bounds, relative to its items
  r->lig_item_off.assign(r->n_lig, 0);
  r->lig_n_items.assign(r->n_lig, 0);
  if (p->form == DOCK_FORM_PLAIN) {
    for (int l = 0; l < r->n_lig; ++l) {
      const Bucket& B = r->buckets[r->lig_bucket[l]];
      const int gpb = B.block / B.lpp;
      r->lig_item_off[l] = int(items.size());
      if (!(ov && ov->subset && !(*ov->subset)[l]))
        for (int t0 = 0; t0 < r->T; t0 += gpb) items.push_back(make_int2(l, t0));
      r->lig_n_items[l] = int(items.size()) - r->lig_item_off[l];
    }
  } else {
    const int np = r->n_part;
    for (Bucket& B : r->buckets) {
      const int gpb = B.block / B.lpp;
      // per partition (pocket mod np), the ligands of one pocket together
      // and, within a pocket, longest work first: cost ~ pair slots (empty
      // ones included) + 4 * atoms per evaluation
      std::vector<int> ligs = B.ligs;
      const auto cost = [&](int l) {
        const LigDev& g = L->h_ligs[l];
        const int n_pass = B.alt ? g.alt.n_pass : g.n_pass, n_prec = B.alt ? g.alt.n_prec : g.n_prec;
        return (n_pass > 0 ? n_prec : g.n_pairs) + 4 * g.n_atoms;
      };
      const auto order = [&](int l) {
        const int pk = L->h_ligs[l].pocket;
        return std::make_tuple(np > 1 ? pk % np : 0, np > 1 ? pk : 0, -cost(l));
      };
      std::stable_sort(ligs.begin(), ligs.end(), [&](int x, int y) { return order(x) < order(y); });
      B.item_off = int(items.size());
      B.part_base = int(part_bounds.size());
      int cur = 0;
      part_bounds.push_back(0);
      for (int l : ligs) {
        if (ov && ov->subset && !(*ov->subset)[l]) continue;
        const int q = np > 1 ? L->h_ligs[l].pocket % np : 0;
        while (cur < q) {
          part_bounds.push_back(int(items.size()) - B.item_off);
          ++cur;
        }
        for (int t0 = 0; t0 < r->T; t0 += gpb) items.push_back(make_int2(l, t0));
      }
      while (cur < np) {
        part_bounds.push_back(int(items.size()) - B.item_off);
        ++cur;
      }
      B.n_items = int(items.size()) - B.item_off;
      const size_t lds = sample_lds_bytes(B.lpp, B.apl, B.block, B.max_pairs);
      if (lds > 64 * 1024) return bail(DOCK_E_LIMIT, "pair list too long for the LDS budget");
      const int per_cu = sample_max_blocks_per_cu(B.lpp, B.apl, B.block, r->mode, lds);
      B.grid = std::min(B.n_items, per_cu * n_cu);
      B.per_cu = per_cu;
    }
    // launch groups: one per occupancy class of the buckets whose grid fills
    // the chip, highest first; a bucket too small to fill the chip joins the
    // first group (it gains from overlapping and displaces little)
    auto fills = [&](const Bucket& B) { return B.grid >= B.per_cu * n_cu; };
    int top = 0;
    for (const Bucket& B : r->buckets)
      if (fills(B)) top = std::max(top, B.per_cu);
    auto rank = [&](int b) { return fills(r->buckets[b]) ? r->buckets[b].per_cu : top; };
    std::vector<int> order(r->buckets.size());
    for (size_t b = 0; b < order.size(); ++b) order[b] = int(b);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return rank(x) > rank(y); });
    for (const int b : order) {
      if (r->occ_groups.empty() || rank(r->occ_groups.back()[0]) != rank(b)) r->occ_groups.emplace_back();
      r->occ_groups.back().push_back(b);
    }
  }
  for (const Bucket& B : r->buckets)
    if (sample_lds_bytes(B.lpp, B.apl, B.block, B.max_pairs) > 64 * 1024)
      return bail(DOCK_E_LIMIT, "pair list too long for the LDS budget");
  size_t widest = 0;
  for (const auto& P : r->occ_groups) widest = std::max(widest, P.size());
  if (p->form == DOCK_FORM_BATCHED && widest > 1) {
    if (side_streams(widest - 1, &r->side) != DOCK_OK) {
      const std::string m = g_err;
      return bail(DOCK_E_HIP, m);
    }
    hipError_t se = hipSuccess;
    r->fork.assign(r->occ_groups.size(), nullptr);
    r->join.resize(r->occ_groups.size());
    for (size_t gi = 0; gi < r->occ_groups.size() && se == hipSuccess; ++gi) {
      if (r->occ_groups[gi].size() < 2) continue;
      se = hipEventCreateWithFlags(&r->fork[gi], hipEventDisableTiming);
      for (size_t k = 1; k < r->occ_groups[gi].size() && se == hipSuccess; ++k) {
        hipEvent_t j = nullptr;
        se = hipEventCreateWithFlags(&j, hipEventDisableTiming);
        if (se == hipSuccess) r->join[gi].push_back(j);
      }
    }
    if (se != hipSuccess) return bail(DOCK_E_HIP, std::string("bucket events: ") + hipGetErrorString(se));
  }
  // ---- buffers
  const size_t nt = size_t(r->n_lig) * r->T;
  const int chunk = p->steps_per_launch > 0 ? p->steps_per_launch : std::max(1, p->n_steps);
  r->n_queue = int(r->buckets.size()) * std::max(1, (p->n_steps + chunk - 1) / chunk) * r->n_part;
  hipError_t e = dev_alloc(&r->q_cur, nt * r->q_stride);
  if (e == hipSuccess) e = dev_alloc(&r->q_best, nt * r->q_stride);
  if (e == hipSuccess) e = dev_alloc(&r->E_cur, nt);
  if (e == hipSuccess) e = dev_alloc(&r->E_best, nt);
  if (e == hipSuccess) e = dev_alloc(&r->n_evals, nt);
  if (e == hipSuccess) e = dev_alloc(&r->d_step, 2);
  if (e == hipSuccess) e = dev_alloc(&r->d_items, items.size());
  if (e == hipSuccess) e = dev_alloc(&r->d_queue, size_t(std::max(1, r->n_queue)));
  if (e == hipSuccess) e = dev_alloc(&r->d_part, std::max<size_t>(1, part_bounds.size()));
  if (e == hipSuccess && p->record_trace) {
    const int per_step = p->local_opt == DOCK_LOCAL_LINESEARCH ? 1 + 11 * p->n_local : p->n_local + 1;
    r->trace_cap = 1 + p->n_steps * per_step;
    r->trace_stride = std::max(1, p->trace_lig_stride);
    r->trace_tt = p->trace_traj > 0 ? std::min(p->trace_traj, r->T) : r->T;
    r->n_trace = ((r->n_lig + r->trace_stride - 1) / r->trace_stride) * r->trace_tt;
    e = dev_alloc(&r->trace, size_t(r->n_trace) * size_t(r->trace_cap) * (2 * r->q_stride + 1));
  }
  if (e != hipSuccess) return bail(DOCK_E_OOM, std::string("run allocation: ") + hipGetErrorString(e));
  // the kernels write the n_dof leading slots of every pose row; the padding
  // slots up to q_stride read back as zeros
  e = hipMemsetAsync(r->q_cur, 0, sizeof(float) * nt * r->q_stride, s);
  if (e == hipSuccess) e = hipMemsetAsync(r->q_best, 0, sizeof(float) * nt * r->q_stride, s);
  if (e != hipSuccess) return bail(DOCK_E_HIP, std::string("run state clear: ") + hipGetErrorString(e));
  e = hipMemcpy(r->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !part_bounds.empty())
    e = hipMemcpy(r->d_part, part_bounds.data(), sizeof(int) * part_bounds.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bail(DOCK_E_HIP, std::string("item upload: ") + hipGetErrorString(e));
  if ((e = hipEventCreate(&r->ev0)) != hipSuccess || (e = hipEventCreate(&r->ev1)) != hipSuccess)
    return bail(DOCK_E_HIP, std::string("event: ") + hipGetErrorString(e));
  e = launch_fill_int(r->n_evals, int(nt), 0, s);
  if (e == hipSuccess) e = launch_fill_int(r->d_step, 1, 0, s);
  if (e == hipSuccess) e = launch_fill_int(r->d_step + 1, 1, int(p->seed), s);
  if (e == hipSuccess && r->trace) {
    // trace rows default to NaN
    e = hipMemsetAsync(r->trace, 0xff,
                       size_t(r->n_trace) * size_t(r->trace_cap) * (2 * r->q_stride + 1) * sizeof(float), s);
  }
  if (e != hipSuccess) return bail(DOCK_E_HIP, std::string("init: ") + hipGetErrorString(e));
  rc = timed_phases(r, true, p->n_steps, s);
  if (rc != DOCK_OK) {
    std::string m = g_err;
    free_run(r);
    return fail(rc, m);
  }
  *out = r;
  return DOCK_OK;
}

int dock_sample(const dock_pocket_t* pockets, int32_t n_pockets, dock_ligands_t L,
                const dock_sample_params* p, void* stream, dock_run_t* out) try {
  return create_run(pockets, n_pockets, L, p, stream, out, nullptr);
} catch (...) {
  return exception_status();
}

int dock_autotune(const dock_pocket_t* pockets, int32_t n_pockets, dock_ligands_t L,
                  const dock_sample_params* p, int32_t trial_steps, void* stream) try {
  if (!L || !p) return fail(DOCK_E_ARG, "null argument");
  if (trial_steps < 1) return fail(DOCK_E_ARG, "trial_steps must be >= 1");
  int rc = check_pockets(pockets, n_pockets, L);
  if (rc) return rc;
  rc = check_params(p);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // natural lane configurations present in L, with the layout decision a
  // run of all of L makes (the trials, on subsets, are held to it)
  const bool opl = run_one_per_lane(L, p->n_traj, device_cu_count(), nullptr);
  std::map<std::pair<int, int>, std::vector<char>> nat;
  for (int l = 0; l < L->n; ++l) {
    const LaneCfg c = lane_cfg(L->h_ligs[l], 0, opl);
    auto& m = nat[std::make_pair(c.lpp, c.apl)];
    if (m.empty()) m.assign(L->n, 0);
    m[l] = 1;
  }
  dock_sample_params q = *p;
  q.n_steps = 0;
  q.form = DOCK_FORM_BATCHED;
  q.use_graph = 0;
  q.steps_per_launch = 0;
  q.record_trace = 0;
  q.lanes_per_pose = 0;
  const std::string arch = device_arch();
  for (auto& kv : nat) {
    const int lpp0 = kv.first.first, apl = kv.first.second;
    std::vector<int> widths{lpp0};
    if (apl == 1 && lpp0 < 64) widths.push_back(lpp0 * 2);
    TuneChoice best{lpp0, 256, 1e30f};
    for (int lpp : widths)
      for (int block : {64, 128, 256}) {
        if (block < lpp) continue;
        PlanOverride ov;
        ov.nat_lpp = lpp0;
        ov.nat_apl = apl;
        ov.lpp = lpp;
        ov.block = block;
        ov.subset = &kv.second;
        ov.one_per_lane = opl ? 1 : 0;
        dock_run_t run = nullptr;
        rc = create_run(pockets, n_pockets, L, &q, stream, &run, &ov);
        if (rc) return rc;
        rc = dock_run_advance(run, trial_steps, stream);
        float ms = 0.f;
        if (rc == DOCK_OK) rc = dock_run_kernel_ms(run, &ms);
        dock_free_run(run);
        if (rc) return rc;
        if (ms < best.ms) best = TuneChoice{lpp, block, ms};
      }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[std::make_tuple(arch, lpp0, apl)] = best;
  }
  HIP_TRY(hipStreamSynchronize(s));
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_autotune_report(char* buf, int32_t cap, int32_t* needed) try {
  std::string out = "[";
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    bool firstv = true;
    for (auto& kv : g_tune) {
      if (!firstv) out += ", ";
      firstv = false;
      char line[256];
      std::snprintf(line, sizeof line,
                    "{\"arch\": \"%s\", \"lanes\": %d, \"atoms_per_lane\": %d, \"chosen_lanes\": %d, "
                    "\"block\": %d, \"trial_ms\": %.4f}",
                    std::get<0>(kv.first).c_str(), std::get<1>(kv.first), std::get<2>(kv.first),
                    kv.second.lpp, kv.second.block, kv.second.ms);
      out += line;
    }
  }
  out += "]";
  if (needed) *needed = int32_t(out.size() + 1);
  if (buf && cap > 0) {
    std::strncpy(buf, out.c_str(), size_t(cap) - 1);
    buf[cap - 1] = 0;
  }
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_autotune_set(const char* arch, int32_t lanes, int32_t atoms_per_lane, int32_t chosen_lanes,
                      int32_t block, float trial_ms) try {
  if (!arch || !*arch) return fail(DOCK_E_ARG, "empty architecture name");
  const bool lanes_ok = lanes == 16 || lanes == 32 || lanes == 64;
  if (!lanes_ok || (atoms_per_lane != 1 && atoms_per_lane != 2))
    return fail(DOCK_E_ARG, "lanes must be 16, 32 or 64 and atoms_per_lane 1 or 2");
  if (chosen_lanes != lanes && !(atoms_per_lane == 1 && chosen_lanes == 2 * lanes && chosen_lanes <= 64))
    return fail(DOCK_E_ARG, "chosen_lanes must be the natural width or, with one atom per lane, twice it");
  if ((block != 64 && block != 128 && block != 256) || block < chosen_lanes)
    return fail(DOCK_E_ARG, "block must be 64, 128 or 256 and hold one group");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[std::make_tuple(std::string(arch), int(lanes), int(atoms_per_lane))] =
      TuneChoice{chosen_lanes, block, std::isfinite(trial_ms) ? trial_ms : 0.f};
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_autotune_clear(void) try {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_run_advance(dock_run_t r, int32_t n_steps, void* stream) try {
  if (!r) return fail(DOCK_E_ARG, "null run");
  if (n_steps < 0) return fail(DOCK_E_ARG, "negative n_steps");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int chunk = r->p.steps_per_launch > 0 ? r->p.steps_per_launch : std::max(1, n_steps);
  const int need = int(r->buckets.size()) * std::max(1, (n_steps + chunk - 1) / chunk) * r->n_part;
  if (need > r->n_queue) {
    dev_free(r->d_queue);
    r->n_queue = 0;
    HIP_TRY(dev_alloc(&r->d_queue, size_t(need)));
    r->n_queue = need;
    if (r->gexec) (void)hipGraphExecDestroy(r->gexec);
    if (r->graph) (void)hipGraphDestroy(r->graph);
    r->gexec = nullptr;
    r->graph = nullptr;
    r->graph_steps = -1;
  }
  return timed_phases(r, false, n_steps, s);
} catch (...) {
  return exception_status();
}

int dock_run_restart(dock_run_t r, uint32_t seed, void* stream) try {
  if (!r) return fail(DOCK_E_ARG, "null run");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t nt = size_t(r->n_lig) * r->T;
  // counters and the trace back to their initial values with fill kernels
  // rather than memsets (the call enqueues kernels only and allocates
  // nothing)
  HIP_TRY(launch_fill_int(r->n_evals, int(nt), 0, s));
  HIP_TRY(launch_fill_int(r->d_step, 1, 0, s));
  HIP_TRY(launch_fill_int(r->d_step + 1, 1, int(seed), s));
  if (r->trace)
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(r->trace),
                            (long long)r->n_trace * r->trace_cap * (2 * r->q_stride + 1), 0xffffffffu, s));
  r->p.seed = seed;
  r->step = 0;
  return timed_phases(r, true, r->p.n_steps, s);
} catch (...) {
  return exception_status();
}

int dock_run_view_get(dock_run_t r, dock_run_view* v) try {
  if (!r || !v) return fail(DOCK_E_ARG, "null argument");
  v->n_ligands = r->n_lig;
  v->n_traj = r->T;
  v->q_stride = r->q_stride;
  v->step = r->step;
  v->q_cur = r->q_cur;
  v->E_cur = r->E_cur;
  v->q_best = r->q_best;
  v->E_best = r->E_best;
  v->n_evals = r->n_evals;
  v->trace = r->trace;
  v->trace_cap = r->trace_cap;
  v->trace_lig_stride = r->trace_stride;
  v->trace_traj = r->trace_tt;
  v->n_trace = r->n_trace;
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_run_copy_state(dock_run_t r, float* q_cur, float* E_cur, float* q_best, float* E_best,
                        int32_t* n_evals, float* trace, void* stream) try {
  if (!r) return fail(DOCK_E_ARG, "null run");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t nt = size_t(r->n_lig) * r->T;
  const auto D2D = hipMemcpyDeviceToDevice;
  if (q_cur) HIP_TRY(hipMemcpyAsync(q_cur, r->q_cur, nt * r->q_stride * sizeof(float), D2D, s));
  if (q_best) HIP_TRY(hipMemcpyAsync(q_best, r->q_best, nt * r->q_stride * sizeof(float), D2D, s));
  if (E_cur) HIP_TRY(hipMemcpyAsync(E_cur, r->E_cur, nt * sizeof(float), D2D, s));
  if (E_best) HIP_TRY(hipMemcpyAsync(E_best, r->E_best, nt * sizeof(float), D2D, s));
  if (n_evals) HIP_TRY(hipMemcpyAsync(n_evals, r->n_evals, nt * sizeof(int), D2D, s));
  if (trace) {
    if (!r->trace) return fail(DOCK_E_ARG, "run has no trace");
    HIP_TRY(hipMemcpyAsync(trace, r->trace, size_t(r->n_trace) * size_t(r->trace_cap) * (2 * r->q_stride + 1) * sizeof(float),
                           D2D, s));
  }
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_run_set_state(dock_run_t r, const float* q_cur, const float* E_cur, const float* q_best,
                       const float* E_best, int32_t step, void* stream) try {
  if (!r || !q_cur || !E_cur || !q_best || !E_best) return fail(DOCK_E_ARG, "null argument");
  if (step < 0) return fail(DOCK_E_ARG, "negative step");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t nt = size_t(r->n_lig) * r->T;
  HIP_TRY(hipMemcpyAsync(r->q_cur, q_cur, nt * r->q_stride * sizeof(float), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(r->q_best, q_best, nt * r->q_stride * sizeof(float), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(r->E_cur, E_cur, nt * sizeof(float), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(r->E_best, E_best, nt * sizeof(float), hipMemcpyDeviceToDevice, s));
  HIP_TRY(launch_fill_int(r->d_step, 1, step, s));
  r->step = step;
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_run_kernel_ms(dock_run_t r, float* ms) try {
  if (!r || !ms) return fail(DOCK_E_ARG, "null argument");
  if (!r->timed) return fail(DOCK_E_ARG, "run has no timed launches");
  HIP_TRY(hipEventSynchronize(r->ev1));
  HIP_TRY(hipEventElapsedTime(ms, r->ev0, r->ev1));
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_run_launch_stats(dock_run_t r, dock_launch_stat* out, int32_t cap, int32_t* n) try {
  if (!r || !n) return fail(DOCK_E_ARG, "null argument");
  if (!r->launches.empty()) HIP_TRY(hipEventSynchronize(r->launches.back().b));
  int k = 0;
  for (auto& L : r->launches) {
    if (out && k < cap) {
      dock_launch_stat st = L.st;
      float ms = -1.f;
      if (hipEventElapsedTime(&ms, L.a, L.b) == hipSuccess) st.ms = ms;
      out[k] = st;
    }
    ++k;
  }
  *n = k;
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_run_plan(dock_run_t r, int32_t* lig_bucket, int32_t* bucket_lanes, int32_t* bucket_apl,
                  int32_t* n_buckets) try {
  if (!r) return fail(DOCK_E_ARG, "null run");
  if (lig_bucket)
    for (int l = 0; l < r->n_lig; ++l) lig_bucket[l] = r->lig_bucket[l];
  for (size_t b = 0; b < r->buckets.size(); ++b) {
    if (bucket_lanes) bucket_lanes[b] = r->buckets[b].lpp;
    if (bucket_apl) bucket_apl[b] = r->buckets[b].apl;
  }
  if (n_buckets) *n_buckets = int(r->buckets.size());
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_free_run(dock_run_t r) try {
  if (!r) return DOCK_OK;
  (void)hipDeviceSynchronize();
  free_run(r);
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

// ================================================================ best poses

int dock_best_poses(dock_ligands_t L, int32_t n_traj, const float* E_best, const float* q_best,
                    int32_t q_stride, int32_t top_n, float rmsd_cluster, float w_tor, float* E_out,
                    float* E_screen, float* q_out, int32_t* idx_out, float* xyz_out, int32_t xyz_stride,
                    int32_t* n_out, void* stream) try {
  if (!L) return fail(DOCK_E_ARG, "null ligands");
  if (L->host_only) return fail(DOCK_E_ARG, "ligand handle was loaded host_only");
  if (n_traj < 1 || n_traj > 8192) return fail(DOCK_E_ARG, "n_traj must be in [1, 8192]");
  if (top_n < 1 || top_n > 32) return fail(DOCK_E_ARG, "top_n must be in [1, 32]");
  if (!E_best || !q_best) return fail(DOCK_E_ARG, "null candidate arrays");
  if (q_stride < 6 + L->max_tors) return fail(DOCK_E_ARG, "q_stride < 6 + max torsions");
  if (xyz_out && xyz_stride < 3 * L->max_atoms) return fail(DOCK_E_ARG, "xyz_stride < 3 * max atoms");
  if (!std::isfinite(rmsd_cluster) || !std::isfinite(w_tor)) return fail(DOCK_E_ARG, "non-finite parameter");
  BestArgs a{};
  a.L = L->arrays();
  a.n_ligands = L->n;
  a.n_traj = n_traj;
  a.q_stride = q_stride;
  a.E_best = E_best;
  a.q_best = q_best;
  a.top_n = top_n;
  a.rmsd_cut = rmsd_cluster;
  a.w_tor = w_tor;
  a.E_out = E_out;
  a.E_screen = E_screen;
  a.q_out = q_out;
  a.idx_out = idx_out;
  a.xyz_out = xyz_out;
  a.xyz_stride = xyz_stride;
  a.n_out = n_out;
  int tp = 1;
  while (tp < n_traj) tp <<= 1;
  a.t_pad = tp;
  if ((size_t(tp) * 8 + 15) / 16 * 16 + size_t(top_n) * kMaxAtoms * 16 > 64 * 1024)
    return fail(DOCK_E_LIMIT, "n_traj * top_n too large for the best-pose LDS budget");
  HIP_TRY(launch_best(a, reinterpret_cast<hipStream_t>(stream)));
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_pocket_map_adjoint(dock_pocket_t p, const float* dLdG, float* dLdxyz, double* dLdtheta,
                            void* stream) try {
  if (!p || !dLdG) return fail(DOCK_E_ARG, "null argument");
  if (p->dev.inter_mode != DOCK_INTER_GRID || !p->d_rec)
    return fail(DOCK_E_ARG, "the map adjoint needs a grid-mode pocket");
  if (p->dev.preset != DOCK_PRESET_TRIDS) return fail(DOCK_E_ARG, "the map adjoint covers the TRIDS terms");
  MapAdjArgs a{};
  a.rec = p->d_rec;
  a.n_rec = p->n_rec;
  a.grid = p->dev.grid;
  type_pair_table(DOCK_PRESET_TRIDS, a.tab);
  a.lam = dLdG;
  a.dLdxyz = dLdxyz;
  a.dLdtheta = dLdtheta;
  HIP_TRY(launch_map_adjoint(a, reinterpret_cast<hipStream_t>(stream)));
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

// The rank passes of dock_screen_rank: each keeps top_k of every block of
// kRankBlock entries (at least halving the count) until one block remains,
// whose output is the answer.  bufs / ibufs: two ping-pong buffers of
// ceil(n / kRankBlock) * top_k entries each (unused when one block holds n).
static hipError_t rank_passes(const float* scores, int64_t n, int32_t stride, int32_t top_k, float* score_out,
                              int32_t* lig_out, float* const bufs[2], int* const ibufs[2], hipStream_t s) {
  RankArgs a{};
  a.score = scores;
  a.idx = nullptr;
  a.n = n;
  a.stride = stride;
  a.k = top_k;
  int cur = 0;
  for (;;) {
    const long long blocks = (a.n + kRankBlock - 1) / kRankBlock;
    if (blocks <= 1) {
      // final pass, straight into the outputs (n = 0: one block of empty slots)
      a.out_score = score_out;
      a.out_idx = lig_out;
      return launch_rank(a, s);
    }
    a.out_score = bufs[cur];
    a.out_idx = ibufs[cur];
    const hipError_t e = launch_rank(a, s);
    if (e != hipSuccess) return e;
    a.score = bufs[cur];
    a.idx = ibufs[cur];
    a.n = blocks * top_k;
    a.stride = 1;
    cur ^= 1;
  }
}

static int check_rank_args(const float* scores, int64_t n, int32_t stride, int32_t top_k, const float* score_out,
                           const int32_t* lig_out) {
  if (n < 0 || n > (int64_t(1) << 31) - 2) return fail(DOCK_E_ARG, "n must be in [0, 2^31 - 2]");
  if (stride < 1) return fail(DOCK_E_ARG, "stride must be >= 1");
  if (top_k < 1 || top_k > 1024) return fail(DOCK_E_ARG, "top_k must be in [1, 1024]");
  if (!score_out || !lig_out || (n > 0 && !scores)) return fail(DOCK_E_ARG, "null array");
  return DOCK_OK;
}

int dock_screen_rank(const float* scores, int64_t n, int32_t stride, int32_t top_k, float* score_out,
                     int32_t* lig_out, void* stream) try {
  int rc = check_rank_args(scores, n, stride, top_k, score_out, lig_out);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long long blocks0 = (n + kRankBlock - 1) / kRankBlock;
  float* bufs[2] = {nullptr, nullptr};
  int* ibufs[2] = {nullptr, nullptr};
  hipError_t e = hipSuccess;
  if (blocks0 > 1) {
    const size_t cap = size_t(blocks0) * size_t(top_k);
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
      e = hipMallocAsync(reinterpret_cast<void**>(&bufs[b]), cap * sizeof(float), s);
      if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&ibufs[b]), cap * sizeof(int), s);
    }
  }
  if (e == hipSuccess) e = rank_passes(scores, n, stride, top_k, score_out, lig_out, bufs, ibufs, s);
  for (int b = 0; b < 2; ++b) {
    if (bufs[b]) (void)hipFreeAsync(bufs[b], s);
    if (ibufs[b]) (void)hipFreeAsync(ibufs[b], s);
  }
  if (e != hipSuccess) return fail(DOCK_E_HIP, hipGetErrorString(e));
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

// Scratch of dock_screen_rank_noalloc: the two ping-pong buffer pairs
// (float scores, int ligand indices) of kNoAllocRankEntries entries each,
// one copy per GPU for the life of the process.  Host code never passes this
// name to a kernel: it stands for a host-side shadow, not the device address.
// The address on each device comes from hipGetSymbolAddress (noalloc_scratch).
constexpr size_t kNoAllocRankEntries = size_t(DOCK_NOALLOC_RANK_ENTRIES);
static __device__ __align__(256) unsigned char scratch[4 * kNoAllocRankEntries * 4];

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
static int noalloc_scratch(unsigned char** out) {
  static std::mutex mu;
  static std::map<int, unsigned char*> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(DOCK_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DOCK_E_HIP, std::string("scratch symbol address: ") + hipGetErrorString(e));
    it = addr.emplace(dev, static_cast<unsigned char*>(p)).first;
  }
  *out = it->second;
  return DOCK_OK;
}

int dock_screen_rank_noalloc(const float* scores, int64_t n, int32_t stride, int32_t top_k, float* score_out,
                             int32_t* lig_out, void* stream) try {
  int rc = check_rank_args(scores, n, stride, top_k, score_out, lig_out);
  if (rc) return rc;
  const long long blocks0 = (n + kRankBlock - 1) / kRankBlock;
  if (blocks0 > 1 && size_t(blocks0) * size_t(top_k) > kNoAllocRankEntries)
    return fail(DOCK_E_LIMIT, "ceil(n / 2048) * top_k exceeds the static scratch (" +
                                  std::to_string(kNoAllocRankEntries) + " entries)");
  unsigned char* base = nullptr;
  rc = noalloc_scratch(&base);
  if (rc) return rc;
  // every pass writes each entry it later reads: nothing needs clearing
  float* bufs[2] = {reinterpret_cast<float*>(base), reinterpret_cast<float*>(base + 4 * kNoAllocRankEntries)};
  int* ibufs[2] = {reinterpret_cast<int*>(base + 8 * kNoAllocRankEntries),
                   reinterpret_cast<int*>(base + 12 * kNoAllocRankEntries)};
  const hipError_t e = rank_passes(scores, n, stride, top_k, score_out, lig_out, bufs, ibufs,
                                   reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(DOCK_E_HIP, hipGetErrorString(e));
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

int dock_philox(const uint32_t* counters, uint32_t k0, uint32_t k1, int64_t n, uint32_t* out,
                void* stream) try {
  if (n < 0) return fail(DOCK_E_ARG, "negative n");
  if (n > 0 && (!counters || !out)) return fail(DOCK_E_ARG, "null array");
  HIP_TRY(launch_philox(counters, k0, k1, n, out, reinterpret_cast<hipStream_t>(stream)));
  return DOCK_OK;
} catch (...) {
  return exception_status();
}

}  // extern "C"
