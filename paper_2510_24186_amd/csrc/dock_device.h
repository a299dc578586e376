// Device building blocks of the docking hot path (gfx950, wave64).
//
// A pose is evaluated by a group of LPP lanes (16, 32 or 64) of one
// wavefront.  Lane roles change through the evaluation:
//   * lane r holds DOF r (r < 6 + n_t): q, its gradient, optimiser state;
//   * lane f < n_frags composes fragment f's rigid transform;
//   * lane r owns atoms APL*r .. APL*r+APL-1 (atoms in fragment DFS order);
//   * all lanes stride over the intra-ligand pair list.
// Cross-lane traffic uses shuffles within the group; per-pose coordinates
// and intra forces live in a small LDS slab private to the group.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dock_internal.h"

namespace dock {

#define DK_INLINE __device__ __forceinline__

constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kInvTwoPi = 0.15915494309189533577f;
constexpr float kOutK = 10.0f;

// ------------------------------------------------------------------ sync
DK_INLINE void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ Philox4x32-10
// Salmon et al., SC'11: two 32x32->64 multiplies per round, high halves mixed
// with the other two words and the key, key bumped by Weyl constants.
DK_INLINE uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}
DK_INLINE float u01(uint32_t x) { return float(x >> 8) * 5.9604644775390625e-8f; }
DK_INLINE uint32_t pick4(uint4 w, int i) {
  return i == 0 ? w.x : (i == 1 ? w.y : (i == 2 ? w.z : w.w));
}

// ------------------------------------------------------------------ cross-lane
// Groups of W lanes (W = 16, 32, 64) inside one wavefront.  ds_bpermute
// takes a byte address; when several values come from the same source lane
// the address is computed once (bp_addr) and reused.
template <int W>
DK_INLINE int bp_addr(int src) {
  return int((__lane_id() & ~unsigned(W - 1)) + unsigned(src)) << 2;
}
DK_INLINE float bp(int addr, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
DK_INLINE int bp(int addr, int v) { return __builtin_amdgcn_ds_bpermute(addr, v); }
template <int W>
DK_INLINE float shfl(float v, int src) { return bp(bp_addr<W>(src), v); }
template <int W>
DK_INLINE int shfl(int v, int src) { return bp(bp_addr<W>(src), v); }
// Value of lane `src` (the same for every lane of the group) to all lanes of
// the group: a scalar read of one lane when the group is the whole wave.
template <int W>
DK_INLINE float bcast(float v, int src) {
  if (W == 64) return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
  return shfl<W>(v, src);
}

// DPP controls (GFX9 encoding)
constexpr int kDppQuadXor1 = 0xB1;    // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;    // quad_perm [2,3,0,1]
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShr4 = 0x114;
constexpr int kDppRowShr8 = 0x118;
constexpr int kDppRowMirror = 0x140;      // lane i <-> 15 - i within a row
constexpr int kDppRowHalfMirror = 0x141;  // lane i <-> 7 - i within a half row
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

template <int CTRL, int ROW_MASK = 0xf>
DK_INLINE float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}
// v += (last lane of the previous row) in rows 1 and 3, and v += lane 31 in
// rows 2 and 3: one DPP add each, the disabled rows keeping v.  (Written out
// because the compiler emits a move, an add and a reset of the move's old
// value for the masked form; s_nop 1 gives the two wait states a DPP read
// needs after a VALU write of its source.)
DK_INLINE float add_row_bcast15(float v) {
  asm("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf" : "+v"(v));
  return v;
}
DK_INLINE float add_row_bcast31(float v) {
  asm("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf" : "+v"(v));
  return v;
}

// Sum over the group.  Every step adds a lane's value to its partner's, and
// the partner does the same with the operands swapped, so all lanes end with
// bitwise-identical sums (MC decisions taken from them are uniform).
// Rows (16 lanes) and wave halves are exchanged with the gfx950 permlane
// swaps: with both operands v, the two results hold v and its partner's
// value in opposite order, so their sum is the butterfly step.
template <int W>
DK_INLINE float group_sum(float v) {
  v += dpp<kDppQuadXor1>(v);
  v += dpp<kDppQuadXor2>(v);
  v += dpp<kDppRowHalfMirror>(v);
  v += dpp<kDppRowMirror>(v);
  if (W >= 32) {
    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  }
  if (W >= 64) {
    const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  }
  return v;
}

// Inclusive prefix sum over the group (Hillis-Steele within 16-lane rows,
// then row totals broadcast to the following rows).
template <int W>
DK_INLINE float group_scan(float v) {
  v += dpp<kDppRowShr1>(v);
  v += dpp<kDppRowShr2>(v);
  v += dpp<kDppRowShr4>(v);
  v += dpp<kDppRowShr8>(v);
  if (W >= 32) v = add_row_bcast15(v);
  if (W >= 64) v = add_row_bcast31(v);
  return v;
}

// ------------------------------------------------------------------ terms
// Pair word: i | j << 8 | type_i << 16 | type_j << 20 | flags << 24, plus the
// radius sum as a float.  flags bit0 donor/acceptor pair, bit1 both
// hydrophobic, bit7 empty slot (no pair).
// Pass layout: each slot takes two entries, the pair word and radius sum,
// then the E_clash constants d_clash^2 (negated for a donor/acceptor pair)
// and log2(d_clash) (FP32 bit patterns in a second PairRec), so record p
// still starts at entry 2p; after the n_prec slots come the pull bytes,
// apl * cap per lane and pass (see PassPlan).  An empty slot names atoms 0
// and 0 with a radius sum of -1e4 and zero clash constants, which makes every
// term of both presets exactly zero.
constexpr uint32_t kPairEmpty = 0x80u << 24;
constexpr float kEmptyRsum = -1.0e4f;
struct PairRec {
  uint32_t w;
  float rsum;
};

typedef float f32x4_t __attribute__((ext_vector_type(4)));

// LDS byte addresses.  A gather address is formed in one instruction by a
// byte dot product (v_dot4_u32_u8): byte k of a packed word times 16 plus the
// array's base address.
DK_INLINE uint32_t lds_addr(const void* p) {
  return uint32_t(reinterpret_cast<uintptr_t>((const __attribute__((address_space(3))) char*)p));
}
DK_INLINE uint32_t lds_entry16_k(uint32_t packed, int k, uint32_t base) {
  return __builtin_amdgcn_udot4(packed, 16u << (8 * k), base, false);
}
template <int K>
DK_INLINE uint32_t lds_entry16(uint32_t packed, uint32_t base) {
  return lds_entry16_k(packed, K, base);
}
// 16-byte entries are read and written whole: on gfx950 a 12-byte LDS access
// costs about twice a 16-byte one (the volatile read keeps the compiler from
// narrowing it when the fourth word is unused).
DK_INLINE f32x4_t lds_read4(uint32_t a) {
  return *(const volatile __attribute__((address_space(3))) f32x4_t*)(uintptr_t)a;
}
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
DK_INLINE uint4 lds_read_u4(uint32_t a) {
  const u32x4_t v = *(const __attribute__((address_space(3))) u32x4_t*)(uintptr_t)a;
  return make_uint4(v.x, v.y, v.z, v.w);
}
// two consecutive dwords at a 4-byte aligned address (one ds_read2_b32)
DK_INLINE uint2 lds_read_u2(uint32_t a) {
  const __attribute__((address_space(3))) uint32_t* p = (const __attribute__((address_space(3))) uint32_t*)(uintptr_t)a;
  return make_uint2(p[0], p[1]);
}
DK_INLINE void lds_write4(uint32_t a, float x, float y, float z) {
  const f32x4_t v = {x, y, z, 0.f};
  *(__attribute__((address_space(3))) f32x4_t*)(uintptr_t)a = v;
}

// Loads through a pointer known to address global memory.  Pointers read
// out of device-side structs (the pocket table) are generic to the
// compiler, which then emits FLAT accesses; those also count against the LDS
// wait counter, so every later LDS wait of the wave would drain them too.
template <typename T>
DK_INLINE T ldg(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
typedef float f32x2_t __attribute__((ext_vector_type(2)));
DK_INLINE float4 ldg(const float4* p) {
  const f32x4_t v = *(const __attribute__((address_space(1))) f32x4_t*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
DK_INLINE float2 ldg(const float2* p) {
  const f32x2_t v = *(const __attribute__((address_space(1))) f32x2_t*)p;
  return make_float2(v.x, v.y);
}
typedef int i32x2_t __attribute__((ext_vector_type(2)));
DK_INLINE int2 ldg(const int2* p) {
  const i32x2_t v = *(const __attribute__((address_space(1))) i32x2_t*)p;
  return make_int2(v.x, v.y);
}

// exp(x) on the hardware exp2 (v_exp_f32): callers pass x * log2(e) already
// folded into their constants.  Relative error ~1e-6 for the Gaussian
// arguments used here (|x| < 40).
DK_INLINE float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
// log2 and 1/x on the hardware units (v_log_f32, v_rcp_f32; about 1 ulp) for
// normal positive arguments: the clash term only sees d in [0.1, d_clash).
DK_INLINE float log2_hw(float x) { return __builtin_amdgcn_logf(x); }
DK_INLINE float rcp_hw(float x) { return __builtin_amdgcn_rcpf(x); }
DK_INLINE float sqrt_hw(float x) { return __builtin_amdgcn_sqrtf(x); }

// Weighted TRIDS terms (Methods: E_long, E_clash, E_Hbond) at distance d
// (d2 = d*d): energy and dE/dd.
DK_INLINE void trids_pair(float d2, float d, float rsum, uint32_t flags, const float* w, float& e,
                          float& de) {
  e = 0.f;
  de = 0.f;
  if (d2 < 100.0f) {
    const float s = d - rsum - 3.0f;
    const float ex = exp2_hw(s * s * (-0.25f * kLog2e));
    e -= w[0] * ex;
    de += w[0] * 0.5f * s * ex;
  }
  const bool hb = flags & 1u;
  const float dc = hb ? 2.6f : rsum;
  if (d2 < dc * dc) {
    const float dd = fmaxf(d, 0.1f);
    e -= (w[1] * kLn2) * log2_hw(dd * rcp_hw(dc));
    if (d > 0.1f) de -= w[1] * rcp_hw(dd);
  }
  if (hb && d2 < 3.4f * 3.4f) {
    const float t = d - 2.88f;
    const float ex = exp2_hw(t * t * (-kLog2e / 0.18f));
    e -= w[2] * ex;
    de += w[2] * ex * t * (2.0f / 0.18f);
  }
}

// The TRIDS terms as trids_pair, with the clash cutoff and log2 of the clash
// distance taken from the slot record (|dc2| = d_clash^2, negative for a
// donor/acceptor pair; l2dc = log2 d_clash): -log(dd / dc) =
// -ln2 (log2 dd - log2 dc), and for d > 0.1 the derivative -1/d comes from
// the caller's 1/d.
DK_INLINE void trids_pair_k(float d2, float d, float inv_d, float rsum, float dc2, float l2dc,
                            const float* w, float& e, float& de) {
  const float s = d - rsum - 3.0f;
  float ex = exp2_hw(s * s * (-0.25f * kLog2e));
  ex = d2 < 100.0f ? ex : 0.f;
  e = -w[0] * ex;
  de = (w[0] * 0.5f) * s * ex;
  if (d2 < fabsf(dc2)) {
    const bool far = d > 0.1f;
    e -= (w[1] * kLn2) * (log2_hw(far ? d : 0.1f) - l2dc);
    if (far) de -= w[1] * inv_d;
  }
  // few slots hold a donor/acceptor pair inside 3.4 A: the term is skipped
  // unless some lane of the wave needs it
  const bool hb_in = (dc2 < 0.f) & (d2 < 3.4f * 3.4f);
  if (__builtin_amdgcn_ballot_w64(hb_in)) {
    const float t = d - 2.88f;
    const float eh = hb_in ? exp2_hw(t * t * (-kLog2e / 0.18f)) : 0.f;
    e -= w[2] * eh;
    de += (w[2] * (2.0f / 0.18f)) * t * eh;
  }
}

// Weighted Vina-form terms (gauss1, gauss2, repulsion, hydrophobic, hbond).
DK_INLINE void vina_pair(float d2, float d, float rsum, uint32_t flags, const float* w, float& e,
                         float& de) {
  e = 0.f;
  de = 0.f;
  if (!(d2 < 64.0f)) return;
  const float s = d - rsum;
  const float g1 = exp2_hw(s * s * (-4.0f * kLog2e));
  e += w[0] * g1;
  de -= w[0] * 8.0f * s * g1;
  const float t = s - 3.0f;
  const float g2 = exp2_hw(t * t * (-0.25f * kLog2e));
  e += w[1] * g2;
  de -= w[1] * 0.5f * t * g2;
  if (s < 0.f) {
    e += w[2] * s * s;
    de += w[2] * 2.0f * s;
  }
  if (flags & 2u) {
    if (s < 0.5f) {
      e += w[3];
    } else if (s < 1.5f) {
      e += w[3] * (1.5f - s);
      de -= w[3];
    }
  }
  if (flags & 1u) {
    if (s < -0.7f) {
      e += w[4];
    } else if (s < 0.f) {
      e -= w[4] * s * (1.0f / 0.7f);
      de -= w[4] * (1.0f / 0.7f);
    }
  }
}

// Unweighted per-term values and d/dd of a ligand-internal pair (FP32, cutoff
// decisions on the FP32 squared distance).  Order as the presets' weights.
template <int K>
DK_INLINE void pair_terms_f32(float d2, float d, float rsum, uint32_t flags, float (&v)[K],
                              float (&dv)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = dv[k] = 0.f;
  if (K == 3) {
    if (d2 < 100.0f) {
      const float s = d - rsum - 3.0f;
      const float ex = expf(-0.25f * s * s);
      v[0] = -ex;
      dv[0] = 0.5f * s * ex;
    }
    const bool hb = flags & 1u;
    const float dc = hb ? 2.6f : rsum;
    if (d2 < dc * dc) {
      const float dd = fmaxf(d, 0.1f);
      v[1] = -logf(dd / dc);
      dv[1] = d > 0.1f ? -1.0f / dd : 0.f;
    }
    if (hb && d2 < 3.4f * 3.4f) {
      const float t = d - 2.88f;
      const float ex = expf(-t * t * (1.0f / 0.18f));
      v[2] = -ex;
      dv[2] = ex * t * (2.0f / 0.18f);
    }
  } else {
    if (!(d2 < 64.0f)) return;
    const float s = d - rsum;
    const float g1 = expf(-4.0f * s * s);
    v[0] = g1;
    dv[0] = -8.0f * s * g1;
    const float t = s - 3.0f;
    const float g2 = expf(-0.25f * t * t);
    v[1] = g2;
    dv[1] = -0.5f * t * g2;
    if (s < 0.f) {
      v[2] = s * s;
      dv[2] = 2.0f * s;
    }
    if (flags & 2u) {
      if (s < 0.5f) {
        v[3] = 1.0f;
      } else if (s < 1.5f) {
        v[3] = 1.5f - s;
        dv[3] = -1.0f;
      }
    }
    if (flags & 1u) {
      if (s < -0.7f) {
        v[4] = 1.0f;
      } else if (s < 0.f) {
        v[4] = -s * (1.0f / 0.7f);
        dv[4] = -1.0f / 0.7f;
      }
    }
  }
}

// Per-term values (no weights) of a receptor/ligand type pair for the map
// build: each term's inside-cutoff decision is taken on the FP32 squared
// distance d2; the values are evaluated in FP64 from the FP64 distance d.
DK_INLINE void pair_terms_unweighted(int preset, float d2, double d, double rsum, float dclash2,
                                     double dclash, uint32_t flags, double* v) {
  if (preset == DOCK_PRESET_TRIDS) {
    v[0] = v[1] = v[2] = 0.0;
    if (d2 < 100.0f) {
      const double s = d - rsum - 3.0;
      v[0] = -exp(-0.25 * s * s);
    }
    if (d2 < dclash2) v[1] = -log(fmax(d, 0.1) / dclash);
    if ((flags & 1u) && d2 < 3.4f * 3.4f) {
      const double t = d - 2.88;
      v[2] = -exp(-t * t / 0.18);
    }
  } else {
    v[0] = v[1] = v[2] = v[3] = v[4] = 0.0;
    if (!(d2 < 64.0f)) return;
    const double s = d - rsum;
    v[0] = exp(-4.0 * s * s);
    const double t = s - 3.0;
    v[1] = exp(-0.25 * t * t);
    v[2] = s < 0.0 ? s * s : 0.0;
    if (flags & 2u) v[3] = s < 0.5 ? 1.0 : (s < 1.5 ? 1.5 - s : 0.0);
    if (flags & 1u) v[4] = s < -0.7 ? 1.0 : (s < 0.0 ? -s / 0.7 : 0.0);
  }
}

// ------------------------------------------------------------------ trilinear
// Cell = floor((p - o) / h) clamped to [0, n-2] at the clamped point; value,
// analytic cell-local gradient, and the out-of-box penalty 10 |p - clamp(p)|_1.
struct Trilerp {
  float v, gx, gy, gz, eout;
  int base;          // flat index of corner (0,0,0)
  float fx, fy, fz;  // cell fractions
};

DK_INLINE void cell_axis(float p, float o, float hi, float inv_h, int n, float& pc, bool& in, int& c,
                         float& f) {
  pc = __builtin_amdgcn_fmed3f(p, o, hi);  // clamp to [o, hi]
  in = pc == p;
  const float u = (pc - o) * inv_h;        // >= 0, so truncation is floor
  c = min(int(u), n - 2);
  f = u - float(c);
}

DK_INLINE Trilerp trilerp(const float* __restrict__ M, const GridDev& g, float px, float py, float pz) {
  Trilerp t;
  float pcx, pcy, pcz;
  bool ix, iy, iz;
  int cx, cy, cz;
  cell_axis(px, g.origin[0], g.hi[0], g.inv_spacing, g.dims[0], pcx, ix, cx, t.fx);
  cell_axis(py, g.origin[1], g.hi[1], g.inv_spacing, g.dims[1], pcy, iy, cy, t.fy);
  cell_axis(pz, g.origin[2], g.hi[2], g.inv_spacing, g.dims[2], pcz, iz, cz, t.fz);
  // nodes per map <= 2^30: 32-bit node indices
  const uint32_t nx = uint32_t(g.dims[0]), nxy = uint32_t(g.dims[0]) * uint32_t(g.dims[1]);
  t.base = int((uint32_t(cz) * uint32_t(g.dims[1]) + uint32_t(cy)) * nx + uint32_t(cx));
  const float* p0 = M + uint32_t(t.base);
  const float c000 = ldg(p0), c100 = ldg(p0 + 1), c010 = ldg(p0 + nx), c110 = ldg(p0 + nx + 1);
  const float c001 = ldg(p0 + nxy), c101 = ldg(p0 + nxy + 1), c011 = ldg(p0 + nxy + nx),
              c111 = ldg(p0 + nxy + nx + 1);
  const float fx = t.fx, fy = t.fy, fz = t.fz;
  // interpolate along x, then y, then z
  const float x00 = c000 + fx * (c100 - c000), x10 = c010 + fx * (c110 - c010);
  const float x01 = c001 + fx * (c101 - c001), x11 = c011 + fx * (c111 - c011);
  const float y0 = x00 + fy * (x10 - x00), y1 = x01 + fy * (x11 - x01);
  t.v = y0 + fz * (y1 - y0);
  const float dx00 = c100 - c000, dx10 = c110 - c010, dx01 = c101 - c001, dx11 = c111 - c011;
  const float dxy0 = dx00 + fy * (dx10 - dx00), dxy1 = dx01 + fy * (dx11 - dx01);
  const float gxf = dxy0 + fz * (dxy1 - dxy0);
  const float gyf = (x10 - x00) + fz * ((x11 - x01) - (x10 - x00));
  const float gzf = y1 - y0;
  // outside the box along an axis the map gradient is zero there and the
  // penalty's slope is +-10 (the offset is nonzero exactly when outside)
  const float ox = px - pcx, oy = py - pcy, oz = pz - pcz;
  t.eout = kOutK * (fabsf(ox) + fabsf(oy) + fabsf(oz));
  t.gx = ix ? gxf * g.inv_spacing : copysignf(kOutK, ox);
  t.gy = iy ? gyf * g.inv_spacing : copysignf(kOutK, oy);
  t.gz = iz ? gzf * g.inv_spacing : copysignf(kOutK, oz);
  return t;
}

// ------------------------------------------------------------------ direct pair mode
// Receptor terms summed pair by pair over the atoms inside the cutoff (the
// paper's cutoff pair kernel).  Cells are half a cutoff wide, so every
// receptor atom within the cutoff lies in the 5 x 5 x 5 cells around the
// ligand atom's cell; for fixed (z, y) the run of 5 x-cells is one contiguous
// range of the cell-sorted atom array.
DK_INLINE void inter_direct(const PocketDev& pk, int preset, const float* w, int lt, float px, float py,
                            float pz, float& e, float& gx, float& gy, float& gz) {
  e = gx = gy = gz = 0.f;
  const float cut2 = preset == DOCK_PRESET_TRIDS ? 100.0f : 64.0f;
  int lo[3], hi[3];
  const float p[3] = {px, py, pz};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float u = fminf(fmaxf((p[c] - pk.cell_origin[c]) * pk.inv_cell, -8.0f), float(pk.cell_dims[c] + 8));
    const int ic = int(floorf(u));
    lo[c] = max(ic - 2, 0);
    hi[c] = min(ic + 2, pk.cell_dims[c] - 1);
  }
  if (lo[0] > hi[0]) return;
  const int nx = pk.cell_dims[0], nxy = pk.cell_dims[0] * pk.cell_dims[1];
  for (int z = lo[2]; z <= hi[2]; ++z) {
    for (int y = lo[1]; y <= hi[1]; ++y) {
      const int row = z * nxy + y * nx;
      const int b = ldg(pk.cell_start + row + lo[0]), end = ldg(pk.cell_start + row + hi[0] + 1);
      for (int i = b; i < end; ++i) {
        const float4 rr = ldg(pk.rec + i);
        const float dx = px - rr.x, dy = py - rr.y, dz = pz - rr.z;
        const float d2 = dx * dx + dy * dy + dz * dz;
        if (!(d2 < cut2)) continue;
        const float2 tp = ldg(pk.tp + lt * kTypes + (__float_as_int(rr.w) & 0xff));
        const float inv_d = d2 > 0.f ? __builtin_amdgcn_rsqf(d2) : 0.f;
        const float d = d2 * inv_d;
        float ee, de;
        if (preset == DOCK_PRESET_TRIDS)
          trids_pair(d2, d, tp.x, __float_as_uint(tp.y), w, ee, de);
        else
          vina_pair(d2, d, tp.x, __float_as_uint(tp.y), w, ee, de);
        e += ee;
        const float cf = de * inv_d;
        gx += cf * dx;
        gy += cf * dy;
        gz += cf * dz;
      }
    }
  }
}

// ------------------------------------------------------------------ E_MDN
// Mixture term of one ligand atom at x (Methods, E_MDN): the residues listed
// for x's lattice cell, the nearest atom of each, and for d < 5 A the
// mixture P(d) from the atom's parameters for that residue (float4 pi, mu,
// log2(e) / (2 sigma^2), 1 / sigma^2).  Adds -w P to e and its gradient to g.
struct MdnArg {
  const float4* par;  // this ligand's table: [atom (DFS)][residue][gaussian]
  int n_res, k;
};

DK_INLINE void mdn_term(const PocketDev& pk, const MdnArg& m, int atom, float px, float py, float pz, float& e,
                        float& gx, float& gy, float& gz) {
  int ic[3];
  const float p[3] = {px, py, pz};
#pragma unroll
  for (int c = 0; c < 3; ++c) ic[c] = int(floorf((p[c] - pk.mcell_origin[c]) * pk.inv_mcell));
  if (ic[0] < 0 || ic[1] < 0 || ic[2] < 0 || ic[0] >= pk.mcell_dims[0] || ic[1] >= pk.mcell_dims[1] ||
      ic[2] >= pk.mcell_dims[2])
    return;  // farther than the cutoff from every receptor atom
  const int cell = (ic[2] * pk.mcell_dims[1] + ic[1]) * pk.mcell_dims[0] + ic[0];
  const int b = ldg(pk.mcell_start + cell), end = ldg(pk.mcell_start + cell + 1);
  const float4* par_atom = m.par + size_t(atom) * m.n_res * m.k;
  float es = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
  for (int q = b; q < end; ++q) {
    const int res = ldg(pk.mcell_res + q);
    const int2 rng = ldg(pk.res_range + res);
    float best = INFINITY, bx = 0.f, by = 0.f, bz = 0.f;
    for (int a = rng.x; a < rng.y; ++a) {
      const float4 r = ldg(pk.res_xyz + a);
      const float dx = px - r.x, dy = py - r.y, dz = pz - r.z;
      const float d2 = dx * dx + dy * dy + dz * dz;
      if (d2 < best) {
        best = d2;
        bx = dx;
        by = dy;
        bz = dz;
      }
    }
    if (!(best < kMdnCutoff * kMdnCutoff)) continue;
    const float inv_d = best > 0.f ? __builtin_amdgcn_rsqf(best) : 0.f;
    const float d = best * inv_d;
    const float4* pr = par_atom + size_t(res) * m.k;
    float P = 0.f, dP = 0.f;
    for (int k = 0; k < m.k; ++k) {
      const float4 g = ldg(pr + k);
      const float x = d - g.y;
      const float v = g.x * exp2_hw(-(x * x) * g.z);
      P += v;
      dP -= v * x * g.w;
    }
    es -= P;
    const float c = -dP * inv_d;
    sx += c * bx;
    sy += c * by;
    sz += c * bz;
  }
  e += pk.mdn_w * es;
  gx += pk.mdn_w * sx;
  gy += pk.mdn_w * sy;
  gz += pk.mdn_w * sz;
}

// ------------------------------------------------------------------ pose evaluation
// Static per-ligand data held in registers by each lane of a group.
template <int APL>
struct LaneLig {
  int n_atoms, n_frags, n_dof, n_prec, fk_rounds, preset;
  int n_pass, pass_w, pull_cap, pass_apl;  // pass layout of the pair records (n_pass = 0: strided)
  // atoms owned by this lane
  float ax[APL], ay[APL], az[APL];
  int atype[APL], afrag[APL], aorig[APL];
  // fragment owned by this lane
  float fu[3], fxb[3];
  int fparent, fdof;
  // DOF owned by this lane: range and, for torsions, the chain-rule record
  float lo, hi;
  int tsb, tse, ta, tb;
  float w[kMaxTerms];
};

template <int LPP, int APL>
DK_INLINE void load_lane_lig(LaneLig<APL>& L, const LigDev& lg, const LigDev* __restrict__ lgp,
                             const float4* __restrict__ atoms, const FragDev* __restrict__ frags,
                             const TorsDev* __restrict__ tors, const PocketDev& pk, int r) {
  L.n_atoms = lg.n_atoms;
  L.n_frags = lg.n_frags;
  L.n_dof = lg.n_dof;
  L.n_prec = lg.n_prec;
  L.n_pass = lg.n_pass;
  L.pass_w = lg.pass_w;
  L.pull_cap = lg.pull_cap;
  L.pass_apl = lg.pass_apl;
  L.fk_rounds = lg.fk_rounds;
  L.preset = pk.preset;
#pragma unroll
  for (int s = 0; s < APL; ++s) {
    const int a = APL * r + s;
    if (a < lg.n_atoms) {
      const float4 v = atoms[lg.atom_off + a];
      const int bits = __float_as_int(v.w);
      L.ax[s] = v.x;
      L.ay[s] = v.y;
      L.az[s] = v.z;
      L.atype[s] = bits & 0xff;
      L.afrag[s] = (bits >> 8) & 0xff;
      L.aorig[s] = (bits >> 16) & 0xff;
    } else {
      L.ax[s] = L.ay[s] = L.az[s] = 0.f;
      L.atype[s] = 0;
      L.afrag[s] = 0;
      L.aorig[s] = 0;
    }
  }
  if (r < lg.n_frags) {
    const FragDev f = frags[lg.frag_off + r];
    L.fu[0] = f.u[0]; L.fu[1] = f.u[1]; L.fu[2] = f.u[2];
    L.fxb[0] = f.xb[0]; L.fxb[1] = f.xb[1]; L.fxb[2] = f.xb[2];
    L.fparent = f.parent;
    L.fdof = f.dof;
  } else {
    L.fu[0] = L.fu[1] = L.fu[2] = 0.f;
    L.fxb[0] = L.fxb[1] = L.fxb[2] = 0.f;
    L.fparent = -1;
    L.fdof = -1;
  }
  L.tsb = L.tse = L.ta = L.tb = 0;
  if (r < 3) {
    // lane-indexed: read from memory, not from the register copy `lg`
    L.lo = lgp->box_min[r];
    L.hi = lgp->box_max[r];
  } else {
    L.lo = -kPi;
    L.hi = kPi;
  }
  if (r >= 6 && r < lg.n_dof) {
    const TorsDev t = tors[lg.tors_off + r - 6];
    L.tsb = t.sub_begin;
    L.tse = t.sub_end;
    L.ta = t.a;
    L.tb = t.b;
  }
#pragma unroll
  for (int k = 0; k < kMaxTerms; ++k) L.w[k] = k < pk.n_terms ? pk.w[k] : 0.f;
}

// Hides the per-lane ligand fields from loop-invariant code motion: inside
// the sampler's step loop the compiler would otherwise keep every product of
// them live across evaluations, which costs more registers than recomputing.
template <int APL>
DK_INLINE void launder(LaneLig<APL>& L) {
#pragma unroll
  for (int s = 0; s < APL; ++s) {
    asm volatile("" : "+v"(L.ax[s]), "+v"(L.ay[s]), "+v"(L.az[s]));
    asm volatile("" : "+v"(L.atype[s]), "+v"(L.afrag[s]));
  }
  asm volatile("" : "+v"(L.fu[0]), "+v"(L.fu[1]), "+v"(L.fu[2]));
  asm volatile("" : "+v"(L.fxb[0]), "+v"(L.fxb[1]), "+v"(L.fxb[2]));
  asm volatile("" : "+v"(L.fparent), "+v"(L.fdof), "+v"(L.tsb), "+v"(L.tse));
  asm volatile("" : "+v"(L.ta), "+v"(L.tb));
}

// Per-group LDS slab: coordinates (w = type bits), then either per-atom
// intra-pair force sums (strided pairs, LDS atomics) or, in the pass layout,
// one force per pair slot (plain stores, gathered per atom).
// The per-atom sums are FP64: on gfx950 an FP32 LDS atomic add is executed
// one lane at a time (~3 cycles per active lane), an FP64 one at full rate.
struct GroupSlab {
  float4* xs;   // [LPP*APL]
  double* fx;   // [LPP*APL]
  double* fy;
  double* fz;
  float4* fb;   // [2 LPP + 1] force entries of the pass layout, aliases fx/fy/fz
};

struct EvalOut {
  float E;      // total energy (same on every lane of the group)
  float g;      // dE/dq for this lane's DOF (0 beyond n_dof)
};

// Rigid-body part of a pose, shared by every lane of the group.
struct Rigid {
  float Tx, Ty, Tz, sa, ca, sb, cb;
};

// Forward kinematics, first half: the local transform of the fragment owned
// by lane r (the world rotation and translation for the root; a Rodrigues
// rotation about the torsion axis for the others) as 3 x 4 rows.
struct LocalTf {
  float m[9], t[3];
  Rigid rg;
};
template <int LPP, int APL>
DK_INLINE LocalTf fk_local(const LaneLig<APL>& L, float q, int r) {
  LocalTf o;
  // ---- each lane takes sin/cos of its own angle DOF once; the rigid part
  // and every fragment's torsion are then fetched from the owning lanes
  float sq, cq;
  sincosf(r >= 3 ? q : 0.f, &sq, &cq);
  const float Tx = bcast<LPP>(q, 0), Ty = bcast<LPP>(q, 1), Tz = bcast<LPP>(q, 2);
  const float sa = bcast<LPP>(sq, 3), ca = bcast<LPP>(cq, 3);
  const float sb = bcast<LPP>(sq, 4), cb = bcast<LPP>(cq, 4);
  const float sg = bcast<LPP>(sq, 5), cg = bcast<LPP>(cq, 5);
  const int tsrc = bp_addr<LPP>(L.fdof >= 0 ? L.fdof : 0);
  const float st = bp(tsrc, sq), ct = bp(tsrc, cq);
  float* m = o.m;
  float* t = o.t;
  if (L.fparent < 0) {
    // root (and idle lanes): world rotation R = Rz Ry Rx about c0, which is
    // the origin of the stored coordinates, so the translation is T itself
    m[0] = ca * cb; m[1] = ca * sb * sg - sa * cg; m[2] = ca * sb * cg + sa * sg;
    m[3] = sa * cb; m[4] = sa * sb * sg + ca * cg; m[5] = sa * sb * cg - ca * sg;
    m[6] = -sb;     m[7] = cb * sg;                m[8] = cb * cg;
    t[0] = Tx;
    t[1] = Ty;
    t[2] = Tz;
  } else {
    // Rodrigues rotation about u through xb by theta: y -> B y + (xb - B xb)
    const float ux = L.fu[0], uy = L.fu[1], uz = L.fu[2], oc = 1.f - ct;
    m[0] = ct + ux * ux * oc;      m[1] = ux * uy * oc - uz * st; m[2] = ux * uz * oc + uy * st;
    m[3] = uy * ux * oc + uz * st; m[4] = ct + uy * uy * oc;      m[5] = uy * uz * oc - ux * st;
    m[6] = uz * ux * oc - uy * st; m[7] = uz * uy * oc + ux * st; m[8] = ct + uz * uz * oc;
    t[0] = L.fxb[0] - (m[0] * L.fxb[0] + m[1] * L.fxb[1] + m[2] * L.fxb[2]);
    t[1] = L.fxb[1] - (m[3] * L.fxb[0] + m[4] * L.fxb[1] + m[5] * L.fxb[2]);
    t[2] = L.fxb[2] - (m[6] * L.fxb[0] + m[7] * L.fxb[1] + m[8] * L.fxb[2]);
  }
  o.rg.Tx = Tx; o.rg.Ty = Ty; o.rg.Tz = Tz;
  o.rg.sa = sa; o.rg.ca = ca; o.rg.sb = sb; o.rg.cb = cb;
  return o;
}

// C = A o M for 3 x 4 rows (rotation | translation).
DK_INLINE void compose_rows(const float4& a0, const float4& a1, const float4& a2, const float4& m0,
                            const float4& m1, const float4& m2, float4& c0, float4& c1, float4& c2) {
  c0 = make_float4(a0.x * m0.x + a0.y * m1.x + a0.z * m2.x, a0.x * m0.y + a0.y * m1.y + a0.z * m2.y,
                   a0.x * m0.z + a0.y * m1.z + a0.z * m2.z, a0.x * m0.w + a0.y * m1.w + a0.z * m2.w + a0.w);
  c1 = make_float4(a1.x * m0.x + a1.y * m1.x + a1.z * m2.x, a1.x * m0.y + a1.y * m1.y + a1.z * m2.y,
                   a1.x * m0.z + a1.y * m1.z + a1.z * m2.z, a1.x * m0.w + a1.y * m1.w + a1.z * m2.w + a1.w);
  c2 = make_float4(a2.x * m0.x + a2.y * m1.x + a2.z * m2.x, a2.x * m0.y + a2.y * m1.y + a2.z * m2.y,
                   a2.x * m0.z + a2.y * m1.z + a2.z * m2.z, a2.x * m0.w + a2.y * m1.w + a2.z * m2.w + a2.w);
}

// Forward kinematics: world coordinates of the atoms owned by lane r.
// Fragment transforms are composed root-to-leaf by pointer jumping
// (ceil(log2) rounds of "compose with my current ancestor's transform").  The
// transforms live in LDS as three float4 rows per fragment (T4: 3 * LPP
// float4 of the group): each round reads the fragment's own and its
// ancestor's rows and writes the product back, so nothing is carried in
// registers from round to round.
template <int LPP, int APL>
DK_INLINE Rigid fk_place(const LaneLig<APL>& L, float q, int r, float (&x)[APL][3], float4* T4) {
  const LocalTf lt = fk_local<LPP, APL>(L, q, r);
  int anc = L.fparent;
  T4[r] = make_float4(lt.m[0], lt.m[1], lt.m[2], lt.t[0]);
  T4[LPP + r] = make_float4(lt.m[3], lt.m[4], lt.m[5], lt.t[1]);
  T4[2 * LPP + r] = make_float4(lt.m[6], lt.m[7], lt.m[8], lt.t[2]);
  for (int it = 0; it < L.fk_rounds; ++it) {
    wave_sync();
    const int src = anc >= 0 ? anc : r;
    const int anc2 = bp(bp_addr<LPP>(src), anc);
    const float4 a0 = T4[src], a1 = T4[LPP + src], a2 = T4[2 * LPP + src];
    const float4 m0 = T4[r], m1 = T4[LPP + r], m2 = T4[2 * LPP + r];
    wave_sync();
    if (anc >= 0) {
      float4 c0, c1, c2;
      compose_rows(a0, a1, a2, m0, m1, m2, c0, c1, c2);
      T4[r] = c0;
      T4[LPP + r] = c1;
      T4[2 * LPP + r] = c2;
      anc = anc2;
    }
  }
  wave_sync();
#pragma unroll
  for (int s = 0; s < APL; ++s) {
    const int f = L.afrag[s];
    const float4 r0 = T4[f], r1 = T4[LPP + f], r2 = T4[2 * LPP + f];
    x[s][0] = r0.x * L.ax[s] + r0.y * L.ay[s] + r0.z * L.az[s] + r0.w;
    x[s][1] = r1.x * L.ax[s] + r1.y * L.ay[s] + r1.z * L.az[s] + r1.w;
    x[s][2] = r2.x * L.ax[s] + r2.y * L.ay[s] + r2.z * L.az[s] + r2.w;
  }
  wave_sync();  // the rows are overwritten by the caller's coordinate slab
  return lt.rg;
}

// fk_place by cross-lane shuffles only (no LDS), for kernels without a slab.
template <int LPP, int APL>
DK_INLINE Rigid fk_place_shfl(const LaneLig<APL>& L, float q, int r, float (&x)[APL][3]) {
  LocalTf lt = fk_local<LPP, APL>(L, q, r);
  float* m = lt.m;
  float* t = lt.t;
  int anc = L.fparent;
  for (int it = 0; it < L.fk_rounds; ++it) {
    const int ad = bp_addr<LPP>(anc >= 0 ? anc : r);
    float a[9], b[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) a[k] = bp(ad, m[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) b[k] = bp(ad, t[k]);
    const int anc2 = bp(ad, anc);
    if (anc >= 0) {
      float nm[9], nt[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
          nm[3 * i + j] = a[3 * i] * m[j] + a[3 * i + 1] * m[3 + j] + a[3 * i + 2] * m[6 + j];
        nt[i] = a[3 * i] * t[0] + a[3 * i + 1] * t[1] + a[3 * i + 2] * t[2] + b[i];
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) m[k] = nm[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) t[k] = nt[k];
      anc = anc2;
    }
  }
#pragma unroll
  for (int s = 0; s < APL; ++s) {
    const int ad = bp_addr<LPP>(L.afrag[s]);
    float a[9], b[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) a[k] = bp(ad, m[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) b[k] = bp(ad, t[k]);
    x[s][0] = a[0] * L.ax[s] + a[1] * L.ay[s] + a[2] * L.az[s] + b[0];
    x[s][1] = a[3] * L.ax[s] + a[4] * L.ay[s] + a[5] * L.az[s] + b[1];
    x[s][2] = a[6] * L.ax[s] + a[7] * L.ay[s] + a[8] * L.az[s] + b[2];
  }
  return lt.rg;
}

// Chain rule from atom gradients g (world frame) to the DOF held by lane r:
//   dE/dT = sum g_i;  tau = sum (x_i - T) x g_i;
//   dE/d(alpha, beta, gamma) = tau . (e_z, Rz e_y, Rz Ry e_x);
//   dE/dtheta_k = u_k . sum_{i in subtree(k)} (x_i - x_{b_k}) x g_i.
// Subtree sums are differences of one inclusive prefix scan over the atoms
// (each torsion's subtree is a contiguous DFS range).  Reads the axis atoms'
// coordinates from the slab.
template <int LPP, int APL>
DK_INLINE float chain_rule(const LaneLig<APL>& L, const Rigid& rg, const float (&x)[APL][3],
                           const float (&g)[APL][3], const GroupSlab& S, int r) {
  const float Tx = rg.Tx, Ty = rg.Ty, Tz = rg.Tz;
  const float sa = rg.sa, ca = rg.ca, sb = rg.sb, cb = rg.cb;
  float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float vs[APL][6];
#pragma unroll
  for (int s = 0; s < APL; ++s) {
    const float rx = x[s][0] - Tx, ry = x[s][1] - Ty, rz = x[s][2] - Tz;
    vs[s][0] = g[s][0];
    vs[s][1] = g[s][1];
    vs[s][2] = g[s][2];
    vs[s][3] = ry * g[s][2] - rz * g[s][1];
    vs[s][4] = rz * g[s][0] - rx * g[s][2];
    vs[s][5] = rx * g[s][1] - ry * g[s][0];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = s == 0 ? vs[0][k] : v[k] + vs[s][k];
  }
  // inclusive scan over lanes (lane r covers atoms up to APL*r + APL - 1)
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = group_scan<LPP>(v[k]);
  // prefix at an atom boundary: P(end) = sum of atoms [0, end)
  // lane holding atoms [APL*l, APL*l+APL): inclusive value v; with APL = 2,
  // the partial up to its first atom is v - vs[1].
  float vlast[6];
  float vfirst[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    vlast[k] = v[k];
    vfirst[k] = APL == 2 ? v[k] - vs[APL - 1][k] : v[k];
  }
  auto prefix = [&](int end, float* out) {
    // all lanes call this with their own `end`; returns sum over [0, end)
    const int a = end - 1;
    const int ad = bp_addr<LPP>(a >= 0 ? a / APL : 0);
    const bool first = APL == 2 && (a % APL) == 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const float lv = bp(ad, vlast[k]);
      const float fv = APL == 2 ? bp(ad, vfirst[k]) : lv;
      out[k] = a < 0 ? 0.f : (first ? fv : lv);
    }
  };
  // rigid lanes need the total (prefix at n_atoms minus prefix at 0), torsion
  // lanes their subtree's range: one pair of prefix lookups serves both
  const bool rigid = r < 6;
  float pb[6], pe[6];
  prefix(rigid ? 0 : L.tsb, pb);
  prefix(rigid ? L.n_atoms : L.tse, pe);
  float Sg[3], St[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Sg[k] = pe[k] - pb[k];
    St[k] = pe[3 + k] - pb[3 + k];
  }
  // ---- gradient of this lane's DOF
  float gq = 0.f;
  if (r < 3) {
    gq = r == 0 ? Sg[0] : (r == 1 ? Sg[1] : Sg[2]);
  } else if (r == 3) {
    gq = St[2];
  } else if (r == 4) {
    gq = -sa * St[0] + ca * St[1];
  } else if (r == 5) {
    gq = ca * cb * St[0] + sa * cb * St[1] - sb * St[2];
  } else if (r < L.n_dof) {
    // axis atoms of this lane's torsion
    const f32x4_t xa = lds_read4(lds_addr(S.xs + L.ta)), xb = lds_read4(lds_addr(S.xs + L.tb));
    float ux = xb.x - xa.x, uy = xb.y - xa.y, uz = xb.z - xa.z;
    const float inv = __builtin_amdgcn_rsqf(ux * ux + uy * uy + uz * uz);
    ux *= inv; uy *= inv; uz *= inv;
    const float bx = xb.x - Tx, by = xb.y - Ty, bz = xb.z - Tz;
    // sum_sub (x_i - x_b) x g_i = St - r_b x Sg
    const float cx = St[0] - (by * Sg[2] - bz * Sg[1]);
    const float cy = St[1] - (bz * Sg[0] - bx * Sg[2]);
    const float cz = St[2] - (bx * Sg[1] - by * Sg[0]);
    gq = ux * cx + uy * cy + uz * cz;
  }
  return gq;
}

// Energy of one intra-ligand pair and the force f = (dE/dd / d) (x_i - x_j)
// to add to atom i (and subtract from atom j).
template <int APL>
DK_INLINE float pair_force(const LaneLig<APL>& L, const PairRec& pr, const float4& xi, const float4& xj,
                           float (&f)[3]) {
  const uint32_t flags = pr.w >> 24;
  const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
  const float d2 = dx * dx + dy * dy + dz * dz;
  // 1/d from the hardware reciprocal square root; d = d2 / d
  const float inv_d = d2 > 0.f ? __builtin_amdgcn_rsqf(d2) : 0.f;
  const float d = d2 * inv_d;
  float e, de;
  if (L.preset == DOCK_PRESET_TRIDS)
    trids_pair(d2, d, pr.rsum, flags, L.w, e, de);
  else
    vina_pair(d2, d, pr.rsum, flags, L.w, e, de);
  const float c = de * inv_d;
  f[0] = c * dx;
  f[1] = c * dy;
  f[2] = c * dz;
  return e;
}

// pair_force for a pass-layout slot: coordinates as read from the slab, the
// clash constants from the slot's second entry.
template <int APL>
DK_INLINE float pair_force_slot(const LaneLig<APL>& L, const uint4& rp, const f32x4_t& xi, const f32x4_t& xj,
                                float (&f)[3]) {
  const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
  const float d2 = dx * dx + dy * dy + dz * dz;
  // d2 = 0 (coincident atoms) gives d = 0 and a finite 1/d
  const float inv_d = __builtin_amdgcn_rsqf(fmaxf(d2, 1e-30f));
  const float d = d2 * inv_d;
  const float rsum = __uint_as_float(rp.y);
  float e, de;
  if (L.preset == DOCK_PRESET_TRIDS)
    trids_pair_k(d2, d, inv_d, rsum, __uint_as_float(rp.z), __uint_as_float(rp.w), L.w, e, de);
  else
    vina_pair(d2, d, rsum, rp.x >> 24, L.w, e, de);
  const float c = de * inv_d;
  f[0] = c * dx;
  f[1] = c * dy;
  f[2] = c * dz;
  return e;
}

// Pass-layout gather: each atom of the lane reads CAP force entries, the
// first CAP/2 added and the rest subtracted, all reads issued before the
// first sum.  The lane's pull bytes (APL * CAP of them) are packed in pw:
// CAP 8: x then y; CAP 4: atom s in word s; CAP 2: atom s in bytes 2s, 2s+1.
// `between` runs after the reads are issued and before the sums (the next
// pass's position reads go there, so their latency overlaps the sums).
template <int APL, int CAP, class Between>
DK_INLINE void gather_forces(const uint2& pw, uint32_t fb_a, float (&fsum)[APL][3], Between&& between) {
  uint32_t ad[APL][CAP];
#pragma unroll
  for (int s = 0; s < APL; ++s)
#pragma unroll
    for (int c = 0; c < CAP; ++c) {
      uint32_t word;
      int k;
      if (CAP == 8) {
        word = c < 4 ? pw.x : pw.y;
        k = c & 3;
      } else if (CAP == 4) {
        word = s == 0 ? pw.x : pw.y;
        k = c;
      } else {
        word = pw.x;
        k = 2 * s + c;
      }
      ad[s][c] = lds_entry16_k(word, k, fb_a);
    }
  // all addresses first: no VALU-to-LDS-address wait states between reads
  __builtin_amdgcn_sched_barrier(0);
  f32x4_t v[APL][CAP];
#pragma unroll
  for (int s = 0; s < APL; ++s)
#pragma unroll
    for (int c = 0; c < CAP; ++c) v[s][c] = lds_read4(ad[s][c]);
  between();
  // keeps the scheduler from pulling the sums up between the reads (each
  // would then wait for the read just issued)
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int s = 0; s < APL; ++s)
#pragma unroll
    for (int c = 0; c < CAP; ++c) {
      const float sg = c < CAP / 2 ? 1.f : -1.f;
      fsum[s][0] += sg * v[s][c].x;
      fsum[s][1] += sg * v[s][c].y;
      fsum[s][2] += sg * v[s][c].z;
    }
  // the unused 4th components stay live through the sums (their registers
  // would otherwise be reused there, each use waiting for its read)
#pragma unroll
  for (int s = 0; s < APL; ++s)
#pragma unroll
    for (int c = 0; c < CAP; ++c) asm volatile("" ::"v"(v[s][c].w));
}

// One evaluation of E and dE/dq at the pose whose DOF r is held by lane r.
// Optionally leaves world coordinates and atom gradients in xo/go; adds the
// E_MDN term when mdn.par is set.
// MODE: 0 receptor terms from the grid maps, 1 summed pair by pair over the
// receptor cell list, 2 grid maps plus the E_MDN term.
constexpr int kModeGrid = 0, kModeDirect = 1, kModeGridMdn = 2;

template <int LPP, int APL, bool WANT_X = false, int MODE = kModeGrid>
DK_INLINE EvalOut eval_pose(const LaneLig<APL>& Lin, float q, const PocketDev& pk,
                            const PairRec* __restrict__ pairs, const GroupSlab& S, int r,
                            float (*xo)[3] = nullptr, float (*go)[3] = nullptr,
                            const MdnArg& mdn = MdnArg{nullptr, 0, 0}) {
  LaneLig<APL> L = Lin;
  launder(L);
  // ---- atoms: place, interpolate, publish coordinates to the slab
  float x[APL][3], g[APL][3];
  const Rigid rg = fk_place<LPP, APL>(L, q, r, x, S.xs);
  float e_lane = 0.f;
#pragma unroll
  for (int s = 0; s < APL; ++s) {
    const int atom = APL * r + s;
    if (atom < L.n_atoms) {
      if (MODE == kModeDirect) {
        float ei;
        inter_direct(pk, L.preset, L.w, L.atype[s], x[s][0], x[s][1], x[s][2], ei, g[s][0], g[s][1],
                     g[s][2]);
        e_lane += ei;
      } else {
        const size_t nxyz = size_t(pk.grid.dims[0]) * pk.grid.dims[1] * pk.grid.dims[2];
        const Trilerp tl = trilerp(pk.M + size_t(L.atype[s]) * nxyz, pk.grid, x[s][0], x[s][1], x[s][2]);
        e_lane += tl.v + tl.eout;
        g[s][0] = tl.gx;
        g[s][1] = tl.gy;
        g[s][2] = tl.gz;
      }
      if (MODE == kModeGridMdn && mdn.par)
        mdn_term(pk, mdn, atom, x[s][0], x[s][1], x[s][2], e_lane, g[s][0], g[s][1], g[s][2]);
      S.xs[atom] = make_float4(x[s][0], x[s][1], x[s][2], 0.f);
    } else {
      g[s][0] = g[s][1] = g[s][2] = 0.f;
    }
  }
  wave_sync();
  float fsum[APL][3];
#pragma unroll
  for (int s = 0; s < APL; ++s) fsum[s][0] = fsum[s][1] = fsum[s][2] = 0.f;
  if (L.n_pass > 0 && L.pass_apl == APL && (APL == 1 || L.pass_w == LPP)) {
    // ---- pass layout: lane r evaluates slot r of every pass and stores the
    // force on its pair's first endpoint in entry r; then each atom adds the
    // entries named by the first half of its pull word and subtracts those
    // named by the second half (1 + 1, 2 + 2 or 4 + 4 entries; unused bytes
    // name the zero entry W).  Plain stores and a fixed summation order: the
    // result does not depend on timing.
    const int W = L.pass_w;
    const bool slot_lane = r < W;
    // pull bytes: APL * cap per lane and pass (4 or 8), the lane's atoms one
    // after the other.  Two consecutive dwords are always read (one
    // ds_read2_b32); with 4 bytes the second belongs to the next lane (or the
    // padding entry the host stages after the pull bytes) and is unused.
    const int cap = L.pull_cap;
    const uint32_t xs_a = lds_addr(S.xs), fb_a = lds_addr(S.fb);
    if (r == 0) {
      // a zero produced here, not a zero tuple kept live (and spilled)
      // across the sampler's loops
      float z = 0.f;
      asm volatile("" : "+v"(z));
      *(__attribute__((address_space(3))) f32x4_t*)(uintptr_t)(fb_a + 16u * uint32_t(W)) = f32x4_t{z, z, z, z};
    }
    // lanes without a slot hold no atom either: their gather is unused
    const uint32_t lane_slot = slot_lane ? uint32_t(r) : 0u;
    const uint32_t recs_a = lds_addr(pairs), pulls_a = recs_a + 16u * uint32_t(L.n_prec);
    // one loop per cap, so the gather's results stay in the same registers
    // from pass to pass
    auto run_passes = [&](auto cap_c) {
      constexpr int CAP = decltype(cap_c)::value;
      constexpr uint32_t kPullBytes = APL * CAP;
      // this lane's record and pull word of the next pass are read before
      // this pass's gather, and the record's two positions during it, so
      // that their latency overlaps the gather and the sums
      uint32_t rec_a = recs_a + 16u * lane_slot, pw_a = pulls_a + kPullBytes * lane_slot;
      const uint32_t rec_step = 16u * uint32_t(W), pw_step = kPullBytes * uint32_t(W);
      uint4 rp = lds_read_u4(rec_a);
      uint2 pw = lds_read_u2(pw_a);
      f32x4_t xi = lds_read4(lds_entry16<0>(rp.x, xs_a));
      f32x4_t xj = lds_read4(lds_entry16<1>(rp.x, xs_a));
      for (int ps = 0; ps < L.n_pass; ++ps) {
        // the unused 4th components stay live until here: otherwise their
        // registers are reused for the gather's sums, which must then wait
        // for these reads to land
        asm volatile("" ::"v"(xi.w), "v"(xj.w));
        float f[3];
        const float e = pair_force_slot(L, rp, xi, xj, f);
        if (slot_lane) {
          e_lane += e;
          lds_write4(fb_a + 16u * uint32_t(r), f[0], f[1], f[2]);
        }
        if (ps + 1 < L.n_pass) {
          rec_a += rec_step;
          pw_a += pw_step;
        }
        const uint4 rp_next = lds_read_u4(rec_a);
        const uint2 pw_next = lds_read_u2(pw_a);
        wave_sync();
        // every entry of the lane is read before any is summed
        gather_forces<APL, CAP>(pw, fb_a, fsum, [&] {
          const uint32_t ai = lds_entry16<0>(rp_next.x, xs_a), aj = lds_entry16<1>(rp_next.x, xs_a);
          xi = lds_read4(ai);
          xj = lds_read4(aj);
        });
        rp = rp_next;
        pw = pw_next;
        wave_sync();
      }
    };
    // caps: 4 or 8 with one atom per lane, 2 or 4 with two
    if (APL == 2 && cap == 2)
      run_passes(std::integral_constant<int, 2>{});
    else if (APL == 2 || cap == 4)
      run_passes(std::integral_constant<int, 4>{});
    else
      run_passes(std::integral_constant<int, 8>{});
  } else {
    // ---- strided: lane r takes records r, r + LPP, ...; forces by LDS atomics
#pragma unroll
    for (int s = 0; s < APL; ++s) {
      const int atom = APL * r + s;
      if (atom < L.n_atoms) {
        S.fx[atom] = 0.0;
        S.fy[atom] = 0.0;
        S.fz[atom] = 0.0;
      }
    }
    wave_sync();
    // a pass-layout ligand evaluated with two atoms per lane (a group sized
    // for a larger ligand of the same call) keeps its records at entry 2p
    const int pstep = L.n_pass > 0 ? 2 : 1;
    for (int p = r; p < L.n_prec; p += LPP) {
      const PairRec pr = pairs[pstep * p];
      if (pr.w & kPairEmpty) continue;
      const int i = pr.w & 0xff, j = (pr.w >> 8) & 0xff;
      float f[3];
      const f32x4_t xi = lds_read4(lds_addr(S.xs + i)), xj = lds_read4(lds_addr(S.xs + j));
      e_lane += pair_force(L, pr, make_float4(xi.x, xi.y, xi.z, 0.f), make_float4(xj.x, xj.y, xj.z, 0.f), f);
      if (f[0] != 0.f || f[1] != 0.f || f[2] != 0.f) {
        atomicAdd(&S.fx[i], double(f[0]));
        atomicAdd(&S.fy[i], double(f[1]));
        atomicAdd(&S.fz[i], double(f[2]));
        atomicAdd(&S.fx[j], -double(f[0]));
        atomicAdd(&S.fy[j], -double(f[1]));
        atomicAdd(&S.fz[j], -double(f[2]));
      }
    }
    wave_sync();
#pragma unroll
    for (int s = 0; s < APL; ++s) {
      const int atom = APL * r + s;
      if (atom < L.n_atoms) {
        fsum[s][0] = float(S.fx[atom]);
        fsum[s][1] = float(S.fy[atom]);
        fsum[s][2] = float(S.fz[atom]);
      }
    }
  }
  // ---- per-atom total gradient: add the intra-pair forces
#pragma unroll
  for (int s = 0; s < APL; ++s) {
    const int atom = APL * r + s;
    if (atom < L.n_atoms) {
      g[s][0] += fsum[s][0];
      g[s][1] += fsum[s][1];
      g[s][2] += fsum[s][2];
    }
    if (WANT_X) {
      xo[s][0] = x[s][0]; xo[s][1] = x[s][1]; xo[s][2] = x[s][2];
      go[s][0] = g[s][0]; go[s][1] = g[s][1]; go[s][2] = g[s][2];
    }
  }
  EvalOut out;
  out.E = group_sum<LPP>(e_lane);
  out.g = chain_rule<LPP, APL>(L, rg, x, g, S, r);
  wave_sync();  // slab reuse by the next evaluation
  return out;
}

// Differentiable form: the score over per-term maps G[t][k] with weights w
// (E = sum_k w_k (sum_i trilerp(G[t_i][k], x_i) + sum_pairs phi_k) + E_out),
// optionally scattering dL/dG for dL/dE = dLdE: into the float maps dLdG by
// float atomics, or (acc non-null) into 64-bit fixed-point accumulators, each
// corner weight rounded once to an integer multiple of 1 / acc_scale (a power
// of two; 0 marks a non-finite bound and drops the scatter).  Integer sums do
// not depend on the order of the atomics.  Intra-pair forces are summed in
// LDS as 64-bit fixed point scaled from a bound on the pair forces, which
// makes them independent of the atomics' order as well.  Atom positions
// come from FK of q (XIN = false) or are given (XIN = true).  Leaves
// per-atom gradients in g, per-term sums (reduced over the group) in ek, and
// returns E.
template <int LPP, int APL, int K, bool XIN>
DK_INLINE float eval_terms(const LaneLig<APL>& L, float q, float (&x)[APL][3], float (&g)[APL][3],
                           Rigid& rg, const float* __restrict__ G, const GridDev& grid,
                           const float (&w)[K], const PairRec* __restrict__ pairs, const GroupSlab& S,
                           int r, float dLdE, float* __restrict__ dLdG, float (&ek)[K],
                           unsigned long long* __restrict__ acc = nullptr, double acc_scale = 0.0) {
  if (!XIN) rg = fk_place<LPP, APL>(L, q, r, x, S.xs);
  const size_t nxyz = size_t(grid.dims[0]) * grid.dims[1] * grid.dims[2];
  const int nx = grid.dims[0], nxy = grid.dims[0] * grid.dims[1];
  float el[K];
#pragma unroll
  for (int k = 0; k < K; ++k) el[k] = 0.f;
  float eout = 0.f;
#pragma unroll
  for (int s = 0; s < APL; ++s) {
    const int atom = APL * r + s;
    g[s][0] = g[s][1] = g[s][2] = 0.f;
    if (atom < L.n_atoms) {
      const float* base = G + size_t(L.atype[s]) * K * nxyz;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const Trilerp tl = trilerp(base + size_t(k) * nxyz, grid, x[s][0], x[s][1], x[s][2]);
        el[k] += tl.v;
        if (k == 0) eout += tl.eout;  // the out-of-box penalty is the same for every term
        // trilerp() adds the out-of-box slope to its gradient; remove it from
        // every term and add it once below
        const float px = x[s][0], py = x[s][1], pz = x[s][2];
        const float sx = px > grid.hi[0] ? kOutK : (px < grid.origin[0] ? -kOutK : 0.f);
        const float sy = py > grid.hi[1] ? kOutK : (py < grid.origin[1] ? -kOutK : 0.f);
        const float sz = pz > grid.hi[2] ? kOutK : (pz < grid.origin[2] ? -kOutK : 0.f);
        g[s][0] += w[k] * (tl.gx - sx);
        g[s][1] += w[k] * (tl.gy - sy);
        g[s][2] += w[k] * (tl.gz - sz);
        if (k == K - 1) {
          g[s][0] += sx;
          g[s][1] += sy;
          g[s][2] += sz;
        }
        if (dLdG || acc) {
          const size_t off = size_t(L.atype[s] * K + k) * nxyz + tl.base;
          const float c = dLdE * w[k];
          const float fx = tl.fx, fy = tl.fy, fz = tl.fz;
          const float cv[8] = {c * (1.f - fx) * (1.f - fy) * (1.f - fz), c * fx * (1.f - fy) * (1.f - fz),
                               c * (1.f - fx) * fy * (1.f - fz),         c * fx * fy * (1.f - fz),
                               c * (1.f - fx) * (1.f - fy) * fz,         c * fx * (1.f - fy) * fz,
                               c * (1.f - fx) * fy * fz,                 c * fx * fy * fz};
          const size_t co[8] = {0, 1, size_t(nx), size_t(nx) + 1, size_t(nxy), size_t(nxy) + 1,
                                size_t(nxy) + nx, size_t(nxy) + nx + 1};
          if (acc) {
            if (acc_scale > 0.0) {
#pragma unroll
              for (int cn = 0; cn < 8; ++cn)
                atomicAdd(acc + off + co[cn],
                          static_cast<unsigned long long>(__double2ll_rn(double(cv[cn]) * acc_scale)));
            }
          } else {
#pragma unroll
            for (int cn = 0; cn < 8; ++cn) atomicAdd(dLdG + off + co[cn], cv[cn]);
          }
        }
      }
      S.xs[atom] = make_float4(x[s][0], x[s][1], x[s][2], 0.f);
      S.fx[atom] = 0.0;
      S.fy[atom] = 0.0;
      S.fz[atom] = 0.0;
    }
  }
  wave_sync();
  // The force slots (zeroed above as 0.0, i.e. integer 0) hold fixed-point
  // sums.  An atom takes at most 127 pair forces, each at most
  // sum_k |w_k| D_k in magnitude, with D_k >= max |d phi_k / dd| over
  // d >= 0.1 (below 0.1 the clash term is flat): TRIDS 1/sqrt(2e), 1/0.1,
  // 2 * 0.3/0.18 * e^-1/2; Vina sqrt(8) e^-1/2, 1/sqrt(2e), 2 * 3.8, 1,
  // 1/0.7, each rounded up.  The scale 2^(62 - e) with 127 sum_k |w_k| D_k
  // <= 2^e keeps every sum inside the signed 64-bit range.
  unsigned long long* fxi = reinterpret_cast<unsigned long long*>(S.fx);
  unsigned long long* fyi = reinterpret_cast<unsigned long long*>(S.fy);
  unsigned long long* fzi = reinterpret_cast<unsigned long long*>(S.fz);
  double force_fix = 0.0, force_unfix = 0.0;
  {
    constexpr float kD3[3] = {0.5f, 10.0f, 2.1f};
    constexpr float kD5[5] = {1.8f, 0.5f, 8.0f, 1.0f, 1.5f};
    double fb = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) fb += fabs(double(w[k])) * double(K == 3 ? kD3[k % 3] : kD5[k % 5]);
    if (fb < 1e300) {  // finite weights (else the intra forces drop out)
      int ex = 0;
      (void)frexp(127.0 * fb, &ex);
      force_fix = ldexp(1.0, 62 - ex);
      force_unfix = ldexp(1.0, ex - 62);
    }
  }
  const int pstep = L.n_pass > 0 ? 2 : 1;
  for (int p = r; p < L.n_prec; p += LPP) {
    const PairRec pr = pairs[pstep * p];
    if (pr.w & kPairEmpty) continue;
    const int i = pr.w & 0xff, j = (pr.w >> 8) & 0xff;
    const f32x4_t xi = lds_read4(lds_addr(S.xs + i)), xj = lds_read4(lds_addr(S.xs + j));
    const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
    const float d2 = dx * dx + dy * dy + dz * dz;
    const float d = sqrtf(d2);
    float v[K], dv[K];
    pair_terms_f32<K>(d2, d, pr.rsum, pr.w >> 24, v, dv);
    float de = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      el[k] += v[k];
      de += w[k] * dv[k];
    }
    if (de != 0.f && d > 0.f) {
      const float c = de / d;
      const long long ix = __double2ll_rn(double(c * dx) * force_fix),
                      iy = __double2ll_rn(double(c * dy) * force_fix),
                      iz = __double2ll_rn(double(c * dz) * force_fix);
      atomicAdd(&fxi[i], static_cast<unsigned long long>(ix));
      atomicAdd(&fyi[i], static_cast<unsigned long long>(iy));
      atomicAdd(&fzi[i], static_cast<unsigned long long>(iz));
      atomicAdd(&fxi[j], static_cast<unsigned long long>(-ix));
      atomicAdd(&fyi[j], static_cast<unsigned long long>(-iy));
      atomicAdd(&fzi[j], static_cast<unsigned long long>(-iz));
    }
  }
  wave_sync();
#pragma unroll
  for (int s = 0; s < APL; ++s) {
    const int atom = APL * r + s;
    if (atom < L.n_atoms) {
      g[s][0] += float(double(static_cast<long long>(fxi[atom])) * force_unfix);
      g[s][1] += float(double(static_cast<long long>(fyi[atom])) * force_unfix);
      g[s][2] += float(double(static_cast<long long>(fzi[atom])) * force_unfix);
    }
  }
  float E = group_sum<LPP>(eout);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    ek[k] = group_sum<LPP>(el[k]);
    E += w[k] * ek[k];
  }
  return E;
}

DK_INLINE float wrap_angle(float a) { return a - kTwoPi * floorf((a + kPi) * kInvTwoPi); }

}  // namespace dock
