// Internal header of the MI355X pair-cascade PIC library: the per-gap
// descriptor that lives in device memory, launch constants, and device
// helpers (Philox4x64-10 and Philox4x32-10, wave-level scans).  Not part of
// the C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"

// Push pipelining defaults (overridable at build time for tuning sweeps).
#ifndef PIC_PUSH_F_PREFETCH
#define PIC_PUSH_F_PREFETCH 1
#endif
#ifndef PIC_PUSH_F_EGROUP
#define PIC_PUSH_F_EGROUP 4
#endif
#ifndef PIC_PUSH_F_WAVES
#define PIC_PUSH_F_WAVES 4
#endif
#ifndef PIC_PUSH_D_PREFETCH
#define PIC_PUSH_D_PREFETCH 0
#endif
#ifndef PIC_PUSH_D_EGROUP
#define PIC_PUSH_D_EGROUP 4
#endif
#ifndef PIC_PUSH_D_WAVES
#define PIC_PUSH_D_WAVES 3
#endif

namespace pic {

constexpr int kBlock = 256;           // threads per workgroup (4 wave64)
constexpr int kItems = 4;             // particles per thread per work item
constexpr int kChunk = kBlock * kItems;
constexpr int kTile = 2048;           // cells of the per-workgroup LDS current tile
constexpr int kPhChunk = kBlock * 4;  // photons per convert work item
constexpr int kCellChunk = kBlock * 8;  // cells per work item of the field role (and the sorts' counts)
constexpr int kSortTile = 8192;       // buckets of the LDS histogram of the lepton sort
constexpr int kSortShift = 3;         // a lepton sort bucket is a group of 2^kSortShift cells
// lepton chunks per iteration of the lepton sort: counting holds only the
// cells, moving holds the whole lepton state
template <int PASS>
struct SortPer { static constexpr int value = PASS == 0 ? 4 : 2; };
constexpr int kPhUnroll = 4;          // photons per thread per iteration of the photon sort
constexpr int kTailEvery = 5;         // steps between sorts of the appended leptons
constexpr int kPhBins = 8192;         // conversion steps of the LDS histogram of the photon sort
constexpr int kFarKey = 255;          // tail key of a photon not due within 254 steps of the last sort
constexpr int kKeyRun = 16;           // tail keys a lane reads at once (one 16-byte load)
constexpr int kPhAgeMax = 160;        // photon sorts at most this many steps apart (with re-sorts
                                      // at most 80 steps apart, tail keys stay below kFarKey)

// Whether a particle re-sort at this state also sorts the photon store: once
// the tail has grown for the gap's age, or when the store is half full (the
// sort reclaims converted and escaped photons).
__host__ __device__ __forceinline__ bool photon_sort_due(int table_len, long long step,
                                                         long long ph_base, int age,
                                                         unsigned long long n_ph,
                                                         long long ph_cap) {
  return table_len > 0 && (step - ph_base >= age || 2 * (long long)n_ph >= ph_cap);
}
constexpr int32_t kDead = INT32_MIN;  // cell of an absorbed lepton until re-sort
constexpr int kMaxEmit = 64;
constexpr int kPushGrid = 4096;       // workgroups of the push kernel
// Push pipelining per particle type: whether the next chunk's lepton state
// is prefetched, how many items' E values are requested together, and the
// waves per SIMD asked of the compiler (4 means at most 128 VGPRs).
template <typename T>
struct PushCfg;
template <>
struct PushCfg<float> {
  static constexpr bool prefetch = PIC_PUSH_F_PREFETCH;
  static constexpr int e_group = PIC_PUSH_F_EGROUP;
  static constexpr int waves = PIC_PUSH_F_WAVES;
  // the per-lepton-threshold instantiations hold more state per item; at 128
  // VGPRs the compiler spilled some of it inside a divergent branch, where a
  // spill store writes only the active lanes and the others later reloaded
  // stale values, so they get 168 VGPRs (3 waves per SIMD) and spill nothing
  static constexpr int spread_waves = 3;
  static constexpr int spline_waves = PIC_PUSH_F_WAVES;
};
template <>
struct PushCfg<double> {
  static constexpr bool prefetch = PIC_PUSH_D_PREFETCH;
  static constexpr int e_group = PIC_PUSH_D_EGROUP;
  static constexpr int waves = PIC_PUSH_D_WAVES;
  // the binary64 spline and spread instantiations take the registers they need
  static constexpr int spread_waves = 1;
  static constexpr int spline_waves = 1;
};
constexpr int kStripes = 32;          // striped per-gap accumulators of the push kernel
constexpr int kStripeStride = 16;     // doubles between stripes (one 128-byte line each)
constexpr uint64_t kTagSeed = 1, kTagPhoton = 2, kTagThreshold = 3;

// One gap, in device memory.  The host fills the constant part at creation;
// kernels update the counters.  Particle and photon arrays are double
// buffered; `buf` selects the live copy and flips at each re-sort.
// A stored photon: its conversion point on the 2^-K grid and its child
// electron id with bit 0 = (direction > 0).  The two are read together when
// the photon converts, so they share one 16-byte record (one cache line per
// photon where due photons are sparse in the store).
struct __attribute__((aligned(16))) PhotonRec {
  long long x;
  uint64_t child;
};

struct GapDev {
  // ---- constants
  int32_t n_cells, boundary, K, table_len;
  int32_t precision, diag_every, hist_rows, shape;
  int64_t one, domain, photon_step, cap, ph_cap;
  int64_t slots;                     // lepton slots per species: cap plus the reserve that
                                     // absorbed leptons hold until the next re-sort
  double dt, dx, weight, wq, e0;
  double jmdt;                       // imposed current times dt (section 7), 0 elsewhere
  double sigma, gthr64, thr_lo;      // spread of gamma_thr, gamma_thr in binary64, lowest threshold
  double dtdx, gthr, gpair, pchild;  // values exactly representable in the particle type
  double gpair64, child_gamma64;     // binary64 pair energy; child gamma in the particle precision
  uint64_t seed;
  double* E;
  float* Ef;  // E rounded to binary32 (read by the binary32 push; same values as (float)E)
  long long* F;
  long long* F_last;
  long long* rho_acc;
  uint32_t* table;
  int32_t* sort_cnt[2];
  pic_history_row* hist;
  int32_t* cell[2][2];  // [buf][species]
  void* off[2][2];
  void* p[2][2];
  uint64_t* id[2][2];
  PhotonRec* ph_rec[2];   // position (2^-K grid) and child id with the direction, one record
  int32_t* ph_step[2];
  int32_t* ph_bucket;     // photon store sorted by conversion step: end of each bucket
  uint8_t* ph_key;        // per slot of the unsorted tail: conversion step - ph_base when
                          // below kFarKey, else kFarKey (escaped photons too)
  float inv_lnq;          // 1 / ln q of the photon path, q = exp(-dt / (l_gamma dx))
  int32_t ph_age;         // steps the photon tail may grow before a re-sort sorts the store
  unsigned long long* evmap;  // pair-event map (caller's device buffer), or null
  int32_t* emit_cnt;          // the batch's emitters per chunk (same in every gap)
  uint32_t* emit_ent;         // the batch's emitter lists, kChunk entries per chunk
  uint32_t* wg_emit;          // the batch's emitters per push workgroup
  long long emit_split;       // steps whose plan holds fewer lepton chunks emit in the push
  float conv_c;               // ln 2 l_gamma dx / dt (the photon path in steps per unit of
                              // -log2 of the survival probability)
  int32_t pad6;
  int32_t ev_x, ev_steps, ev_rows, pad5;

  // ---- counters (device-updated)
  unsigned long long n[2];       // slots in use at step start
  unsigned long long pair_next;  // pairs appended this step: both species grow by the same
                                 // count, electron j at n[0] + j and positron j at n[1] + j
  unsigned long long esc_next;   // photons that left the domain this step
  unsigned long long dead[2];    // absorbed slots since the last re-sort
  unsigned long long live[2];    // live leptons after the last completed step
  unsigned long long n_ph, n_ph_next, inflight;  // photon slots at step start, append cursor
  unsigned long long pairs_created, photons_emitted, photons_escaped, absorbed[2];
  unsigned long long pushes;
  unsigned long long push_emitted;  // emissions drawn inside the push kernel (cumulative)
  unsigned long long hist_count;
  // order-independent sums of the step, cleared by the finalize: the sum of
  // the Lorentz factors of the leptons pushed this step and of those
  // absorbed (fix64, four limbs), and the field energy and the positive and
  // negative parts of the sum of E (wide_add, kWideLimbs limbs)
  unsigned long long ke_limb[4], lost_limb[4];
  unsigned long long fe_wide[8], esp_wide[8], esn_wide[8];
  // their values, written by the first phase of the finalize
  double ke_step, lost_step, fe_step, es_step;
  unsigned long long sorted_n[2], ph_sorted;
  unsigned long long body_n[2];  // leptons sorted by the last full re-sort (the rest were appended since)
  unsigned long long ph_body_n;  // photons in the sorted body of the store
  long long ph_base;             // conversion step of bucket 0 of the sorted body
  long long step;
  int32_t status, buf, phbuf;
  int32_t ph_due;                // the current re-sort also sorts the photon store
  int32_t overflow, nonfinite, emit_err, slot_overflow;
  double lost_energy;  // cumulative, a binary64 sum over steps in step order
  pic_history_row last;
};

// Pointers loaded from a descriptor are generic to the compiler; casting
// them to the global address space lets it emit global (not flat) memory
// instructions.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> glb(T* p) { return (gptr<T>)p; }
template <class T>
__device__ __forceinline__ gptr<T> glb(void* p) { return (gptr<T>)(T*)p; }

// Photon records moved as one 16-byte vector (one load or store instruction).
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void put_photon(gptr<PhotonRec> a, long long i, long long x,
                                           uint64_t child) {
  *(gptr<u64x2>)(a + i) = u64x2{(unsigned long long)x, child};
}
__device__ __forceinline__ u64x2 get_photon(gptr<const PhotonRec> a, long long i) {
  return *(gptr<const u64x2>)(a + i);
}

__device__ __forceinline__ void gadd(gptr<unsigned long long> p, unsigned long long v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Fixed-point offset arithmetic: 2^-24 offsets fit 32-bit integers, 2^-40
// offsets need 64 bits.
template <typename T>
struct Fixed;
template <>
struct Fixed<float> { using I = int; };
template <>
struct Fixed<double> { using I = long long; };

// ---------------------------------------------------------------- Philox
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies with a key schedule bumped by the Weyl constants.
struct U64x4 { uint64_t v[4]; };

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                               uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  // rounds kept as a loop: unrolled, the scheduler interleaves them and
  // holds far more registers than one round needs
#pragma unroll 1
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  U64x4 o;
  o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// Philox4x32-10 (same paper): the 32-bit form, two 32x32 -> 64-bit products
// per round.  The draws of the run use it: lepton `id`'s draw with tag t at
// step n and index j has counter (n, j | t << 8, id low, id high) and key
// (seed low, seed high); words 1:0 form a 64-bit value, word 2 a 32-bit one.
struct RunDraw { uint64_t bits; uint32_t u32; };

__device__ __forceinline__ RunDraw draw_run(uint64_t id, uint64_t seed, uint32_t step, uint32_t j,
                                            uint32_t tag) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = step, c1 = j | (tag << 8), c2 = (uint32_t)id, c3 = (uint32_t)(id >> 32);
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll 1
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    const uint64_t a = (uint64_t)M0 * c0, b = (uint64_t)M1 * c2;
    const uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0, n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)b;
    c3 = (uint32_t)a;
    c0 = n0;
    c2 = n2;
  }
  RunDraw d;
  d.bits = ((uint64_t)c1 << 32) | c0;
  d.u32 = c2;
  return d;
}

// Two independent draws at once (two leptons' or emissions' counters under
// one key), their rounds interleaved so that each hides the other's
// multiply latency; the same values as two draw_run calls.
__device__ __forceinline__ void draw_run2(uint64_t ida, uint64_t idb, uint64_t seed, uint32_t step,
                                          uint32_t ja, uint32_t jb, uint32_t tag, RunDraw& da,
                                          RunDraw& db) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t a0 = step, a1 = ja | (tag << 8), a2 = (uint32_t)ida, a3 = (uint32_t)(ida >> 32);
  uint32_t b0 = step, b1 = jb | (tag << 8), b2 = (uint32_t)idb, b3 = (uint32_t)(idb >> 32);
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll 1
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    const uint64_t pa = (uint64_t)M0 * a0, qa = (uint64_t)M1 * a2;
    const uint64_t pb = (uint64_t)M0 * b0, qb = (uint64_t)M1 * b2;
    const uint32_t na0 = (uint32_t)(qa >> 32) ^ a1 ^ k0, na2 = (uint32_t)(pa >> 32) ^ a3 ^ k1;
    const uint32_t nb0 = (uint32_t)(qb >> 32) ^ b1 ^ k0, nb2 = (uint32_t)(pb >> 32) ^ b3 ^ k1;
    a1 = (uint32_t)qa; a3 = (uint32_t)pa; a0 = na0; a2 = na2;
    b1 = (uint32_t)qb; b3 = (uint32_t)pb; b0 = nb0; b2 = nb2;
  }
  da.bits = ((uint64_t)a1 << 32) | a0;
  da.u32 = a2;
  db.bits = ((uint64_t)b1 << 32) | b0;
  db.u32 = b2;
}

// Emission threshold of lepton `id` under a spread sigma of gamma_thr, a fixed
// property of the lepton, uniform in gamma_thr (1 - sigma, 1 + sigma): the top
// 53 bits of the 64-bit value of its tag-3 draw as a fraction u, then
// gamma_thr (1 + sigma (2u - 1)) in binary64 with one rounding per operation,
// rounded to the particle precision.
template <typename T>
__device__ __forceinline__ T lepton_threshold(uint64_t id, uint64_t seed, double gthr64,
                                              double sigma) {
  const RunDraw u = draw_run(id, seed, 0, 0, (uint32_t)kTagThreshold);
  const double x = (double)(u.bits >> 11) * 0x1p-53;
  const double a = 2.0 * x - 1.0;
  return (T)(gthr64 * (1.0 + sigma * a));
}

// Pair-event map: pairs made at step n in cell c count in row
// (n / ev_steps) % ev_rows, column c * ev_x / n_cells.
__device__ __forceinline__ void count_pairs(const GapDev* G, long long step, int c, unsigned long long k) {
  const long long row = (step / G->ev_steps) % G->ev_rows;
  const long long col = (long long)c * G->ev_x / G->n_cells;
  atomicAdd(G->evmap + row * G->ev_x + col, k);
}

// Accumulator a (0 kinetic energy, 1 lost energy: four limbs each; 2-3
// absorbed electrons / positrons) of gap g, stripe st: each stripe on its own
// cache line, so the workgroups of the push kernel do not all hit one address.
__device__ __forceinline__ unsigned long long* stripe_slot(unsigned long long* stripes, int g, int a,
                                                           int st) {
  return stripes + (((size_t)g * 4 + a) * kStripes + st) * kStripeStride;
}

// ------------------------------------------------- order-independent sums
// A binary64 diagnostic summed over leptons or cells must not depend on the
// order in which threads, workgroups or atomics visit them (leptons change
// slots at every re-sort).  Two exact integer accumulations serve:
//  - Lorentz factors (each at least 1; the uniform weight is applied to the
//    total): each term is rounded once, toward zero, onto the fixed grid
//    2^-64 as a signed 128-bit integer (below 2^63), summed in registers and
//    then as four 32-bit limbs added to 64-bit accumulators with integer
//    atomics, which commute;
//  - field sums, whose terms can be arbitrarily small (a screened or
//    equilibrium field): each workgroup's partial sum over its cells, taken in
//    a fixed order, is added exactly to a 256-bit accumulator on the grid
//    2^-192 (wide_add; magnitudes below 2^-192 vanish, which is far below any
//    field the diagnostics resolve).
// The value of accumulated limbs is the exact sum of the rounded terms,
// converted to binary64 by a fixed sequence of roundings.
__device__ __forceinline__ __int128 fix64(double t) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(t);
  const int e = (int)((bits >> 52) & 0x7FF);
  if (e == 0 || e == 0x7FF) return 0;  // zero, subnormal (far below 2^-64), or not finite
  const unsigned long long m = (bits & 0xFFFFFFFFFFFFFull) | (1ull << 52);
  const int sh = e - 1075 + 64;        // t = m 2^(e - 1075); the grid unit is 2^-64
  __int128 v;
  if (sh >= 0) v = (__int128)m << (sh < 74 ? sh : 74);
  else v = sh > -53 ? (__int128)(m >> -sh) : (__int128)0;
  return (bits >> 63) ? -v : v;
}

// Sum of a 128-bit integer over the 64 lanes of a wave (every lane gets it).
__device__ __forceinline__ __int128 wave_sum128(__int128 x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const unsigned long long lo = (unsigned long long)x, hi = (unsigned long long)(x >> 64);
    const unsigned long long ol = __shfl_xor(lo, d, 64), oh = __shfl_xor(hi, d, 64);
    x += (__int128)(((unsigned __int128)oh << 64) | ol);
  }
  return x;
}

// Adds a 128-bit integer to four limb accumulators (two's complement limbs;
// the sum is taken modulo 2^128 when read, which is exact for any true sum
// below 2^127 in magnitude).
__device__ __forceinline__ void limbs_add(unsigned long long* acc, __int128 v) {
  if (v == 0) return;
  const unsigned __int128 u = (unsigned __int128)v;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const unsigned long long l = (unsigned long long)(u >> (32 * k)) & 0xFFFFFFFFull;
    if (l) __hip_atomic_fetch_add(acc + k, l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

constexpr int kWideLimbs = 8;   // 256 bits
constexpr int kWideLow = 192;   // grid 2^-192

// Adds |t| (finite, below 2^63) on the grid 2^-192 to kWideLimbs limb
// accumulators: the 53-bit significand lands in at most three 32-bit limbs.
__device__ __forceinline__ void wide_add(unsigned long long* acc, double t) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(t);
  const int e = (int)((bits >> 52) & 0x7FF);
  if (e == 0 || e == 0x7FF) return;
  unsigned long long m = (bits & 0xFFFFFFFFFFFFFull) | (1ull << 52);
  int pos = e - 1075 + kWideLow;  // bit index of the significand's lowest bit
  if (pos < 0) {
    if (pos <= -53) return;
    m >>= -pos;
    pos = 0;
  }
  const int k = pos >> 5;
  const unsigned __int128 v = (unsigned __int128)m << (pos & 31);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const unsigned long long l = (unsigned long long)(v >> (32 * q)) & 0xFFFFFFFFull;
    if (l && k + q < kWideLimbs)
      __hip_atomic_fetch_add(acc + k + q, l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Value of kWideLimbs limb accumulators.  Limb k holds h_k 2^32 + l_k, so
// position j (weight 2^(32 j - 192)) collects l_j + h_(j-1), below 2^33 and
// exact in binary64; the positions are summed from the most significant
// down, a fixed sequence of roundings.
__device__ __forceinline__ double wide_value(const unsigned long long* acc) {
  double v = 0.0;
#pragma unroll
  for (int j = kWideLimbs; j >= 0; --j) {
    const unsigned long long lo = j < kWideLimbs ? (acc[j] & 0xFFFFFFFFull) : 0ull;
    const unsigned long long hi = j > 0 ? (acc[j - 1] >> 32) : 0ull;
    v += ldexp((double)(lo + hi), 32 * j - kWideLow);
  }
  return v;
}

// Value of four limb accumulators: the 128-bit sum times 2^-64.
__device__ __forceinline__ double limbs_value(const unsigned long long* acc) {
  unsigned __int128 s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += (unsigned __int128)acc[k] << (32 * k);
  const __int128 v = (__int128)s;
  const long long hi = (long long)(v >> 64);
  const unsigned long long lo = (unsigned long long)v;
  return ((double)hi * 0x1p64 + (double)lo) * 0x1p-64;
}

// ---------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Inclusive prefix sum over the 64 lanes of a wave.
template <typename I>
__device__ __forceinline__ I wave_incl_scan(I x) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    I y = __shfl_up(x, d, 64);
    if (l >= d) x += y;
  }
  return x;
}

// Inclusive prefix sum of ints over the 64 lanes of a wave with DPP moves
// (rows of 16 lanes by shifts of 1, 2, 4 and 8, then the row totals
// broadcast to the rows above): no lane masks or shuffle addresses, which a
// caller's loop would otherwise keep in registers throughout.
__device__ __forceinline__ int wave_incl_scan_dpp(int x) {
  // dpp_ctrl row_shr:n = 0x110 + n; lanes shifted in from below the row read 0
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);
  // row_bcast:15 (0x142) adds lane 15's total to row 1 and lane 47's to row 3;
  // row_bcast:31 (0x143) adds lane 31's to rows 2 and 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);
  return x;
}

template <typename V>
__device__ __forceinline__ V wave_sum(V x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Locate the gap owning work item w: largest g with start[g] <= w.
__device__ __forceinline__ int find_gap(const long long* __restrict__ start, int B, long long w) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= w) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Contiguous share of `total` work items for each workgroup.  Workgroups
// reach the 8 XCDs round-robin (workgroup b runs on XCD b % 8), so the items
// are first cut into 8 consecutive eighths, one per XCD, and each XCD's
// workgroups split its eighth: the field lines of an XCD's cells stay in its
// own L2, and every XCD has work however few items there are.  The logical
// index of workgroup b (xcd_logical) orders the shares by item: share lb
// starts where share lb - 1 ends.
__device__ __forceinline__ int xcd_logical(int b, int nb) {
  return (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
}

// Items [w0, w1) of logical share lb of nb.
__device__ __forceinline__ void share_range(long long total, int lb, int nb, long long& w0,
                                            long long& w1) {
  if ((nb & 7) != 0) {
    const long long per = (total + nb - 1) / nb;
    w0 = (long long)lb * per;
    w0 = w0 < total ? w0 : total;
    w1 = w0 + per < total ? w0 + per : total;
    return;
  }
  const int x = lb / (nb >> 3), r = lb % (nb >> 3);
  const long long t0 = total * x / 8, t1 = total * (x + 1) / 8;
  const long long per = (t1 - t0 + (nb >> 3) - 1) / (nb >> 3);
  w0 = t0 + (long long)r * per;
  w0 = w0 < t1 ? w0 : t1;
  w1 = w0 + per < t1 ? w0 + per : t1;
}

__device__ __forceinline__ void xcd_range(long long total, long long& w0, long long& w1,
                                          int b, int nb) {
  share_range(total, xcd_logical(b, nb), nb, w0, w1);
}

__device__ __forceinline__ void xcd_range(long long total, long long& w0, long long& w1) {
  xcd_range(total, w0, w1, (int)blockIdx.x, (int)gridDim.x);
}

}  // namespace pic
