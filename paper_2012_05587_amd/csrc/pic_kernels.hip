// HIP kernels (gfx950) of the pair-cascade PIC step.
//
// One step of a gap (arXiv:2012.05587, sections 2-3):
//   k_push     gather E at each lepton, relativistic push, move with an exact
//              integer charge-conserving flux (per-workgroup LDS tile reduced
//              into the global int64 grid), absorb/wrap, and the threshold
//              test: the emitter loses k * gamma_pair; in small steps each
//              chunk's emitters then draw their photons (or in-place pairs)
//              from Philox and append them, in large steps they are listed
//              for k_post; instantiated with the linear or quadratic-spline
//              shape and with or without per-lepton thresholds;
//   k_post     four roles on disjoint block ranges of one launch: Ampere's
//              law E -= w 2^-K F (Eq. 4 in normalised units; plus j_m dt in
//              the co-rotating frame) with the field diagnostics; the listed
//              emitters' photons, balanced by emitter; photons due this step
//              become pairs; the striped push tallies are folded;
//   k_finalize counters, history row and the work items of the next step,
//              one gap per wave; k_plan_scan their prefixes (one block).
// Every S steps the leptons are re-sorted by cell group (8 cells) and the
// photon store by conversion step (counting sorts), which drops absorbed
// leptons and converted photons.
//
// All kernels take the gaps of a batch at once: work items are chunks of
// particles, photons or cells, numbered across gaps by prefix arrays that
// the device itself maintains, so a sequence of steps needs no host
// synchronisation and can be captured in a graph.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "pic_device.hpp"
#include "pic_kernels.hpp"

namespace pic {

__device__ __forceinline__ unsigned long long as_u64(long long v) { return (unsigned long long)v; }

// n_conv = min{k >= 1 : u >= T_k} over the decreasing integer table T
// (T_{len-1} = 0).  T_k ~ q^k 2^32, so k ~ ln(u 2^-32) / ln q; the estimate
// only picks where to look: the answer is decided by the table entries.
__device__ __forceinline__ int conv_estimate(int len, uint32_t u, float inv_lnq) {
  int k;
  if (u == 0u) {
    k = len - 1;
  } else {
    const float est = __logf((float)u * 2.3283064365386963e-10f) * inv_lnq;
    k = (int)ceilf(est);
  }
  return k < 1 ? 1 : (k > len - 1 ? len - 1 : k);
}

// The answer from the estimate k and the entries T_{k-1}, T_k, T_{k+1}
// around it (clamped to the table), which the caller requested together.
__device__ __forceinline__ int conv_decide(const uint32_t* __restrict__ table, int len, uint32_t u,
                                          int k, uint32_t tm, uint32_t t0, uint32_t tp) {
  int lo = 1, hi = len - 1;
  if (u >= t0) {
    if (k == 1 || u < tm) return k;
    hi = k - 1;  // the answer lies below k - 1 + 1
  } else {
    if (k + 1 <= len - 1 && u >= tp) return k + 1;
    lo = k + 1 < len - 1 ? k + 1 : len - 1;
  }
  // bisection over the rest (not reached for tables built by the runtime)
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (u >= table[mid]) hi = mid; else lo = mid + 1;
  }
  return lo;
}

__device__ __forceinline__ int conv_steps(const uint32_t* __restrict__ table, int len, uint32_t u,
                                         float inv_lnq) {
  const int k = conv_estimate(len, u, inv_lnq);
  // the estimate is within a step of the answer: the entries around it are
  // requested together (T_{len-1} = 0, so some k answers)
  gptr<const uint32_t> tab = glb<const uint32_t>((void*)table);
  const uint32_t tm = tab[k - 1 > 0 ? k - 1 : 0], t0 = tab[k];
  const uint32_t tp = tab[k + 1 < len ? k + 1 : len - 1];
  return conv_decide(table, len, u, k, tm, t0, tp);
}

// n_conv without the table where the answer is clear.  T_k = floor(V_k) with
// V_k = 2^32 q^k as the host evaluates it, so for an integer u, u >= T_k
// exactly when V_k < u + 1, that is when k exceeds
// x = (32 - log2(u + 1)) ln 2 / r (q = e^-r), and n_conv = floor(x) + 1.  In
// binary32, u + 1 is rounded once (relative 2^-24), log2f is within one ulp
// (4e-6 for results below 32), 32 - log2 is rounded once more (2e-6) and the
// product with c = ln 2 / r, itself rounded, twice (1.2e-7 relative); the
// host's V_k is within 3e-15 relative.  So x is off by less than
// 6.1e-6 c + 1.3e-7 x, and tol = 2e-5 c + 5e-7 x + 1e-6 covers that three
// times over: wherever x lies farther than tol from an integer the rule gives
// the table's answer.  Near an integer, or at the table's end, the table
// decides.
__device__ __forceinline__ int conv_steps_direct(const uint32_t* __restrict__ table, int len,
                                                 uint32_t u, float c, float inv_lnq) {
  const float x = (32.0f - log2f((float)((uint64_t)u + 1u))) * c;
  const float fl = floorf(x), fr = x - fl;
  const float tol = 2e-5f * c + 5e-7f * x + 1e-6f;
  if (fr > tol && fr < 1.0f - tol && fl + 1.0f < (float)len) return (int)fl + 1;
  return conv_steps(table, len, u, inv_lnq);
}

// X modulo the domain length D, in [0, D), for |X| < 2^62 and D >= 2^24
// (a photon's conversion point in a periodic gap): the quotient taken in
// binary64 is within one of the true floor (its magnitude is below 2^38, so
// its rounding error is far below one), and the remainder is then brought
// into range exactly in integers.
__device__ __forceinline__ long long wrap_periodic(long long X, long long D) {
  const long long q = (long long)floor((double)X / (double)D);
  X -= q * D;
  if (X < 0) X += D;
  else if (X >= D) X -= D;
  return X;
}

// Block-wide min and max of ints; every thread gets the result.
__device__ __forceinline__ void block_minmax(int& mn, int& mx, int* s_red) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    mn = min(mn, __shfl_xor(mn, d, 64));
    mx = max(mx, __shfl_xor(mx, d, 64));
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (lane_id() == 0) { s_red[w] = mn; s_red[4 + w] = mx; }
  __syncthreads();
  mn = min(min(s_red[0], s_red[1]), min(s_red[2], s_red[3]));
  mx = max(max(s_red[4], s_red[5]), max(s_red[6], s_red[7]));
}

// Block-wide min and max of ints for a loop that calls it once per
// iteration: the scratch is double-buffered by iteration parity, so only
// one barrier is needed (the one between two uses of a buffer is the
// barrier of the call in between).
__device__ __forceinline__ void block_minmax_pp(int& mn, int& mx, int (*s_red)[8], int& parity) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    mn = min(mn, __shfl_xor(mn, d, 64));
    mx = max(mx, __shfl_xor(mx, d, 64));
  }
  int* r = s_red[parity];
  parity ^= 1;
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) { r[w] = mn; r[4 + w] = mx; }
  __syncthreads();
  mn = min(min(r[0], r[1]), min(r[2], r[3]));
  mx = max(max(r[4], r[5]), max(r[6], r[7]));
}

// Pairs of a step share one slot cursor: the workgroup reserves `tot` pairs
// (electron slots from n[0], positron slots from n[1]).  Appends beyond the
// slots are not written and freeze the gap; the capacity itself (live
// leptons) is checked by the finalize.
__device__ __forceinline__ unsigned long long reserve_pairs(GapDev* G, unsigned long long tot) {
  const unsigned long long b = atomicAdd(&G->pair_next, tot);
  const unsigned long long slots = (unsigned long long)G->slots;
  if (G->n[0] + b + tot > slots || G->n[1] + b + tot > slots) G->slot_overflow = 1;
  return b;
}

// Block-wide exclusive prefix sum of ints (256 threads); `total` gets the sum.
__device__ __forceinline__ int block_excl_scan(int x, int* s_tmp, int& total) {
  const int incl = wave_incl_scan_dpp(x);
  // the wave's index, uniform: its LDS slot and the compares below are scalar
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  __syncthreads();
  if (lane_id() == 63) s_tmp[w] = incl;
  __syncthreads();
  int off = 0, t = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; ++k) {
    const int v = s_tmp[k];
    if (k < w) off += v;
    t += v;
  }
  total = t;
  return off + incl - x;
}

// ------------------------------------------------------------------ emit
// Where a step's emission runs depends on its size.  A step whose plan holds
// fewer than kEmitInPushChunks lepton chunks emits inside the push, right
// after each chunk (emit_chunk): there the emission role's own chain of
// dependent loads would dominate the step.  A larger step lists each
// chunk's emitters (chunk-local index << 8 | k) in the chunk's slice of
// emit_ent, with their count in emit_cnt and each push workgroup's total in
// wg_emit, and the emission role of k_post draws them, balanced by emitters
// across its workgroups: there a per-chunk emission phase would put its
// round trips into the push's streaming loop for every one of ~1e5 chunks.
// The split (emit_split, the same in every descriptor) is set by the host.

// What the emission of one gap needs, read from its descriptor once per gap
// segment of a wave.
template <typename T>
struct EmitGap {
  GapDev* G;
  gptr<int32_t> cell[2];
  gptr<T> off[2], p[2];
  gptr<uint64_t> id[2];
  gptr<PhotonRec> phr;
  gptr<int32_t> phs;
  gptr<uint8_t> phk;
  const uint32_t* table;
  int table_len, K;
  float inv_lnq, conv_c;
  long long domain, photon_step, ph_base;
  unsigned long long ph_cap, slots, n0, n1;
  uint32_t step;
  uint64_t seed;
  T pchild, inv_scale, scale;
  bool absorbing, in_place, evmap;
};

template <typename T>
__device__ __forceinline__ EmitGap<T> emit_gap(GapDev* __restrict__ G) {
  EmitGap<T> E;
  E.G = G;
  const int buf = G->buf, pb = G->phbuf;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    E.cell[s] = glb(G->cell[buf][s]);
    E.off[s] = glb<T>(G->off[buf][s]);
    E.p[s] = glb<T>(G->p[buf][s]);
    E.id[s] = glb(G->id[buf][s]);
  }
  E.phr = glb(G->ph_rec[pb]);
  E.phs = glb(G->ph_step[pb]);
  E.phk = glb(G->ph_key);
  E.ph_base = G->ph_base;
  E.table = G->table;
  E.table_len = G->table_len;
  E.K = G->K;
  E.inv_lnq = G->inv_lnq;
  E.conv_c = G->conv_c;
  E.domain = G->domain;
  E.photon_step = G->photon_step;
  E.ph_cap = (unsigned long long)G->ph_cap;
  E.slots = (unsigned long long)G->slots;
  E.n0 = G->n[0];
  E.n1 = G->n[1];
  E.step = (uint32_t)G->step;
  E.seed = G->seed;
  E.pchild = (T)G->pchild;
  E.scale = (T)(double)G->one;
  E.inv_scale = (T)(1.0 / (double)G->one);
  E.absorbing = G->boundary == PIC_BC_ABSORBING;
  E.in_place = G->table_len == 0;
  E.evmap = G->evmap != nullptr;
  return E;
}

// The k photons (or in-place pairs) of listed emitter i of species s, from
// its stored state after the push (position, the momentum's sign for the
// direction, id), written at slots slot0 .. slot0 + k - 1 (pair slots
// n[0] + slot, n[1] + slot).  Emission j of an emitter at step n is its
// tag-2 draw (draw_run): the child electron id is the 64-bit value with bit
// 0 cleared (the positron's has it set), and the photon's path in steps,
// n_conv = min{k >= 1 : u >= T_k} for u the 32-bit value, comes from the
// gap's conversion table.  Returns the number of photons that left the
// domain.
template <typename T>
__device__ __forceinline__ unsigned emit_listed(const EmitGap<T>& E, int s, long long i, int k,
                                                unsigned long long slot0) {
  const gptr<int32_t> cA = s == 0 ? E.cell[0] : E.cell[1];
  const gptr<T> oA = s == 0 ? E.off[0] : E.off[1];
  const gptr<T> pA = s == 0 ? E.p[0] : E.p[1];
  const gptr<uint64_t> iA = s == 0 ? E.id[0] : E.id[1];
  const int c = cA[i];
  const long long oq = (long long)(oA[i] * E.scale);
  const T pv = pA[i];
  const uint64_t id = iA[i];
  const int dir = signbit(pv) ? -1 : 1;
  unsigned esc = 0;
  if (E.in_place) {
    const T pc = dir > 0 ? E.pchild : -E.pchild;
    const T offn = (T)oq * E.inv_scale;
    for (int jj = 0; jj < k; ++jj) {
      const RunDraw u = draw_run(id, E.seed, E.step, (uint32_t)jj, (uint32_t)kTagPhoton);
      const uint64_t child = u.bits & ~(uint64_t)1;
      const unsigned long long se = E.n0 + slot0 + jj, sp = E.n1 + slot0 + jj;
      if (se < E.slots) { E.cell[0][se] = c; E.off[0][se] = offn; E.p[0][se] = pc; E.id[0][se] = child; }
      if (sp < E.slots) {
        E.cell[1][sp] = c; E.off[1][sp] = offn; E.p[1][sp] = pc; E.id[1][sp] = child | 1u;
      }
    }
    if (E.evmap) count_pairs(E.G, (long long)E.step, c, (unsigned long long)k);
    return 0;
  }
  const long long X0 = ((long long)c << E.K) + oq;
  for (int jj = 0; jj < k; ++jj) {
    const RunDraw u = draw_run(id, E.seed, E.step, (uint32_t)jj, (uint32_t)kTagPhoton);
    const uint64_t child = u.bits & ~(uint64_t)1;
    const int ncv = conv_steps_direct(E.table, E.table_len, u.u32, E.conv_c, E.inv_lnq);
    long long X = X0 + (long long)dir * (long long)ncv * E.photon_step;
    int cstep = (int)((long long)E.step + ncv);
    if (E.absorbing) {
      if (X < 0 || X >= E.domain) { cstep = INT32_MIN; ++esc; }
    } else if (X < 0 || X >= E.domain) {
      X = wrap_periodic(X, E.domain);
    }
    const unsigned long long slot = slot0 + jj;
    if (slot < E.ph_cap) {
      put_photon(E.phr, (long long)slot, X, child | (dir > 0 ? 1u : 0u));
      E.phs[slot] = cstep;
      // the tail key: steps from the last sort to the conversion (>= 1)
      const long long rel = (long long)cstep - E.ph_base;
      E.phk[slot] = (uint8_t)(cstep != INT32_MIN && rel < kFarKey ? rel : kFarKey);
    }
  }
  return esc;
}

// ------------------------------------------------------- emission in the push
// Emission of one pushed chunk of species s (section 2: a lepton that reaches
// gamma_thr emits; with a finite photon path the photon is stored and converts
// later, else the pair is made in place).  The push lists the chunk's ne
// emitters in LDS: entry (chunk-local index << 8 | k, the k emissions of this
// step) and the position after the move on the 2^-K grid (<< 1 | forward).
// Each thread takes four consecutive entries and requests their ids; a block
// scan of their photon counts gives each emitter its first photon (kept in
// its entry's place), and one global atomic reserves the chunk's slots.  The
// chunk's photons are then spread evenly over the threads.  Each emitter
// writes its index at its photons' places in s_map (the flux tile, empty
// between the flush and the next chunk, holds kMapPhotons of them), so a
// photon finds its emitter with one LDS read; the thread that reads an entry
// clears it, which leaves the tile zero again.  Photons past kMapPhotons
// (more than eight per lepton of the chunk) search the prefixes instead.
// Emission j of an emitter at step n is its tag-2 draw (draw_run): the child
// electron id is the 64-bit value with bit 0 cleared (the positron's has it
// set), and the photon's path in steps, n_conv = min{k >= 1 : u >= T_k} for u
// the 32-bit value, comes from the gap's conversion table.  The gap's
// emission constants are read here, where they are used, not held in
// registers through the push.
constexpr int kMapPhotons = kTile * 4;  // 16-bit entries in the flux tile
template <typename T, bool kTwo>
__device__ __forceinline__ void emit_chunk(GapDev* __restrict__ G, int s, long long i0, int ne,
                                           uint32_t* s_emit, const long long* s_emx,
                                           uint64_t* s_emid, int* s_scan,
                                           unsigned long long* s_slot, uint16_t* s_map) {
  const int tid = threadIdx.x;
  const int buf = G->buf;
  const bool in_place = G->table_len == 0;
  int kt;
  {
    // thread t owns the entries 4t .. 4t + 3 (list order): their ids, and a
    // block scan of their photon counts gives each its first photon; the
    // entry's slot in s_emit then holds that prefix
    gptr<const uint64_t> idA = glb<const uint64_t>((void*)G->id[buf][s]);
    uint32_t e[4];
    uint64_t idv[4];
    int mine = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = 4 * tid + j;
      e[j] = q < ne ? s_emit[q] : 0u;
      idv[j] = q < ne ? idA[i0 + (long long)(e[j] >> 8)] : 0ull;
      mine += (int)(e[j] & 255u);
    }
    const int ex0 = block_excl_scan(mine, s_scan, kt);  // ends with a barrier
    int ex = ex0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = 4 * tid + j;
      if (q < ne) {
        s_emit[q] = (uint32_t)ex;
        s_emid[q] = idv[j];
      }
      ex += (int)(e[j] & 255u);
    }
    // each emitter's index at its photons' places in the map (the thread's
    // own entries, read back: the next entry's first photon ends the range)
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {
      const int q = 4 * tid + j;
      if (q >= ne) break;
      const int a = (int)s_emit[q];
      const int b = j < 3 && q + 1 < ne ? (int)s_emit[q + 1] : ex0 + mine;
      const int mend = b < kMapPhotons ? b : kMapPhotons;
      for (int m = a; m < mend; ++m) s_map[m] = (uint16_t)q;
    }
    if (tid == 0) {
      if (in_place) {
        *s_slot = reserve_pairs(G, (unsigned long long)kt);
      } else {
        const unsigned long long b0 = atomicAdd(&G->n_ph_next, (unsigned long long)kt);
        if (b0 + (unsigned long long)kt > (unsigned long long)G->ph_cap) G->overflow = 1;
        *s_slot = b0;
      }
    }
  }
  __syncthreads();
  const unsigned long long base = *s_slot;
  const uint32_t step = (uint32_t)G->step;
  const uint64_t seed = G->seed;
  const int K = G->K;
  // the emitter of the chunk's photon p (read once, by the thread that owns
  // p): its map entry, or past the map the last entry whose first photon is
  // at most p
  auto emitter_of = [&](int p) {
    if (p < kMapPhotons) {
      const int q = s_map[p];
      s_map[p] = 0;
      return q;
    }
    int lo = 0, hi = ne - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((int)s_emit[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
  };
  if (in_place) {
    // pairs made in place (the paper's zero mean free path), both children
    // at the emitter's position moving along its direction
    const unsigned long long n0 = G->n[0], n1 = G->n[1], slots = (unsigned long long)G->slots;
    const long long mask = G->one - 1;
    const T inv_scale = (T)(1.0 / (double)G->one), pchild = (T)G->pchild;
    const bool evmap = G->evmap != nullptr;
    gptr<int32_t> c0 = glb(G->cell[buf][0]), c1 = glb(G->cell[buf][1]);
    gptr<T> o0 = glb<T>(G->off[buf][0]), o1 = glb<T>(G->off[buf][1]);
    gptr<T> p0 = glb<T>(G->p[buf][0]), p1 = glb<T>(G->p[buf][1]);
    gptr<uint64_t> d0 = glb(G->id[buf][0]), d1 = glb(G->id[buf][1]);
#pragma unroll 1
    for (int p = tid; p < kt; p += kBlock) {
      const int q = emitter_of(p);
      const int jj = p - (int)s_emit[q];
      const long long xe = s_emx[q];
      const long long X0 = xe >> 1;
      const int c = (int)(X0 >> K);
      const T offn = (T)(X0 & mask) * inv_scale;
      const T pc = (xe & 1) ? pchild : -pchild;
      const RunDraw u = draw_run(s_emid[q], seed, step, (uint32_t)jj, (uint32_t)kTagPhoton);
      const uint64_t child = u.bits & ~(uint64_t)1;
      const unsigned long long se = n0 + base + p, sp = n1 + base + p;
      if (se < slots) { c0[se] = c; o0[se] = offn; p0[se] = pc; d0[se] = child; }
      if (sp < slots) { c1[sp] = c; o1[sp] = offn; p1[sp] = pc; d1[sp] = child | 1u; }
      if (evmap) count_pairs(G, (long long)step, c, 1ull);
    }
    return;
  }
  const int pb = G->phbuf;
  gptr<PhotonRec> phr = glb(G->ph_rec[pb]);
  gptr<int32_t> phs = glb(G->ph_step[pb]);
  gptr<uint8_t> phk = glb(G->ph_key);
  const uint32_t* table = G->table;
  const int len = G->table_len;
  const float inv_lnq = G->inv_lnq;
  const float conv_c = G->conv_c;
  const long long domain = G->domain, photon_step = G->photon_step, ph_base = G->ph_base;
  const unsigned long long ph_cap = (unsigned long long)G->ph_cap;
  const bool absorbing = G->boundary == PIC_BC_ABSORBING;
  unsigned esc = 0;
  // the photon p of emitter q with its draw u: conversion step and store
  auto put = [&](int p, int q, const RunDraw& u) {
    const int ncv = conv_steps_direct(table, len, u.u32, conv_c, inv_lnq);
    const long long xe = s_emx[q];
    const long long dirq = (xe & 1) ? photon_step : -photon_step;
    long long X = (xe >> 1) + (long long)ncv * dirq;
    int cstep = (int)((long long)step + ncv);
    if (absorbing) {
      if (X < 0 || X >= domain) { cstep = INT32_MIN; ++esc; }
    } else if (X < 0 || X >= domain) {
      X = wrap_periodic(X, domain);
    }
    const unsigned long long sl = base + (unsigned long long)p;
    if (sl < ph_cap) {
      put_photon(phr, (long long)sl, X, (u.bits & ~(uint64_t)1) | (uint64_t)(xe & 1));
      phs[sl] = cstep;
      // the tail key: steps from the last sort to the conversion (>= 1)
      const long long rel = (long long)cstep - ph_base;
      phk[sl] = (uint8_t)(cstep != INT32_MIN && rel < kFarKey ? rel : kFarKey);
    }
  };
  if constexpr (kTwo) {
    // two photons per thread and round, their draws interleaved
#pragma unroll 1
    for (int p = tid; p < kt; p += 2 * kBlock) {
      const int p2 = p + kBlock;
      const bool two = p2 < kt;
      const int qa = emitter_of(p);
      const int qb = two ? emitter_of(p2) : qa;
      RunDraw ua, ub;
      draw_run2(s_emid[qa], s_emid[qb], seed, step, (uint32_t)(p - (int)s_emit[qa]),
                (uint32_t)((two ? p2 : p) - (int)s_emit[qb]), (uint32_t)kTagPhoton, ua, ub);
      put(p, qa, ua);
      if (two) put(p2, qb, ub);
    }
  } else {
#pragma unroll 1
    for (int p = tid; p < kt; p += kBlock) {
      const int q = emitter_of(p);
      put(p, q, draw_run(s_emid[q], seed, step, (uint32_t)(p - (int)s_emit[q]),
                         (uint32_t)kTagPhoton));
    }
  }
  if (absorbing) {
    const unsigned long long esc_w = wave_sum((unsigned long long)esc);
    if (lane_id() == 0 && esc_w > 0) atomicAdd(&G->esc_next, esc_w);
  }
}

// ------------------------------------------------------------------ push
// Sums of one workgroup over the work items of one gap, flushed to the
// gap's stripes when the workgroup moves to another gap or finishes.  The
// energies are exact integer sums of terms on the 2^-64 grid (fix64), so
// they do not depend on which slots the leptons occupy.  The kinetic energy
// is summed in each thread's registers; absorbed leptons are rare, so their
// count and lost energy go to LDS with atomics (s_abs[0..1] counts, s_abs[2..5]
// the limbs of the lost energy).
__device__ __forceinline__ void flush_tally(unsigned long long* __restrict__ stripes, int g,
                                            __int128& ke_t, bool diag, __int128* s_e,
                                            unsigned long long* s_abs) {
  const __int128 ke = wave_sum128(ke_t);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (lane_id() == 0) s_e[w] = ke;
  __syncthreads();
  if (threadIdx.x == 0) {
    const __int128 k = (s_e[0] + s_e[1]) + (s_e[2] + s_e[3]);
    const int st = blockIdx.x & (kStripes - 1);
    if (diag) limbs_add(stripe_slot(stripes, g, 0, st), k);
    unsigned long long* lost = stripe_slot(stripes, g, 1, st);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (s_abs[2 + q]) atomicAdd(lost + q, s_abs[2 + q]);
    if (s_abs[0]) atomicAdd(stripe_slot(stripes, g, 2, st), s_abs[0]);
    if (s_abs[1]) atomicAdd(stripe_slot(stripes, g, 3, st), s_abs[1]);
#pragma unroll
    for (int q = 0; q < 6; ++q) s_abs[q] = 0;
  }
  ke_t = 0;
}

// Lorentz factor of a lepton of momentum p (the stored value, binary32 in
// mixed precision) for the diagnostics: sqrt(1 + p^2) in binary64.
__device__ __forceinline__ double lepton_gamma64(double p) { return sqrt(1.0 + p * p); }

// The same for the per-step kinetic energy of the push, from the stored
// momentum p and the push's own Lorentz factor g of it.  In binary64 it is
// the square root above.  In binary32, g = sqrt(1 + p^2) rounded twice is
// within 3e-7 of the true value, and one Newton step g + (1 + p^2 - g^2) / (2 g)
// in binary64, with 1 / g from the binary32 reciprocal, leaves an error of
// about the square of that, below 1e-13 relative: far below the binary64
// sum's own tolerance, at a third of the cost of a correctly rounded root.
template <typename T>
__device__ __forceinline__ double diag_gamma(T p, T g);
template <>
__device__ __forceinline__ double diag_gamma<double>(double p, double) { return lepton_gamma64(p); }
template <>
__device__ __forceinline__ double diag_gamma<float>(float p, float g) {
  const double pd = (double)p, gd = (double)g;
  const double a = fma(pd, pd, 1.0);
  const double r = fma(-gd, gd, a);
  const double h = (double)(0.5f * __builtin_amdgcn_rcpf(g));
  return fma(r, h, gd);
}

// fix64 of a Lorentz factor t: for t in [1, 2^51), t 2^64 = m 2^(e + 12)
// (m the 53-bit significand, e >= 0 the exponent) is the integer part
// m >> (52 - e) above 64 fraction bits m << (12 + e); other values take the
// general conversion.
__device__ __forceinline__ __int128 fix64_gamma(double t) {
  if (!(t >= 1.0 && t < 0x1p51)) return fix64(t);
  const unsigned long long bits = (unsigned long long)__double_as_longlong(t);
  const int e = (int)(bits >> 52) - 1023;
  const unsigned long long m = (bits & 0xFFFFFFFFFFFFFull) | (1ull << 52);
  const unsigned long long hi = m >> (52 - e), lo = m << (12 + e);
  return (__int128)(((unsigned __int128)hi << 64) | lo);
}

// E at the cells left of, at and right of cell cl (a dead slot reads cell 0),
// with the boundary ghosts of the gather.  The binary32 push reads the
// binary32 copy of E (the same values as rounding E), binary64 reads E.
template <typename T>
struct ESrc;
template <>
struct ESrc<float> {
  static __device__ __forceinline__ gptr<const float> of(const GapDev* G) { return glb<const float>((void*)G->Ef); }
};
template <>
struct ESrc<double> {
  static __device__ __forceinline__ gptr<const double> of(const GapDev* G) { return glb<const double>((void*)G->E); }
};

template <typename T>
__device__ __forceinline__ void load_e3(gptr<const T> E, int cl, bool periodic, int nc, T& em, T& ec,
                                        T& ep) {
  const int c = cl == kDead ? 0 : cl;
  int cm = c - 1, cp = c + 1;
  if (periodic) { cm = cm < 0 ? nc - 1 : cm; cp = cp >= nc ? 0 : cp; }
  else { cm = cm < 0 ? 0 : cm; cp = cp >= nc ? nc - 1 : cp; }
  em = E[cm];
  ec = E[c];
  ep = E[cp];
}

// E at the four cells around the nodes jo-1, jo, jo+1 of the quadratic
// spline of a lepton in cell cl (jo = 1 when its offset is at least 1/2):
// cells cl+jo-2 .. cl+jo+1, wrapped (periodic) or clamped to the edge cells
// (absorbing: the gather's zero-gradient ghosts).
template <typename T>
__device__ __forceinline__ void load_e4(gptr<const T> E, int cl, T off, bool periodic, int nc,
                                        T& e0, T& e1, T& e2, T& e3) {
  const int c = cl == kDead ? 0 : cl;
  const int k0 = c + (off >= (T)0.5 ? 1 : 0) - 2;
  int i0 = k0, i1 = k0 + 1, i2 = k0 + 2, i3 = k0 + 3;
  if (periodic) {
    i0 = i0 < 0 ? i0 + nc : i0;
    i1 = i1 < 0 ? i1 + nc : i1;
    i2 = i2 >= nc ? i2 - nc : i2;
    i3 = i3 >= nc ? i3 - nc : i3;
  } else {
    i0 = i0 < 0 ? 0 : i0;
    i1 = i1 < 0 ? 0 : i1;
    i2 = i2 >= nc ? nc - 1 : i2;
    i3 = i3 >= nc ? nc - 1 : i3;
  }
  e0 = E[i0];
  e1 = E[i1];
  e2 = E[i2];
  e3 = E[i3];
}

// Quadratic-spline weights of a lepton at X (units 2^-K cells from a node,
// -3/2 .. 5/2 cells):
// nearest node j = floor(X / 2^K + 1/2), delta = X - j 2^K in [-1/2, 1/2) 2^K;
// the outer nodes get floor((2^(K-1) -/+ delta)^2 / 2^(K+1)), the middle one
// the rest of 2^K, so the three sum to 2^K exactly.
template <typename I>
__device__ __forceinline__ void spline_weights(I X, I ONE, int K, int& j, I& wl, I& wc, I& wr) {
  const I HALF = ONE >> 1;
  const I t = X + HALF;  // in [-2^K, 3 2^K]: a move within a cell, or one carried past a wall
  j = t < 0 ? -1 : (t >= 3 * ONE ? 3 : (t >= 2 * ONE ? 2 : (t >= ONE ? 1 : 0)));
  const I delta = X - (I)j * ONE;
  if constexpr (sizeof(I) == 4) {
    // 2^-24 grid: both factors fit 32 bits, one 32 x 32 -> 64 product each
    const uint32_t a = (uint32_t)(HALF - delta), b = (uint32_t)(HALF + delta);
    wl = (I)(((uint64_t)a * a) >> (K + 1));
    wr = (I)(((uint64_t)b * b) >> (K + 1));
  } else {
    const unsigned long long a = (unsigned long long)(HALF - delta);
    const unsigned long long b = (unsigned long long)(HALF + delta);
    wl = (I)(((unsigned __int128)a * a) >> (K + 1));
    wr = (I)(((unsigned __int128)b * b) >> (K + 1));
  }
  wc = ONE - wl - wr;
}

// E at a lepton at offset o of its cell, from the E values around it:
// linear shape (em, ec, ep = cells c-1, c, c+1): the node averages
// interpolated linearly; spline (em..ex = cells c+j-2 .. c+j+1): the
// averages at the nodes j-1, j, j+1 weighted by the lepton's integer weights
// w0..w2 (in 2^-K; exact in the particle type).
template <typename T, bool kSpline, typename I>
__device__ __forceinline__ T gather_e(T o, I w0, I w1, I w2, T inv_scale, T em, T ec, T ep, T ex) {
  const T half_t = (T)0.5;
  if constexpr (kSpline) {
    const T en0 = half_t * (em + ec);
    const T en1 = half_t * (ec + ep);
    const T en2 = half_t * (ep + ex);
    const T sw0 = (T)w0 * inv_scale, sw1 = (T)w1 * inv_scale, sw2 = (T)w2 * inv_scale;
    return (sw0 * en0 + sw1 * en1) + sw2 * en2;
  } else {
    const T el = half_t * (em + ec);
    const T er = half_t * (ec + ep);
    return el + o * (er - el);
  }
}

// Lepton range of work item w of gap G: species s, indices [i0, i1).
__device__ __forceinline__ void push_item(long long local, long long chunks0, long long n0,
                                          long long n1, int& s, long long& i0, long long& i1) {
  s = local < chunks0 ? 0 : 1;
  i0 = (s == 0 ? local : local - chunks0) * kChunk;
  const long long nS = s == 0 ? n0 : n1;
  i1 = i0 + kChunk < nS ? i0 + kChunk : nS;
}

// One work item is a chunk of kChunk leptons of one species of one gap.
// Leptons are sorted by groups of 8 cells (between re-sorts they drift by a
// few cells), so a chunk touches a short range of cells: its current is summed in a
// per-workgroup LDS tile over that range and added to the grid with one
// atomic per touched cell.  Chunks spread over more than kTile cells (the
// sparse early cascade, unsorted appended leptons) add to the grid directly.
//
// The lepton arrays are streamed once per step, so their loads and stores
// are non-temporal and leave the caches to E and the grid.
//
// Loads are issued in phases (all lepton state of a chunk, then all its E
// values) so that each phase waits once.  In binary32 the loop is also
// software-pipelined: the lepton state of the next chunk of the same gap is
// loaded while the current one is pushed, and the E values of the current
// chunk are requested before that prefetch, so waiting for them leaves the
// prefetch in flight.  The gap's constants are read once per gap.  kSpread
// instantiates the per-lepton thresholds of a spread of gamma_thr, kSpline
// the quadratic-spline shape; batches without them run the
// kernel without that code.
template <typename T, bool kSpread, bool kSpline>
__global__ __launch_bounds__(kBlock, kSpread ? PushCfg<T>::spread_waves
                                     : (kSpline ? PushCfg<T>::spline_waves : PushCfg<T>::waves)) void k_push(GapDev* __restrict__ gaps,
                                                 const long long* __restrict__ wi, int B,
                                                 unsigned long long* __restrict__ stripes) {
  using I = typename Fixed<T>::I;
  __shared__ long long s_flux[kTile];
  __shared__ uint32_t s_emit[kChunk];  // chunk-local index << 8 | k
  __shared__ long long s_emx[kChunk];  // the emitter's position after the move << 1 | forward
  __shared__ uint64_t s_emid[kChunk];  // the emitter's id (emission in the push)
  __shared__ int s_scan[kBlock / 64];
  __shared__ unsigned long long s_slot;  // the chunk's first photon (or pair) slot
  __shared__ int s_red[2][8];
  __shared__ __int128 s_e[4];
  __shared__ unsigned long long s_abs[6];
  __shared__ int s_emit_n;
  // leptons of the chunk that need their own threshold, and the thresholds
  __shared__ uint32_t s_cand[kSpread ? kChunk : 1];
  __shared__ T s_thr[kSpread ? kChunk : 1];
  __shared__ int s_ncand;

  // the flux tile is kept zero between chunks (each flush clears what it
  // read), so it is zeroed once here
  for (int k = threadIdx.x; k < kTile; k += kBlock) s_flux[k] = 0;
  if (threadIdx.x < 6) s_abs[threadIdx.x] = 0;
  __syncthreads();
  int parity = 0;

  const long long total = wi[B];
  long long w0, w1;
  xcd_range(total, w0, w1);
  const int tid = threadIdx.x;
  const bool in_push = total < gaps->emit_split;  // this step emits in the push
  const int lane = lane_id();
  __int128 ke_t = 0;  // this thread's kinetic energy terms (diagnosed steps)
  uint32_t my_emitters = 0;  // emitters listed by this workgroup (thread 0)

  // constants of the current gap
  int g = -1;
  long long gbeg = 0, gend = -1, chunks0 = 0, n0 = 0, n1 = 0;
  bool diag = false, periodic = false, gap_ok = false;
  int nc = 0;
  gptr<int32_t> cellS[2] = {nullptr, nullptr};
  gptr<T> offS[2] = {nullptr, nullptr}, pS[2] = {nullptr, nullptr};
  gptr<const T> E = nullptr;
  gptr<unsigned long long> F = nullptr;
  I ONE = 0;
  T scale = 0, inv_scale = 0, dt_t = 0, dtdx = 0, gthr = 0, gpair = 0, thr_lo = 0;
  double sigma = 0.0, gthr64 = 0.0;
  int Kb = 0;  // offset grid bits (the spline's weights, the emitters' positions)
  uint64_t kseed = 0;
  gptr<uint64_t> idS[2] = {nullptr, nullptr};
  GapDev* __restrict__ G = gaps;

  // lepton state of the chunk about to be pushed (prefetched when `have`)
  int cl[kItems];
  T ov[kItems], pv[kItems];
  bool have = false;

  for (long long w = w0; w < w1; ++w) {
    if (w >= gend) {  // uniform: the first chunk of another gap
      if (g >= 0) flush_tally(stripes, g, ke_t, diag, s_e, s_abs);
      g = find_gap(wi, B, w);
      G = gaps + g;
      gbeg = wi[g];
      gend = wi[g + 1];
      gap_ok = G->status == PIC_OK;
      diag = (G->step % G->diag_every) == 0;
      const int buf = G->buf;
      n0 = (long long)G->n[0];
      n1 = (long long)G->n[1];
      chunks0 = (n0 + kChunk - 1) / kChunk;
      for (int sp = 0; sp < 2; ++sp) {
        cellS[sp] = glb(G->cell[buf][sp]);
        offS[sp] = glb<T>(G->off[buf][sp]);
        pS[sp] = glb<T>(G->p[buf][sp]);
        if constexpr (kSpread) idS[sp] = glb(G->id[buf][sp]);
      }
      E = ESrc<T>::of(G);
      F = glb<unsigned long long>((void*)G->F);
      nc = G->n_cells;
      periodic = G->boundary == PIC_BC_PERIODIC;
      ONE = (I)G->one;
      scale = (T)(double)G->one;
      inv_scale = (T)(1.0 / (double)G->one);
      dt_t = (T)G->dt;
      dtdx = (T)G->dtdx;
      gthr = (T)G->gthr;
      gpair = (T)G->gpair;
      Kb = G->K;
      if constexpr (kSpread) {
        sigma = G->sigma;
        gthr64 = G->gthr64;
        thr_lo = (T)G->thr_lo;
        kseed = G->seed;
      }
      have = false;
    }
    if (!gap_ok) continue;
    int listed = 0;  // emitters of this chunk
    int s;
    long long i0, i1;
    push_item(w - gbeg, chunks0, n0, n1, s, i0, i1);
    gptr<int32_t> cellA = cellS[s];
    gptr<T> offA = offS[s];
    gptr<T> pA = pS[s];
    gptr<uint64_t> idA = idS[s];
    if (!have) {
      // unconditional loads (slots past the end read slot 0 and are discarded),
      // so that all of them are in flight at once
#pragma unroll
      for (int j = 0; j < kItems; ++j) {
        const long long i = i0 + tid + (long long)j * kBlock;
        const long long ii = i < i1 ? i : 0;
        const int cv = __builtin_nontemporal_load(&cellA[ii]);
        const T ovv = __builtin_nontemporal_load(&offA[ii]), pvv = __builtin_nontemporal_load(&pA[ii]);
        cl[j] = i < i1 ? cv : kDead;
        ov[j] = i < i1 ? ovv : (T)0;
        pv[j] = i < i1 ? pvv : (T)0;
      }
    }
    int mn = INT32_MAX, mx = INT32_MIN;
#pragma unroll
    for (int j = 0; j < kItems; ++j)
      if (cl[j] != kDead) { mn = min(mn, cl[j]); mx = max(mx, cl[j]); }
    if (tid == 0) {
      s_emit_n = 0;
      if constexpr (kSpread) s_ncand = 0;
    }
    block_minmax_pp(mn, mx, s_red, parity);
    // E at the cells around each lepton (dead slots read cell 0), requested
    // for the first group of items now and for later groups just before
    // they are pushed
    constexpr int kEG = PushCfg<T>::e_group;
    T Em[kItems], Ec[kItems], Ep[kItems], Ex[kItems];
#pragma unroll
    for (int j = 0; j < kEG; ++j) {
      if constexpr (kSpline) load_e4(E, cl[j], ov[j], periodic, nc, Em[j], Ec[j], Ep[j], Ex[j]);
      else load_e3(E, cl[j], periodic, nc, Em[j], Ec[j], Ep[j]);
    }
    // prefetch the next chunk of this gap; the loads are issued whether or
    // not there is one (then they read slot 0 and are discarded), so the
    // wait for the E values above never waits for them
    const bool pre = PushCfg<T>::prefetch && w + 1 < w1 && w + 1 < gend;
    int cln[kItems];
    T ovn[kItems], pvn[kItems];
    if constexpr (PushCfg<T>::prefetch) {
      int s2 = s;
      long long j0 = 0, j1 = 0;
      if (pre) push_item(w + 1 - gbeg, chunks0, n0, n1, s2, j0, j1);
      gptr<const int32_t> c2A = cellS[s2];
      gptr<const T> o2A = offS[s2];
      gptr<const T> p2A = pS[s2];
#pragma unroll
      for (int j = 0; j < kItems; ++j) {
        const long long i = j0 + tid + (long long)j * kBlock;
        const long long ii = i < j1 ? i : 0;
        const int cv = __builtin_nontemporal_load(&c2A[ii]);
        const T ovv = __builtin_nontemporal_load(&o2A[ii]), pvv = __builtin_nontemporal_load(&p2A[ii]);
        cln[j] = i < j1 ? cv : kDead;
        ovn[j] = i < j1 ? ovv : (T)0;
        pvn[j] = i < j1 ? pvv : (T)0;
      }
    }
    if (mx >= mn) {  // uniform: some lepton of this chunk is alive
      // cells a lepton's current can reach: c-1..c+1 (linear), c-2..c+2 (spline)
      constexpr int kReach = kSpline ? 2 : 1;
      const int base = mn - kReach;
      const int span = mx - mn + 1 + 2 * kReach;
      const bool lds = span <= kTile;
      const T qdt = s == 0 ? -dt_t : dt_t;
      const T one_t = (T)1;
      bool bad = false, emit_bad = false;
      // Under a spread of gamma_thr, every item is pushed first; the leptons
      // at or above the lowest threshold are listed in LDS and the workgroup
      // draws their thresholds together, one lepton per thread, instead of
      // each wave drawing for whichever of its lanes need it.
      [[maybe_unused]] T pre_pn[kItems], pre_gam[kItems];
      [[maybe_unused]] int cpos[kItems];
      if constexpr (kSpread) {
        static_assert(PushCfg<T>::e_group == kItems, "the E values of every item are loaded here");
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
          const T o = ov[j];
          int jw = 0;
          I w0 = 0, w1 = 0, w2 = 0;
          if constexpr (kSpline) spline_weights<I>((I)(o * scale), ONE, Kb, jw, w0, w1, w2);
          const T Epart = gather_e<T, kSpline>(o, w0, w1, w2, inv_scale, Em[j], Ec[j], Ep[j], Ex[j]);
          pre_pn[j] = pv[j] + qdt * Epart;
          pre_gam[j] = sqrt(one_t + pre_pn[j] * pre_pn[j]);
          cpos[j] = -1;
          if (cl[j] != kDead && sigma != 0.0 && pre_gam[j] >= thr_lo) {
            cpos[j] = atomicAdd(&s_ncand, 1);
            s_cand[cpos[j]] = (uint32_t)(tid + j * kBlock);
          }
        }
        __syncthreads();
        const int ncand = s_ncand;
        for (int q = tid; q < ncand; q += kBlock)
          s_thr[q] = lepton_threshold<T>(idA[i0 + s_cand[q]], kseed, gthr64, sigma);
        __syncthreads();
      }
#pragma unroll
      for (int j = 0; j < kItems; ++j) {
        if (j > 0 && j % kEG == 0) {
#pragma unroll
          for (int jj = j; jj < j + kEG; ++jj) {
            if constexpr (kSpline) load_e4(E, cl[jj], ov[jj], periodic, nc, Em[jj], Ec[jj], Ep[jj], Ex[jj]);
            else load_e3(E, cl[jj], periodic, nc, Em[jj], Ec[jj], Ep[jj]);
          }
        }
        const long long i = i0 + tid + (long long)j * kBlock;
        const int c = cl[j];
        if (c == kDead) continue;
        const T o = ov[j];
        const I oq = (I)(o * scale);
        // the spline's weights at the start of the step serve gather and deposit
        int jo = 0;
        I wo0 = 0, wo1 = 0, wo2 = 0;
        if constexpr (kSpline) spline_weights<I>(oq, ONE, Kb, jo, wo0, wo1, wo2);
        // gather, push and move
        T pn, gam;
        if constexpr (kSpread) {
          pn = pre_pn[j];
          gam = pre_gam[j];
        } else {
          const T Epart = gather_e<T, kSpline>(o, wo0, wo1, wo2, inv_scale, Em[j], Ec[j], Ep[j], Ex[j]);
          pn = pv[j] + qdt * Epart;
          gam = sqrt(one_t + pn * pn);
        }
        const T v = pn / gam;
        const T d = v * dtdx;
        const I dq = (I)rint(d * scale);
        I nq = oq + dq;
        int c2 = c;
        bool keep = true;
        if constexpr (kSpline) {
          // charge-conserving deposit of the spline: the flux through cell c+k
          // (between nodes c+k and c+k+1) is the charge that left the nodes up
          // to c+k, the running sum of old minus new weight from the leftmost
          // node either spline touches (it returns to zero after the last)
          // A lepton can leave only from an edge cell.  Through an absorbing
          // wall it is carried on to 3/2 cells beyond it, where its spline no
          // longer touches the wall node, and removed; fluxes through cells
          // outside the domain are dropped.
          const bool out_left = !periodic && c == 0 && nq < 0;
          const bool out_right = !periodic && c == nc - 1 && nq >= ONE;
          if (out_left || out_right) {
            const I target = out_left ? -(ONE + (ONE >> 1)) : 2 * ONE + (ONE >> 1);
            int jn;
            I wn0, wn1, wn2;
            spline_weights<I>(target, ONE, Kb, jn, wn0, wn1, wn2);
            const int lo = min(jo, jn) - 1, hi = max(jo, jn) + 1;
            I run = 0;
            for (int k = lo; k < hi; ++k) {
              const int ko = k - jo + 1, kn = k - jn + 1;
              const I wo = ko == 0 ? wo0 : (ko == 1 ? wo1 : (ko == 2 ? wo2 : (I)0));
              const I wn = kn == 0 ? wn0 : (kn == 1 ? wn1 : (kn == 2 ? wn2 : (I)0));
              run += wo - wn;
              const int cc = c + k;
              const long long f = s == 0 ? -(long long)run : (long long)run;
              if (f != 0 && cc >= 0 && cc < nc) {
                if (lds) atomicAdd((unsigned long long*)&s_flux[cc - base], as_u64(f));
                else gadd(F + cc, as_u64(f));
              }
            }
            keep = false;
          } else {
          int jn;
          I wn0, wn1, wn2;
          spline_weights<I>(nq, ONE, Kb, jn, wn0, wn1, wn2);
          const int lo = min(jo, jn) - 1;
          I run = 0;  // at most 2^K in magnitude
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            const int k = lo + r;
            const int ko = k - jo + 1, kn = k - jn + 1;
            const I wo = ko == 0 ? wo0 : (ko == 1 ? wo1 : (ko == 2 ? wo2 : (I)0));
            const I wn = kn == 0 ? wn0 : (kn == 1 ? wn1 : (kn == 2 ? wn2 : (I)0));
            run += wo - wn;
            const long long f = s == 0 ? -(long long)run : (long long)run;
            const int cu = c + k;  // unwrapped cell
            // beside an absorbing wall the spline's flux through the cells
            // beyond it is dropped; periodic gaps wrap it (at the flush)
            if (f != 0 && (periodic || (cu >= 0 && cu < nc))) {
              if (lds) {
                // unwrapped tile index: c - 2 .. c + 2 lie in [base, base + span)
                atomicAdd((unsigned long long*)&s_flux[cu - base], as_u64(f));
              } else {
                const int cc = cu < 0 ? cu + nc : (cu >= nc ? cu - nc : cu);
                gadd(F + cc, as_u64(f));
              }
            }
          }
          // the lepton's cell after the move (inside the domain here)
          if (nq >= ONE) { nq -= ONE; c2 = c + 1 >= nc ? 0 : c + 1; }
          else if (nq < 0) { nq += ONE; c2 = c - 1 < 0 ? nc - 1 : c - 1; }
          }
        } else {
          I a1, a2 = 0;   // flux of a positive charge through this cell and the next
          int cross = 0;  // -1, 0, +1: node crossed to the left / none / right
          if (nq >= ONE) {
            a1 = ONE - oq;
            cross = 1;
            c2 = c + 1;
            nq -= ONE;
            a2 = nq;
            if (c2 >= nc) { if (periodic) c2 = 0; else keep = false; }
          } else if (nq < 0) {
            a1 = -oq;
            cross = -1;
            c2 = c - 1;
            nq += ONE;
            a2 = nq - ONE;
            if (c2 < 0) { if (periodic) c2 = nc - 1; else keep = false; }
          } else {
            a1 = dq;
          }
          const long long f1 = s == 0 ? -(long long)a1 : (long long)a1;
          const long long f2 = s == 0 ? -(long long)a2 : (long long)a2;
          const bool second = cross != 0 && keep;
          if (lds) {
            // tile indices are unwrapped: c - 1 .. c + 1 all lie in [base, base + span)
            atomicAdd((unsigned long long*)&s_flux[c - base], as_u64(f1));
            if (second) atomicAdd((unsigned long long*)&s_flux[c + cross - base], as_u64(f2));
          } else {
            gadd(F + c, as_u64(f1));
            if (second) gadd(F + c2, as_u64(f2));
          }
        }
        if (!isfinite(pn) || !isfinite(gam)) bad = true;
        if (keep) {
          // emission: repeated subtraction of gamma_pair while at or above threshold
          // (the lepton's own threshold under a spread of gamma_thr, needed only at
          // or above the lowest one)
          T thr = gthr;
          if constexpr (kSpread)
            if (cpos[j] >= 0) thr = s_thr[cpos[j]];
          int k = 0;
          T gm = gam;
          while (gm >= thr && k <= kMaxEmit) {
            gm = gm - gpair;
            ++k;
          }
          if (k > kMaxEmit) { emit_bad = true; k = 0; }
          if (k > 0) {
            // the recoil keeps the direction: the stored momentum's sign bit
            // is the emitter's direction even when its magnitude is zero
            const T mag = sqrt(gm * gm - one_t);
            pn = pn > (T)0 ? mag : -mag;
            const int pos = atomicAdd(&s_emit_n, 1);
            s_emit[pos] = ((uint32_t)(i - i0) << 8) | (uint32_t)k;
            // its photons (or pairs) start at its position after the move,
            // along the stored momentum's sign
            const long long X0 = ((long long)c2 << Kb) + (long long)nq;
            s_emx[pos] = (X0 << 1) | (signbit(pn) ? 0ll : 1ll);
          }
          __builtin_nontemporal_store(pn, &pA[i]);
          __builtin_nontemporal_store((T)nq * inv_scale, &offA[i]);
          if (c2 != c) __builtin_nontemporal_store(c2, &cellA[i]);
          // energy diagnostics in binary64 from the stored momentum
          if (diag) ke_t += fix64_gamma(diag_gamma<T>(pn, gm));
        } else {
          const unsigned __int128 u = (unsigned __int128)fix64(lepton_gamma64((double)pn));
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const unsigned long long l = (unsigned long long)(u >> (32 * q)) & 0xFFFFFFFFull;
            if (l) atomicAdd(&s_abs[2 + q], l);
          }
          atomicAdd(&s_abs[s], 1ull);
          pA[i] = pn;
          cellA[i] = kDead;
        }
      }

      const unsigned long long bad_w = __ballot(bad);
      const unsigned long long ebad_w = __ballot(emit_bad);
      if (lane == 0) {
        if (bad_w) G->nonfinite = 1;
        if (ebad_w) G->emit_err = 1;
      }

      __syncthreads();
      if (lds) {
        for (int k = tid; k < span; k += kBlock) {
          const long long f = s_flux[k];
          if (f != 0) {
            s_flux[k] = 0;
            int cc = base + k;
            if (cc < 0) cc += nc;
            else if (cc >= nc) cc -= nc;
            gadd(F + cc, as_u64(f));
          }
        }
      }
      // ---- this chunk's emitters: their photons (or in-place pairs) now, or
      // listed in the chunk's own slice of the list for the emission role
      const int ne = __builtin_amdgcn_readfirstlane(s_emit_n);
      if (ne > 0 && in_push) {
        emit_chunk<T, PushCfg<T>::prefetch && !kSpread && !kSpline>(G, s, i0, ne, s_emit, s_emx,
                                                                      s_emid, s_scan, &s_slot,
                      reinterpret_cast<uint16_t*>(s_flux));
      } else if (ne > 0) {
        listed = ne;
        gptr<uint32_t> el = glb(G->emit_ent + w * (long long)kChunk);
        for (int k = tid; k < ne; k += kBlock) el[k] = s_emit[k];
      }
      __syncthreads();
    }
    if (tid == 0) {
      glb(G->emit_cnt)[w] = listed;
      my_emitters += (uint32_t)listed;
    }
    if constexpr (PushCfg<T>::prefetch) {
#pragma unroll
      for (int j = 0; j < kItems; ++j) { cl[j] = cln[j]; ov[j] = ovn[j]; pv[j] = pvn[j]; }
    }
    have = pre;
  }
  if (g >= 0) flush_tally(stripes, g, ke_t, diag, s_e, s_abs);
  // emitters of this workgroup's chunk range, indexed in chunk order (every
  // descriptor holds the batch's array)
  if (tid == 0) glb(gaps->wg_emit)[xcd_logical((int)blockIdx.x, (int)gridDim.x)] = my_emitters;
}

// ------------------------------------------------------- emission role
// Walks the emitters with flattened indices [qa, qb) (chunk order, then list
// order within a chunk) among chunks [x, xend) of gap E.G, whose first
// emitter has flattened index Q, and emits their photons (or in-place
// pairs).  Windows of kBlock chunks are scanned for their emitter counts;
// each round hands one emitter to each thread, a block scan of the emitters'
// photon counts gives each its place, and the round's slots are reserved
// with one atomic.  On return x and Q point past the last window walked.
template <typename T>
__device__ __forceinline__ void emit_walk(const EmitGap<T>& E, long long& x, long long xend,
                                          unsigned long long& Q, unsigned long long qa,
                                          unsigned long long qb, long long wg0, unsigned& esc,
                                          gptr<const uint32_t> cntA, gptr<const uint32_t> entA,
                                          int* s_nb, int* s_tmp, unsigned long long* s_base) {
  // electron chunks come first in the gap's items
  const long long chunks0 = ((long long)E.n0 + kChunk - 1) / kChunk;
  while (x < xend && Q < qb) {
    const long long xc0 = x + threadIdx.x;
    const int ne = xc0 < xend ? (int)cntA[xc0] : 0;
    int nwin;
    const int nb = block_excl_scan(ne, s_tmp, nwin);
    s_nb[threadIdx.x] = nb;
    __syncthreads();
    const unsigned long long lo = qa > Q ? qa : Q;
    const unsigned long long hi = qb < Q + (unsigned long long)nwin ? qb : Q + (unsigned long long)nwin;
    for (unsigned long long r = lo; r < hi; r += kBlock) {
      const unsigned long long q = r + threadIdx.x;
      int k = 0, s = 0;
      long long i = 0;
      if (q < hi) {
        const int ql = (int)(q - Q);
        // the chunk holding emitter ql of the window: last t with s_nb[t] <= ql
        int a = 0, b = kBlock - 1;
        while (a < b) {
          const int mid = (a + b + 1) >> 1;
          if (s_nb[mid] <= ql) a = mid; else b = mid - 1;
        }
        const long long xc = x + a;
        const uint32_t en = entA[xc * kChunk + (ql - s_nb[a])];
        k = (int)(en & 255u);
        const long long local = xc - wg0;
        s = local < chunks0 ? 0 : 1;
        i = (s == 0 ? local : local - chunks0) * kChunk + (long long)(en >> 8);
      }
      int kt;
      const int ex = block_excl_scan(k, s_tmp, kt);  // ends with a barrier
      if (kt == 0) continue;                          // uniform
      if (threadIdx.x == 0) {
        if (E.in_place) {
          s_base[0] = reserve_pairs(E.G, (unsigned long long)kt);
        } else {
          const unsigned long long b0 = atomicAdd(&E.G->n_ph_next, (unsigned long long)kt);
          if (b0 + (unsigned long long)kt > E.ph_cap) E.G->overflow = 1;
          s_base[0] = b0;
        }
      }
      __syncthreads();
      const unsigned long long base = s_base[0];
      if (k > 0) esc += emit_listed<T>(E, s, i, k, base + (unsigned long long)ex);
      __syncthreads();  // s_base is rewritten by the next round
    }
    x = x + kBlock < xend ? x + kBlock : xend;
    Q += (unsigned long long)nwin;
    __syncthreads();  // s_nb is rewritten by the next window
  }
}

// Emission is balanced by emitters, not by chunks: the push left the number
// of emitters of each of its workgroups (in chunk order), so every
// workgroup here scans those counts, takes an equal share of the flattened
// emitter list, and walks it gap by gap in one pass.
template <typename T>
__device__ void emit_role(GapDev* __restrict__ gaps, const long long* __restrict__ wi, int B,
                          const int32_t* __restrict__ emit_cnt,
                          const uint32_t* __restrict__ emit_ent,
                          const uint32_t* __restrict__ wg_emit, int vb, int nvb,
                          uint32_t* s_pre, unsigned long long* s_base, int* s_nb, int* s_tmp) {
  constexpr int kPer = kPushGrid / kBlock;
  const long long total = wi[B];
  if (total < gaps->emit_split) return;  // this step emitted in the push
  // exclusive prefix of the push workgroups' emitter counts
  uint32_t v[kPer];
  uint32_t loc = 0;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    v[j] = glb<const uint32_t>((void*)wg_emit)[threadIdx.x * kPer + j];
    loc += v[j];
  }
  // block scan of the per-thread sums (a batch holds fewer than 2^32 lepton slots)
  const uint32_t incl = wave_incl_scan(loc);
  __syncthreads();
  if (lane_id() == 63) s_tmp[threadIdx.x >> 6] = (int)incl;
  __syncthreads();
  uint32_t off = 0, Etot = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; ++k) {
    const uint32_t t = (uint32_t)s_tmp[k];
    if (k < (int)(threadIdx.x >> 6)) off += t;
    Etot += t;
  }
  off += incl - loc;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    s_pre[threadIdx.x * kPer + j] = off;
    off += v[j];
  }
  __syncthreads();
  if (Etot == 0) return;
  const unsigned long long share = ((unsigned long long)Etot + nvb - 1) / nvb;
  const unsigned long long q0 = (unsigned long long)vb * share;
  if (q0 >= Etot) return;
  const unsigned long long q1 = q0 + share < Etot ? q0 + share : Etot;
  // the push workgroup holding emitter q0: last lb with s_pre[lb] <= q0
  int a = 0, b = kPushGrid - 1;
  while (a < b) {
    const int mid = (a + b + 1) >> 1;
    if (s_pre[mid] <= q0) a = mid; else b = mid - 1;
  }
  long long x, xa_end;
  share_range(total, a, kPushGrid, x, xa_end);
  unsigned long long Q = s_pre[a];
  gptr<const uint32_t> cntA = glb<const uint32_t>((void*)emit_cnt);
  gptr<const uint32_t> entA = glb<const uint32_t>((void*)emit_ent);
  while (x < total && Q < q1) {
    const int g = find_gap(wi, B, x);
    GapDev* __restrict__ G = gaps + g;
    const long long xend = wi[g + 1];
    const long long wg0 = wi[g];
    const EmitGap<T> E = emit_gap<T>(G);
    unsigned esc = 0;
    emit_walk<T>(E, x, xend, Q, q0, q1, wg0, esc, cntA, entA, s_nb, s_tmp, s_base);
    if (E.absorbing && !E.in_place) {
      const unsigned long long esc_w = wave_sum((unsigned long long)esc);
      if (lane_id() == 0 && esc_w > 0) atomicAdd(&G->esc_next, esc_w);
    }
  }
}

// ----------------------------------------------------------------- field
__device__ void field_role(GapDev* __restrict__ gaps, const long long* __restrict__ cwi, int B,
                           int vb, double* s_red) {
  const int g = find_gap(cwi, B, vb);
  GapDev* __restrict__ G = gaps + g;
  if (G->status != PIC_OK) return;
  const long long c0 = (vb - cwi[g]) * (long long)kCellChunk;
  const int nc = G->n_cells;
  const double wq = G->wq, dxh = G->dx, jmdt = G->jmdt;
  gptr<long long> F = glb(G->F);
  gptr<double> E = glb(G->E);
  gptr<float> Ef = glb(G->Ef);
  gptr<long long> Fl = glb(G->F_last);
  // the thread's cells c0 + tid + j kBlock: every load is requested before
  // any cell is updated
  constexpr int kPer = kCellChunk / kBlock;
  long long fv[kPer];
  double ev[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const long long c = c0 + threadIdx.x + (long long)j * kBlock;
    const long long cc = c < nc ? c : 0;
    fv[j] = F[cc];
    ev[j] = E[cc];
  }
  double fe = 0.0, es = 0.0;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const long long c = c0 + threadIdx.x + (long long)j * kBlock;
    if (c >= nc) break;
    const long long f = fv[j];
    double e = ev[j] - wq * (double)f;
    if (jmdt != 0.0) e = e + jmdt;  // imposed current of the co-rotating frame
    E[c] = e;
    Ef[c] = (float)e;
    Fl[c] = f;
    F[c] = 0;
    fe += e * e * dxh * 0.5;
    es += e;
  }
  // the chunk's partial sums in a fixed order (cells are fixed to threads),
  // then added exactly across chunks
  fe = wave_sum(fe);
  es = wave_sum(es);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) { s_red[w] = fe; s_red[4 + w] = es; }
  __syncthreads();
  if (threadIdx.x == 0) {
    wide_add(G->fe_wide, (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]));
    const double esum = (s_red[4] + s_red[5]) + (s_red[6] + s_red[7]);
    wide_add(esum >= 0.0 ? G->esp_wide : G->esn_wide, esum);
  }
}

// --------------------------------------------------------------- convert
// Photons due at step n: bucket n - ph_base of the sorted body, plus those
// appended to the unsorted tail since the last re-sort.
__device__ __forceinline__ void photon_ranges(const GapDev* G, long long& b0, long long& b1,
                                              long long& t0, long long& t1) {
  const long long k = G->step - G->ph_base;
  b0 = 0;
  b1 = 0;
  if (G->table_len > 0 && k >= 0 && k < G->table_len) {
    b0 = k == 0 ? 0 : (long long)G->ph_bucket[k - 1];
    b1 = (long long)G->ph_bucket[k];
  }
  t0 = (long long)G->ph_body_n;
  t1 = (long long)G->n_ph;
}

// Conversion items of a gap: chunks of kPhChunk photons of the due bucket,
// then of the tail, whose chunks start on kKeyRun boundaries (the first one
// at or below the tail's start) so that keys are read with aligned loads.
__device__ __forceinline__ long long tail_items(long long t0, long long t1) {
  return t1 > t0 ? (t1 - (t0 & ~(long long)(kKeyRun - 1)) + kPhChunk - 1) / kPhChunk : 0;
}

// Item `local` of a gap whose due ranges are [b0, b1) (sorted body) and
// [t0, t1) (unsorted tail): photons [i0, i1) of the item starting at slot
// ib.  Returns whether it is a tail item.
__device__ __forceinline__ bool convert_item(long long b0, long long b1, long long t0, long long t1,
                                             long long local, long long& ib, long long& i0,
                                             long long& i1) {
  const long long nb = (b1 - b0 + kPhChunk - 1) / kPhChunk;
  if (local < nb) {
    ib = i0 = b0 + local * kPhChunk;
    i1 = i0 + kPhChunk < b1 ? i0 + kPhChunk : b1;
    return false;
  }
  ib = (t0 & ~(long long)(kKeyRun - 1)) + (local - nb) * kPhChunk;
  i0 = ib > t0 ? ib : t0;
  i1 = ib + kPhChunk < t1 ? ib + kPhChunk : t1;
  return true;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Bit 4q + j set where byte j of word q of a 16-byte key run equals key.
__device__ __forceinline__ uint32_t key_matches(u32x4 kv, uint32_t key) {
  const uint32_t w[4] = {kv.x, kv.y, kv.z, kv.w};
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < 4; ++j) m |= (((w[q] >> (8 * j)) & 0xFFu) == key ? 1u : 0u) << (4 * q + j);
  return m;
}

constexpr int kConvGroup = kBlock / 64;  // waves of a conversion workgroup, each with its own list
constexpr int kDueFlush = 128;           // listed due photons that start a conversion round
constexpr int kConvPerGroup = 32;        // conversion items a workgroup takes at least
constexpr int kDueList = 2 * kPhChunk;   // a wave's list: below kDueFlush, plus one item
static_assert(kDueList >= kDueFlush - 1 + kPhChunk, "a wave's list holds a flush's worth and an item");

// The due mask of one lane's kKeyRun photons of conversion item `local` of a
// gap whose due ranges are [rb0, rb1) and [rt0, rt1): bit b set when photon
// ib + 16 lane + b converts this step.  Bucket items are all due; tail
// photons are found by their one-byte keys while the step is within
// kFarKey - 1 steps of the last sort (keyed), else by their conversion steps.
struct ConvRun {
  long long ib;  // first slot of the item
  uint32_t in;   // the lane's photons inside the item's range
  bool tail;
};

__device__ __forceinline__ ConvRun conv_run(long long rb0, long long rb1, long long rt0, long long rt1,
                                            long long local, int lane) {
  ConvRun r;
  long long i0, i1;
  r.tail = convert_item(rb0, rb1, rt0, rt1, local, r.ib, i0, i1);
  const long long s0 = r.ib + (long long)lane * kKeyRun;
  const long long lo = i0 - s0, hi = i1 - s0;
  const int a = lo < 0 ? 0 : (lo > kKeyRun ? kKeyRun : (int)lo);
  const int e = hi < 0 ? 0 : (hi > kKeyRun ? kKeyRun : (int)hi);
  r.in = ((1u << e) - 1u) & ~((1u << a) - 1u);
  return r;
}

// Photons due at the end of the step become pairs at their conversion
// points, moving along the photon (section 2).  Each wave works apart: it
// takes a contiguous range of the plan's conversion items (its workgroup's
// range cut in four); for each item every lane tests kKeyRun consecutive
// photons (one 16-byte load of keys), and a wave scan of the lanes' counts
// appends the item's due photons to the wave's LDS list (offsets from the
// first listed item's slot).  Once the list holds two rounds of the wave
// (kDueFlush), or the gap's items end, lane 0 reserves the list's pair slots
// with one atomic and the lanes convert it one photon each; the list has
// room for kDueFlush - 1 photons and a whole item.  The keys of the wave's
// next item of the same gap are requested before the current item is
// tested.  No workgroup barrier.
template <typename T>
__device__ void convert_role(GapDev* __restrict__ gaps, const long long* __restrict__ pwi, int B,
                             int vb, int nvb, uint32_t* s_due) {
  static_assert(kPhChunk == 64 * kKeyRun, "an item is one key run per lane");
  const int lane = lane_id();
  // the wave's index, uniform
  const int v = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  uint32_t* due = s_due + v * kDueList;
  const long long total = pwi[B];
  // only as many workgroups as hold kConvPerGroup items each (a multiple of
  // the 8 XCDs, at most the role's blocks) take part: in small steps the
  // others' start-up (finding their gap, its descriptor and due ranges)
  // would cost more than the items they would take
  long long nact = (total + kConvPerGroup - 1) / kConvPerGroup;
  nact = (nact + 7) / 8 * 8;
  if (nact > nvb) nact = nvb;
  if (vb >= nact) return;
  long long x0, x1;
  xcd_range(total, x0, x1, vb, (int)nact);
  const long long per = (x1 - x0 + kConvGroup - 1) / kConvGroup;
  long long w = x0 + (long long)v * per;
  w = w < x1 ? w : x1;
  const long long w1 = w + per < x1 ? w + per : x1;
  while (w < w1) {
    const int g = find_gap(pwi, B, w);
    const long long wend = pwi[g + 1] < w1 ? pwi[g + 1] : w1;
    GapDev* __restrict__ G = gaps + g;
    if (G->status != PIC_OK) { w = wend; continue; }
    const int pb = G->phbuf, buf = G->buf;
    const int stepn = (int)G->step;
    const long long wg0 = pwi[g];
    long long rb0, rb1, rt0, rt1;  // the gap's due ranges, read once
    photon_ranges(G, rb0, rb1, rt0, rt1);
    const long long kstep = G->step - G->ph_base;
    const bool keyed = kstep < kFarKey;
    gptr<const uint8_t> phk = glb<const uint8_t>((void*)G->ph_key);
    gptr<const int32_t> phs = glb<const int32_t>((void*)G->ph_step[pb]);
    gptr<const PhotonRec> phr = glb<const PhotonRec>((void*)G->ph_rec[pb]);
    gptr<int32_t> cell0 = glb(G->cell[buf][0]), cell1 = glb(G->cell[buf][1]);
    gptr<T> off0 = glb<T>(G->off[buf][0]), off1 = glb<T>(G->off[buf][1]);
    gptr<T> p0 = glb<T>(G->p[buf][0]), p1 = glb<T>(G->p[buf][1]);
    gptr<uint64_t> id0 = glb(G->id[buf][0]), id1 = glb(G->id[buf][1]);
    const unsigned long long ne0 = G->n[0], ne1 = G->n[1];
    const unsigned long long cap = (unsigned long long)G->slots;
    const int K = G->K;
    const long long mask = G->one - 1;
    const T inv_scale = (T)(1.0 / (double)G->one);
    const T pchild = (T)G->pchild;
    const bool evmap = G->evmap != nullptr;
    // the keys of a tail item's lane run (s0 is a multiple of kKeyRun below
    // the tail's end: the run lies in the key array, sized up to a multiple of
    // kKeyRun); zero for bucket items and unkeyed tails
    auto keys_of = [&](const ConvRun& r) {
      u32x4 kv = {0u, 0u, 0u, 0u};
      if (r.tail && keyed && r.in != 0u) kv = *(gptr<const u32x4>)(phk + r.ib + (long long)lane * kKeyRun);
      return kv;
    };
    // the wave's list: `pending` due photons at offsets from slot `lb`
    uint32_t pending = 0;
    long long lb = 0;
    auto convert_list = [&]() {
      __builtin_amdgcn_wave_barrier();  // the list is complete before any lane reads it
      unsigned long long base = 0;
      if (lane == 0) base = reserve_pairs(G, pending);
      base = __shfl(base, 0, 64);
#pragma unroll 1
      for (uint32_t q = (uint32_t)lane; q < pending; q += 64) {
        const long long i = lb + (long long)due[q];
        const u64x2 pr = get_photon(phr, i);
        const long long X = (long long)pr.x;
        const uint64_t ch = pr.y;
        const int cc = (int)(X >> K);
        const T offn = (T)(X & mask) * inv_scale;
        const T pc = (ch & 1u) ? pchild : -pchild;
        const uint64_t child = ch & ~(uint64_t)1;
        const unsigned long long se = ne0 + base + q, sp = ne1 + base + q;
        if (se < cap) { cell0[se] = cc; off0[se] = offn; p0[se] = pc; id0[se] = child; }
        if (sp < cap) { cell1[sp] = cc; off1[sp] = offn; p1[sp] = pc; id1[sp] = child | 1u; }
        if (evmap) count_pairs(G, (long long)stepn, cc, 1ull);
      }
      __builtin_amdgcn_wave_barrier();  // the list is read before it is rewritten
      pending = 0;
    };
    ConvRun r = conv_run(rb0, rb1, rt0, rt1, w - wg0, lane);
    u32x4 kv = keys_of(r);
    for (long long x = w; x < wend; ++x) {
      // this item's due photons
      uint32_t m;
      if (!r.tail) m = r.in;  // the bucket of this step: all due
      else if (keyed) m = key_matches(kv, (uint32_t)kstep) & r.in;
      else {
        m = 0u;
        const long long s0 = r.ib + (long long)lane * kKeyRun;
#pragma unroll
        for (int b = 0; b < kKeyRun; ++b)
          if ((r.in >> b) & 1u) m |= (phs[s0 + b] == stepn ? 1u : 0u) << b;
      }
      const long long ib = r.ib;
      // the next item's keys, requested now
      if (x + 1 < wend) {
        r = conv_run(rb0, rb1, rt0, rt1, x + 1 - wg0, lane);
        kv = keys_of(r);
      }
      const uint32_t c = (uint32_t)__popc(m);
      const uint32_t incl = (uint32_t)wave_incl_scan_dpp((int)c);
      const uint32_t cnt = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)incl, 63, 64));
      if (cnt > 0) {  // uniform (the list holds it: pending < kDueFlush, cnt <= kPhChunk)
        if (pending == 0) lb = ib;
        uint32_t pos = pending + incl - c;
        const uint32_t off = (uint32_t)(ib - lb);
        while (m) {
          const int b = __ffs(m) - 1;
          m &= m - 1u;
          due[pos++] = off + (uint32_t)(lane * kKeyRun + b);
        }
        pending += cnt;
      }
      // convert once the list holds two rounds of the wave, and at the end
      // of the gap's items
      if (pending >= (uint32_t)kDueFlush || (pending > 0u && x + 1 == wend)) convert_list();
    }
    w = wend;
  }
}

// ------------------------------------------------------------ plans
// Work-item prefixes of the next launches: particle chunks per gap (both
// species), due-photon chunks per gap, and chunks of the whole photon store
// (for its re-sort); frozen gaps get none.
struct PlanIn {
  bool ok;
  int table_len, ph_age;
  unsigned long long n0, n1, n_ph, body_n;
  long long step, ph_base, ph_cap;
  const int32_t* bucket;
};

__device__ __forceinline__ PlanIn plan_in(const GapDev* G) {
  PlanIn p;
  p.ok = G->status == PIC_OK;
  p.table_len = G->table_len;
  p.n0 = G->n[0];
  p.n1 = G->n[1];
  p.n_ph = G->n_ph;
  p.body_n = G->ph_body_n;
  p.step = G->step;
  p.ph_base = G->ph_base;
  p.ph_age = G->ph_age;
  p.ph_cap = G->ph_cap;
  p.bucket = G->ph_bucket;
  return p;
}

__device__ __forceinline__ void plan_items(const PlanIn& p, long long& a, long long& b, long long& c) {
  a = b = c = 0;
  if (!p.ok) return;
  a = ((long long)p.n0 + kChunk - 1) / kChunk + ((long long)p.n1 + kChunk - 1) / kChunk;
  long long b0 = 0, b1 = 0;
  const long long k = p.step - p.ph_base;
  if (p.table_len > 0 && k >= 0 && k < p.table_len) {
    b0 = k == 0 ? 0 : (long long)p.bucket[k - 1];
    b1 = (long long)p.bucket[k];
  }
  b = (b1 - b0 + kPhChunk - 1) / kPhChunk + tail_items((long long)p.body_n, (long long)p.n_ph);
  if (photon_sort_due(p.table_len, p.step, p.ph_base, p.ph_age, p.n_ph, p.ph_cap))
    c = ((long long)p.n_ph + kPhChunk - 1) / kPhChunk;
}

// Exclusive prefix sums of three values over a block of up to 1024 threads
// (wave scans, then one pass over the wave totals); t* get the totals.
__device__ __forceinline__ void block_scan3(long long& a, long long& b, long long& c, long long& ta,
                                            long long& tb, long long& tc) {
  __shared__ long long s_w[3 * 16];
  const long long ia = wave_incl_scan(a), ib = wave_incl_scan(b), ic = wave_incl_scan(c);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane_id() == 63) { s_w[w] = ia; s_w[16 + w] = ib; s_w[32 + w] = ic; }
  __syncthreads();
  long long oa = 0, ob = 0, oc = 0;
  ta = tb = tc = 0;
  for (int k = 0; k < nw; ++k) {
    if (k < w) { oa += s_w[k]; ob += s_w[16 + k]; oc += s_w[32 + k]; }
    ta += s_w[k]; tb += s_w[16 + k]; tc += s_w[32 + k];
  }
  a = oa + ia - a;
  b = ob + ib - b;
  c = oc + ic - c;
}

constexpr int kPlanPer = 4;  // gaps per thread whose items a plan keeps in registers

// Writes the prefixes from the items of this thread's gaps tid*per + k.
__device__ __forceinline__ void plan_write(int B, int per, const long long (&a)[kPlanPer],
                                           const long long (&b)[kPlanPer],
                                           const long long (&c)[kPlanPer], long long* __restrict__ wi,
                                           long long* __restrict__ pwi, long long* __restrict__ qwi) {
  long long ra = 0, rb = 0, rc = 0;
#pragma unroll
  for (int k = 0; k < kPlanPer; ++k) { ra += a[k]; rb += b[k]; rc += c[k]; }
  long long ta, tb, tc;
  block_scan3(ra, rb, rc, ta, tb, tc);
#pragma unroll
  for (int k = 0; k < kPlanPer; ++k) {
    const int g = threadIdx.x * per + k;
    if (k < per && g < B) {
      wi[g] = ra; pwi[g] = rb; qwi[g] = rc;
      ra += a[k]; rb += b[k]; rc += c[k];
    }
  }
  if (threadIdx.x == 0) { wi[B] = ta; pwi[B] = tb; qwi[B] = tc; }
}

__device__ void compute_plans(GapDev* __restrict__ gaps, int B, long long* __restrict__ wi,
                              long long* __restrict__ pwi, long long* __restrict__ qwi) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (B + nt - 1) / nt;
  if (per <= kPlanPer) {
    long long a[kPlanPer], b[kPlanPer], c[kPlanPer];
#pragma unroll
    for (int k = 0; k < kPlanPer; ++k) {
      a[k] = b[k] = c[k] = 0;
      const int g = tid * per + k;
      if (k < per && g < B) plan_items(plan_in(gaps + g), a[k], b[k], c[k]);
    }
    plan_write(B, per, a, b, c, wi, pwi, qwi);
    return;
  }
  // very large batches: two passes over the gaps
  long long sa = 0, sb = 0, sc = 0;
  for (int g = tid * per; g < (tid + 1) * per && g < B; ++g) {
    long long a, b, c;
    plan_items(plan_in(gaps + g), a, b, c);
    sa += a; sb += b; sc += c;
  }
  long long ta, tb, tc;
  block_scan3(sa, sb, sc, ta, tb, tc);
  for (int g = tid * per; g < (tid + 1) * per && g < B; ++g) {
    wi[g] = sa; pwi[g] = sb; qwi[g] = sc;
    long long a, b, c;
    plan_items(plan_in(gaps + g), a, b, c);
    sa += a; sb += b; sc += c;
  }
  if (tid == 0) { wi[B] = ta; pwi[B] = tb; qwi[B] = tc; }
}

__global__ __launch_bounds__(1024) void k_plan(GapDev* __restrict__ gaps, int B,
                                               long long* __restrict__ wi,
                                               long long* __restrict__ pwi,
                                               long long* __restrict__ qwi) {
  compute_plans(gaps, B, wi, pwi, qwi);
}

// Ends a step for every gap: freeze on error, roll the counters, write the
// history row, and plan the next step.

// One gap's end of step (the push tallies are already folded into the
// descriptor); in_push: the step's emissions were drawn by the push kernel.
// Every field is read before any is written, so the reads go out together.
__device__ __forceinline__ PlanIn finalize_gap(GapDev* __restrict__ G, bool in_push) {
  const int status = G->status, nonfinite = G->nonfinite, overflow = G->overflow;
  const int slot_overflow = G->slot_overflow;
  const int emit_err = G->emit_err, table_len = G->table_len, diag_every = G->diag_every;
  const int hist_rows = G->hist_rows, n_cells = G->n_cells;
  const unsigned long long pair_next = G->pair_next, esc_next = G->esc_next;
  const unsigned long long n_ph = G->n_ph, n_ph_next = G->n_ph_next;
  const unsigned long long n0 = G->n[0], n1 = G->n[1], dead0 = G->dead[0], dead1 = G->dead[1];
  const unsigned long long live0 = G->live[0], live1 = G->live[1], pushes = G->pushes;
  const unsigned long long absorbed0 = G->absorbed[0], absorbed1 = G->absorbed[1];
  const unsigned long long inflight0 = G->inflight, created0 = G->pairs_created;
  const unsigned long long emitted0 = G->photons_emitted, escaped0 = G->photons_escaped;
  const unsigned long long push_emitted0 = G->push_emitted;
  const unsigned long long hist_count = G->hist_count, body_n = G->ph_body_n;
  const long long done = G->step, ph_base = G->ph_base;
  const int32_t* bucket = G->ph_bucket;
  const double weight = G->weight, gpair64 = G->gpair64, child_gamma64 = G->child_gamma64;
  const unsigned long long cap = (unsigned long long)G->cap;
  // energies: the weight times the exact sums of Lorentz factors
  double ke = weight * G->ke_step;
  const double lost_step = weight * G->lost_step;
  const double fe = G->fe_step, es = G->es_step;
  double lost = G->lost_energy;
  PlanIn out;
  out.ok = false;
  out.table_len = table_len;
  out.body_n = body_n;
  out.ph_base = ph_base;
  out.ph_age = G->ph_age;
  out.ph_cap = G->ph_cap;
  out.bucket = bucket;
  if (status != PIC_OK) return out;
  // what this step appended: dp pairs (in place or converted), dph photons
  // stored, de of which left the domain
  const unsigned long long dp = pair_next, dph = n_ph_next - n_ph, de = esc_next;
  const unsigned long long nn0 = n0 + dp, nn1 = n1 + dp;
  const unsigned long long nl0 = nn0 - dead0, nl1 = nn1 - dead1;
  // the capacity bounds live leptons, as at the end of a step of the
  // oracle; the slots (capacity plus the reserve absorbed leptons hold until
  // the next re-sort) and the photon store bound what can be written
  const int st = nonfinite              ? PIC_ERR_NONFINITE
               : emit_err               ? PIC_ERR_EMISSION
               : (nl0 > cap || nl1 > cap) ? PIC_ERR_CAPACITY
               : overflow               ? PIC_ERR_CAPACITY
               : slot_overflow          ? PIC_ERR_SLOTS : PIC_OK;
  if (st != PIC_OK) {
    G->status = st;
    return out;
  }
  const bool in_place = table_len == 0;
  const bool diag = done % diag_every == 0;
  const unsigned long long created = created0 + dp;
  const unsigned long long emitted = emitted0 + (in_place ? dp : dph);
  const unsigned long long escaped = escaped0 + de;
  const unsigned long long inflight = in_place ? inflight0 : inflight0 + dph - de - dp;
  lost += lost_step;
  if (de) lost += (double)de * weight * gpair64;
  if (diag && dp) ke += (double)dp * 2.0 * weight * child_gamma64;
  G->pairs_created = created;
  G->photons_emitted = emitted;
  if (in_push) G->push_emitted = push_emitted0 + (emitted - emitted0);
  G->photons_escaped = escaped;
  G->inflight = inflight;
  G->lost_energy = lost;
  G->pushes = pushes + live0 + live1;
  G->n[0] = nn0;
  G->n[1] = nn1;
  G->live[0] = nl0;
  G->live[1] = nl1;
  G->pair_next = 0;
  G->esc_next = 0;
  G->n_ph = n_ph_next;
  G->step = done + 1;
  if (diag) {
    pic_history_row r;
    r.step = done;
    r.n_minus = (int64_t)nl0;
    r.n_plus = (int64_t)nl1;
    r.n_photons = (int64_t)inflight;
    r.pairs_created = (int64_t)created;
    r.photons_emitted = (int64_t)emitted;
    r.photons_escaped = (int64_t)escaped;
    r.absorbed_minus = (int64_t)absorbed0;
    r.absorbed_plus = (int64_t)absorbed1;
    r.kinetic = ke;
    r.field = fe;
    r.photon_energy = (double)inflight * weight * gpair64;
    r.lost_energy = lost;
    r.e_mean = es / (double)n_cells;
    G->hist[hist_count % (unsigned long long)hist_rows] = r;
    G->hist_count = hist_count + 1;
    G->last = r;
  }
  out.ok = true;
  out.n0 = nn0;
  out.n1 = nn1;
  out.n_ph = n_ph_next;
  out.step = done + 1;
  return out;
}

// The order-independent sums of the step, turned into binary64 values in
// the descriptor; the limbs are cleared for the next step.  A phase of its
// own, so that the end of step below keeps its registers.
__device__ __forceinline__ void diag_values(GapDev* __restrict__ G) {
  const double ke = limbs_value(G->ke_limb);
  const double lost = limbs_value(G->lost_limb);
  const double fe = wide_value(G->fe_wide);
  const double es = wide_value(G->esp_wide) - wide_value(G->esn_wide);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    G->ke_limb[k] = 0;
    G->lost_limb[k] = 0;
  }
#pragma unroll
  for (int k = 0; k < kWideLimbs; ++k) {
    G->fe_wide[k] = 0;
    G->esp_wide[k] = 0;
    G->esn_wide[k] = 0;
  }
  G->ke_step = ke;
  G->lost_step = lost;
  G->fe_step = fe;
  G->es_step = es;
}

// The work-item prefixes of the next step from the per-gap item counts the
// finalize left in `items` (a: lepton chunks, b: due-photon chunks, c:
// photon-store chunks, B each), one block.
__device__ void plan_from_items(int B, const long long* __restrict__ items, long long* __restrict__ wi,
                                long long* __restrict__ pwi, long long* __restrict__ qwi) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (B + nt - 1) / nt;
  if (per <= kPlanPer) {
    long long a[kPlanPer], b[kPlanPer], c[kPlanPer];
#pragma unroll
    for (int k = 0; k < kPlanPer; ++k) {
      const int g = tid * per + k;
      const bool in = k < per && g < B;
      a[k] = in ? items[g] : 0;
      b[k] = in ? items[B + g] : 0;
      c[k] = in ? items[2 * B + g] : 0;
    }
    plan_write(B, per, a, b, c, wi, pwi, qwi);
    return;
  }
  // very large batches: two passes over the counts
  long long sa = 0, sb = 0, sc = 0;
  for (int g = tid * per; g < (tid + 1) * per && g < B; ++g) {
    sa += items[g];
    sb += items[B + g];
    sc += items[2 * B + g];
  }
  long long ta, tb, tc;
  block_scan3(sa, sb, sc, ta, tb, tc);
  for (int g = tid * per; g < (tid + 1) * per && g < B; ++g) {
    wi[g] = sa; pwi[g] = sb; qwi[g] = sc;
    sa += items[g];
    sb += items[B + g];
    sc += items[2 * B + g];
  }
  if (tid == 0) { wi[B] = ta; pwi[B] = tb; qwi[B] = tc; }
}

// ------------------------------------------------------------------ fold
// The striped push tallies of the step: 32 lanes sum the stripes of one
// (gap, accumulator) pair, clear them, and add the sum to the descriptor
// with one atomic (accumulators 0-1 are binary64 energies, 2-3 counts of
// absorbed electrons and positrons).
__device__ void fold_role(GapDev* __restrict__ gaps, int B, unsigned long long* __restrict__ stripes,
                          int vb) {
  const int pair = vb * (kBlock / kStripes) + (int)threadIdx.x / kStripes;
  const int st = (int)threadIdx.x % kStripes;
  const int a = pair & 3;
  const int nl = a < 2 ? 4 : 1;  // energy limbs, or one count
  unsigned long long v[4] = {0, 0, 0, 0};
  if (pair < 4 * B) {
    gptr<unsigned long long> slot = glb<unsigned long long>((void*)stripe_slot(stripes, pair >> 2, a, st));
    for (int k = 0; k < nl; ++k) {
      v[k] = slot[k];
      slot[k] = 0ull;
    }
  }
#pragma unroll
  for (int d = kStripes / 2; d >= 1; d >>= 1)  // within each group of kStripes lanes
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += __shfl_xor(v[k], d, 64);
  if (st != 0 || pair >= 4 * B) return;
  GapDev* __restrict__ G = gaps + (pair >> 2);
  if (a < 2) {
    unsigned long long* acc = a == 0 ? G->ke_limb : G->lost_limb;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (v[k]) atomicAdd(acc + k, v[k]);
  } else if (v[0]) {
    const int s = a - 2;
    atomicAdd(&G->absorbed[s], v[0]);
    atomicAdd(&G->dead[s], v[0]);
  }
}

// Everything of a step between the push and the finalize: the Ampere
// update (blocks [0, n_field)), the conversions (next n_conv blocks), the
// emission of the listed chunks (next n_emit blocks) and the fold of the
// push tallies (the rest) are independent of each other.  Blocks start in
// index order, so the emission role, idle in steps that emit inside the
// push, comes after the conversions.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_post(GapDev* __restrict__ gaps,
                                                 const long long* __restrict__ cwi,
                                                 const long long* __restrict__ wi,
                                                 const long long* __restrict__ pwi, int B,
                                                 int n_field, int n_emit, int n_conv,
                                                 const int32_t* __restrict__ emit_cnt,
                                                 const uint32_t* __restrict__ emit_ent,
                                                 const uint32_t* __restrict__ wg_emit,
                                                 unsigned long long* __restrict__ stripes) {
  __shared__ double s_red[8];
  __shared__ unsigned long long s_base[1];
  __shared__ int s_nb[kBlock];
  __shared__ int s_tmp[kBlock / 64];
  // the emission role's prefix of the push workgroups' emitters, or the
  // conversion role's lists of due photons, one per wave (a block takes one role)
  __shared__ uint32_t s_buf[kPushGrid > kConvGroup * kDueList ? kPushGrid : kConvGroup * kDueList];
  const int b = blockIdx.x;
  if (b < n_field) field_role(gaps, cwi, B, b, s_red);
  else if (b < n_field + n_conv)
    convert_role<T>(gaps, pwi, B, b - n_field, n_conv, s_buf);
  else if (b < n_field + n_conv + n_emit)
    emit_role<T>(gaps, wi, B, emit_cnt, emit_ent, wg_emit, b - n_field - n_conv, n_emit, s_buf,
                 s_base, s_nb, s_tmp);
  else fold_role(gaps, B, stripes, b - n_field - n_conv - n_emit);
}

// The end of a step, one gap per wave: the wave's gap index is uniform, so
// the descriptor's fields are read with scalar loads, and the gaps are ended
// on as many compute units as there are gaps / 4 (one workgroup ending every
// gap was bound by one unit's scattered loads).  Each gap's item counts of
// the next step go to `items`; k_plan_scan turns them into the prefixes.
__global__ __launch_bounds__(kBlock) void k_finalize(GapDev* __restrict__ gaps, int B,
                                                     const long long* __restrict__ wi,
                                                     long long* __restrict__ items) {
  const int g = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (kBlock / 64) + ((int)threadIdx.x >> 6));
  if (g >= B || lane_id() != 0) return;
  // the step's plan, read before k_plan_scan writes the next one
  const bool in_push = wi[B] < gaps->emit_split;
  GapDev* __restrict__ G = gaps + g;
  diag_values(G);
  long long a, b, c;
  plan_items(finalize_gap(G, in_push), a, b, c);
  items[g] = a;
  items[B + g] = b;
  items[2 * B + g] = c;
}

__global__ __launch_bounds__(1024) void k_plan_scan(int B, const long long* __restrict__ items,
                                                    long long* __restrict__ wi,
                                                    long long* __restrict__ pwi,
                                                    long long* __restrict__ qwi) {
  plan_from_items(B, items, wi, pwi, qwi);
}

// ------------------------------------------------------------------ sort
// Lanes holding the same key in a row of a wave form a run; the first lane
// of a run (its head) does one atomic for the whole run.
__device__ __forceinline__ void wave_runs(int cv, int& head_lane, int& run_len) {
  const int lane = lane_id();
  const int prev = __shfl_up(cv, 1, 64);
  const bool head = lane == 0 || cv != prev;
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  head_lane = 63 - __clzll(heads & upto);
  const unsigned long long above = lane == 63 ? 0ull : (heads & ~upto);
  const int next = above ? (__ffsll((long long)above) - 1) : 64;
  run_len = head ? next - lane : 0;
}

// Buckets of the lepton sort of a gap of nc cells: groups of 2^kSortShift
// cells.  The push needs a chunk's leptons within a short span of cells, not
// in cell order inside a group, and groups make each bucket's run of
// destination slots 2^kSortShift times longer, so the scatter's stores
// coalesce.
__device__ __forceinline__ int sort_buckets(int nc) {
  return (nc + (1 << kSortShift) - 1) >> kSortShift;
}

__global__ __launch_bounds__(kBlock) void k_sort_zero(GapDev* __restrict__ gaps,
                                                      const long long* __restrict__ cwi, int B) {
  const int g = find_gap(cwi, B, blockIdx.x);
  GapDev* __restrict__ G = gaps + g;
  const long long c0 = (blockIdx.x - cwi[g]) * (long long)kCellChunk;
  const int nk = sort_buckets(G->n_cells);
  for (int k = threadIdx.x; k < kCellChunk; k += kBlock) {
    const long long c = c0 + k;
    if (c >= nk) break;
    G->sort_cnt[0][c] = 0;
    G->sort_cnt[1][c] = 0;
  }
  if (blockIdx.x == cwi[g] && threadIdx.x == 0) { G->sorted_n[0] = 0; G->sorted_n[1] = 0; }
}

// Between full re-sorts, the leptons of a species appended since the last
// one (slots body_n .. n) are sorted by cell group among themselves every
// kTailEvery steps, where they are many: their chunks then fit the push's
// LDS tile instead of depositing through global atomics.  Nothing moves
// out of the tail and nothing is dropped; dead leptons keep their slots in
// an extra bucket after the last group.
// A species' tail is sorted when its gap is wider than the push's tile (in
// a narrower gap every chunk fits the tile anyway) and the tail holds at
// least a chunk and a 32nd of the species.
__device__ __forceinline__ bool tail_sorted(const GapDev* G, int s) {
  const unsigned long long n = G->n[s], body = G->body_n[s];
  const unsigned long long tail = n - body;
  return G->status == PIC_OK && G->n_cells > kTile - 8 && tail >= (unsigned long long)kChunk &&
         tail * 32 >= n;
}

// Chunks of the tail sort for species s of gap G: kChunk leptons each from
// slot body_n[s].
__device__ __forceinline__ long long tail_chunks(const GapDev* G, int s) {
  if (!tail_sorted(G, s)) return 0;
  return ((long long)(G->n[s] - G->body_n[s]) + kChunk - 1) / kChunk;
}

// Work-item prefix of the tail sort (species 0 then 1 per gap), one block.
__global__ __launch_bounds__(1024) void k_tail_plan(GapDev* __restrict__ gaps, int B,
                                                    long long* __restrict__ twi) {
  __shared__ long long s_sum[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (B + nt - 1) / nt;
  long long loc = 0;
  for (int g = tid * per; g < (tid + 1) * per && g < B; ++g)
    loc += tail_chunks(gaps + g, 0) + tail_chunks(gaps + g, 1);
  s_sum[tid] = loc;
  __syncthreads();
  for (int d = 1; d < nt; d <<= 1) {
    const long long y = tid >= d ? s_sum[tid - d] : 0;
    __syncthreads();
    s_sum[tid] += y;
    __syncthreads();
  }
  long long run = s_sum[tid] - loc;
  for (int g = tid * per; g < (tid + 1) * per && g < B; ++g) {
    twi[g] = run;
    run += tail_chunks(gaps + g, 0) + tail_chunks(gaps + g, 1);
  }
  if (tid == nt - 1) twi[B] = s_sum[nt - 1];
}

__global__ __launch_bounds__(kBlock) void k_tail_zero(GapDev* __restrict__ gaps,
                                                      const long long* __restrict__ cwi, int B) {
  const int g = find_gap(cwi, B, blockIdx.x);
  GapDev* __restrict__ G = gaps + g;
  const long long c0 = (blockIdx.x - cwi[g]) * (long long)kCellChunk;
  const int nk = sort_buckets(G->n_cells);
  for (int s = 0; s < 2; ++s) {
    if (!tail_sorted(G, s)) continue;
    // the groups and, after them, the dead bucket
    for (int k = threadIdx.x; k < kCellChunk; k += kBlock) {
      const long long c = c0 + k;
      if (c > nk) break;
      G->sort_cnt[s][c] = 0;
    }
  }
}

// Counting sort of the leptons by cell group (sort_buckets).  PASS 0 counts,
// PASS 1 (after the scan turned the counts into bucket starts) moves each
// live lepton to the other buffer.  A chunk whose groups span at most
// kSortTile counts in an LDS histogram first and touches each global bucket
// once; wider chunks (leptons appended since the last sort) use one global
// atomic per run of equal groups.
// An iteration takes up to SortPer consecutive chunks of one (gap, species),
// so the barriers and the round trip of the bucket atomics are shared.
// TAIL sorts only the appended leptons of the species that have many
// (tail_sorted), into the same slots of the other buffer.
template <int PASS, typename T, bool TAIL>
__global__ __launch_bounds__(kBlock) void k_sort_pass(GapDev* __restrict__ gaps,
                                                      const long long* __restrict__ wi, int B) {
  constexpr int kPer = SortPer<PASS>::value;
  constexpr int kN = kItems * kPer;  // leptons per thread per iteration
  __shared__ int32_t s_hist[kSortTile];
  __shared__ int s_red[8];
  const long long total = wi[B];
  long long w0, w1;
  xcd_range(total, w0, w1);
  const int lane = lane_id();
  for (long long w = w0; w < w1;) {
    const int g = find_gap(wi, B, w);
    GapDev* __restrict__ G = gaps + g;
    // chunks of species 0, then 1: all slots (full sort) or the tail from
    // slot body_n (tail sort, whose prefix holds only the tails it sorts)
    const long long chunks0 = TAIL ? tail_chunks(G, 0) : ((long long)G->n[0] + kChunk - 1) / kChunk;
    const long long local = w - wi[g];
    const int s = local < chunks0 ? 0 : 1;
    // chunks [w, wn): the same species of the same gap, inside this range
    // (w lies below both ends, so at least one chunk is taken)
    const long long seg_end = s == 0 ? wi[g] + chunks0 : wi[g + 1];
    long long wn = w + kPer;
    if (wn > seg_end) wn = seg_end;
    if (wn > w1) wn = w1;
    const long long nch = wn - w;
    w = wn;
    if (G->status != PIC_OK) continue;
    const long long lo = TAIL ? (long long)G->body_n[s] : 0;  // first slot taking part
    const int buf = G->buf;
    const int nc = G->n_cells;
    const long long i0 = lo + (s == 0 ? local : local - chunks0) * kChunk;
    const long long nS = (long long)G->n[s];
    const long long i1 = i0 + nch * kChunk < nS ? i0 + nch * kChunk : nS;
    gptr<int32_t> cnt = glb(G->sort_cnt[s]);
    gptr<const int32_t> cin = glb<const int32_t>((void*)G->cell[buf][s]);
    const int nk = sort_buckets(nc);
    // the whole lepton state is requested at once (slots past the end read
    // the first slot and are discarded), before any store of this chunk
    int cvs[kN];
    T ov[kN], pv[kN];
    uint64_t idv[kN];
#pragma unroll
    for (int j = 0; j < kN; ++j) {
      const long long i = i0 + threadIdx.x + (long long)j * kBlock;
      const bool in = i < i1;
      const long long ii = in ? i : i0;
      const int cv = cin[ii];
      if (PASS == 1) {
        ov[j] = glb<const T>(G->off[buf][s])[ii];
        pv[j] = glb<const T>(G->p[buf][s])[ii];
        idv[j] = glb<const uint64_t>((void*)G->id[buf][s])[ii];
      }
      // kDead marks what takes no part: slots outside the range and, in the
      // full sort, dead leptons; the tail sort keeps those in a bucket after
      // the last group (cell n_cells)
      cvs[j] = in ? (TAIL && cv == kDead ? nc : cv) : kDead;
    }
    // the bucket of a taking part lepton: its cell's group, or the dead bucket
    auto key = [&](int cv) { return TAIL && cv == nc ? nk : cv >> kSortShift; };
    int mn = INT32_MAX, mx = INT32_MIN;
#pragma unroll
    for (int j = 0; j < kN; ++j)
      if (cvs[j] != kDead) { mn = min(mn, key(cvs[j])); mx = max(mx, key(cvs[j])); }
    block_minmax(mn, mx, s_red);
    if (mx < mn) continue;  // no live lepton in this chunk (uniform)
    long long dst[kN];
    if (mx - mn < kSortTile) {
      const int span = mx - mn + 1;
      for (int k = threadIdx.x; k < span; k += kBlock) s_hist[k] = 0;
      __syncthreads();
      // sorted leptons share cells, so the lanes of a wave form long runs:
      // one LDS atomic per run, the rank within it from the lane
      int rank[kN];
#pragma unroll
      for (int j = 0; j < kN; ++j) {
        const int kv = cvs[j] != kDead ? key(cvs[j]) : kDead;
        int head_lane, run_len;
        wave_runs(kv, head_lane, run_len);
        int r = 0;
        if (run_len > 0 && kv != kDead) r = atomicAdd(&s_hist[kv - mn], run_len);
        rank[j] = __shfl(r, head_lane, 64) + (lane - head_lane);
      }
      __syncthreads();
      for (int k = threadIdx.x; k < span; k += kBlock) {
        const int c = s_hist[k];
        if (c == 0) continue;
        if (PASS == 0)
          __hip_atomic_fetch_add(cnt + mn + k, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
          s_hist[k] = __hip_atomic_fetch_add(cnt + mn + k, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (PASS == 0) continue;  // the next chunk's block_minmax orders the LDS reuse
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kN; ++j)
        dst[j] = cvs[j] != kDead ? (long long)s_hist[key(cvs[j]) - mn] + rank[j] : 0;
    } else {
#pragma unroll
      for (int j = 0; j < kN; ++j) {
        const int kv = cvs[j] != kDead ? key(cvs[j]) : kDead;
        int head_lane, run_len;
        wave_runs(kv, head_lane, run_len);
        int b = 0;
        if (run_len > 0 && kv != kDead)
          b = __hip_atomic_fetch_add(cnt + kv, run_len, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (PASS == 1) {
          b = __shfl(b, head_lane, 64);
          dst[j] = (long long)b + (lane - head_lane);
        }
      }
      if (PASS == 0) continue;
    }
    const int nb = buf ^ 1;
    gptr<int32_t> cout = glb(G->cell[nb][s]);
    gptr<T> oout = glb<T>(G->off[nb][s]);
    gptr<T> pout = glb<T>(G->p[nb][s]);
    gptr<uint64_t> iout = glb(G->id[nb][s]);
#pragma unroll
    for (int j = 0; j < kN; ++j) {
      if (cvs[j] == kDead) continue;
      const long long d = lo + dst[j];
      cout[d] = TAIL && cvs[j] == nc ? kDead : cvs[j];
      oout[d] = ov[j];
      pout[d] = pv[j];
      iout[d] = idv[j];
    }
  }
}

// Exclusive scan of n int32 counts in place by one 1024-thread block; returns the total.
__device__ long long block_scan_counts(int32_t* __restrict__ cnt, int n, long long* s_sum) {
  // thread t takes a contiguous run of entries, a multiple of 4 long, read
  // and written as 16-byte vectors where a whole vector lies below n (the
  // rest one by one); runs are added up within waves (DPP-free shuffles
  // suffice here) and across the block through LDS
  typedef int i32x4 __attribute__((ext_vector_type(4)));
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (((n + nt - 1) / nt) + 3) & ~3;
  const int c0 = tid * per;
  const int c1 = c0 + per < n ? c0 + per : n;
  long long loc = 0;
  for (int c = c0; c < c1; c += 16) {
    i32x4 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int cq = c + 4 * q;
      v[q] = cq + 4 <= c1 ? *(const i32x4*)(cnt + cq) : i32x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int cq = c + 4 * q;
      if (cq + 4 <= c1) loc += (long long)v[q].x + v[q].y + v[q].z + v[q].w;
      else
        for (int e = cq; e < c1 && e < cq + 4; ++e) loc += cnt[e];
    }
  }
  const long long incl = wave_incl_scan(loc);
  const int w = tid >> 6, nw = nt >> 6;
  if (lane_id() == 63) s_sum[w] = incl;
  __syncthreads();
  long long pre = 0, tot = 0;
  for (int k = 0; k < nw; ++k) {
    const long long t = s_sum[k];
    if (k < w) pre += t;
    tot += t;
  }
  long long run = pre + incl - loc;
  for (int c = c0; c < c1; c += 4) {
    if (c + 4 <= c1) {
      const i32x4 v = *(const i32x4*)(cnt + c);
      i32x4 o;
      o.x = (int32_t)run; run += v.x;
      o.y = (int32_t)run; run += v.y;
      o.z = (int32_t)run; run += v.z;
      o.w = (int32_t)run; run += v.w;
      *(i32x4*)(cnt + c) = o;
    } else {
      for (int e = c; e < c1; ++e) {
        const int v = cnt[e];
        cnt[e] = (int32_t)run;
        run += v;
      }
    }
  }
  return tot;
}

// Exclusive scan of the per-cell counts of one (gap, species) in place (the
// tail sort also scans its dead bucket).
template <bool TAIL>
__global__ __launch_bounds__(1024) void k_sort_scan(GapDev* __restrict__ gaps, int B) {
  __shared__ long long s_sum[1024];
  const int g = blockIdx.x >> 1, s = blockIdx.x & 1;
  GapDev* __restrict__ G = gaps + g;
  if (G->status != PIC_OK) return;
  if (TAIL && !tail_sorted(G, s)) return;  // (tail_sorted also requires PIC_OK)
  const long long tot = block_scan_counts(G->sort_cnt[s], sort_buckets(G->n_cells) + (TAIL ? 1 : 0), s_sum);
  if (!TAIL && threadIdx.x == blockDim.x - 1) G->sorted_n[s] = (unsigned long long)tot;
}

// The sorted tails back from the other buffer into their slots (wi is the
// tail sort's prefix).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tail_copy(GapDev* __restrict__ gaps,
                                                      const long long* __restrict__ wi, int B) {
  const long long total = wi[B];
  long long w0, w1;
  xcd_range(total, w0, w1);
  for (long long w = w0; w < w1; ++w) {
    const int g = find_gap(wi, B, w);
    GapDev* __restrict__ G = gaps + g;
    const long long chunks0 = tail_chunks(G, 0);
    const long long local = w - wi[g];
    const int s = local < chunks0 ? 0 : 1;
    const long long i0 = (long long)G->body_n[s] + (s == 0 ? local : local - chunks0) * kChunk;
    const long long nS = (long long)G->n[s];
    const long long i1 = i0 + kChunk < nS ? i0 + kChunk : nS;
    const int buf = G->buf, nb = buf ^ 1;
    for (long long i = i0 + threadIdx.x; i < i1; i += kBlock) {
      G->cell[buf][s][i] = G->cell[nb][s][i];
      ((T*)G->off[buf][s])[i] = ((const T*)G->off[nb][s])[i];
      ((T*)G->p[buf][s])[i] = ((const T*)G->p[nb][s])[i];
      G->id[buf][s][i] = G->id[nb][s][i];
    }
  }
}

// ---- photon store: counting sort by conversion step, dropping the photons
// that converted or escaped.
// The photon store is sorted by a re-sort only when photon_sort_due says so
// (the plan of the step gave its chunks to the sort on the same condition).
__global__ __launch_bounds__(kBlock) void k_ph_zero(GapDev* __restrict__ gaps, int B) {
  GapDev* __restrict__ G = gaps + blockIdx.x;
  const bool due = G->status == PIC_OK &&
                   photon_sort_due(G->table_len, G->step, G->ph_base, G->ph_age, G->n_ph, G->ph_cap);
  __syncthreads();  // every thread has read the state before thread 0 writes the flag
  if (threadIdx.x == 0) {
    G->ph_due = due ? 1 : 0;
    G->ph_sorted = 0;
  }
  if (!due) return;
  for (int k = threadIdx.x; k <= G->table_len; k += kBlock) G->ph_bucket[k] = 0;
}

// Counting sort of the photon store by conversion step (key = step - now),
// dropping photons that converted or escaped (key < 0).  A workgroup takes a
// contiguous range of one gap's store and counts the keys below kPhBins in
// an LDS histogram, touching each of those global buckets once per range;
// the rare keys beyond (conversion tables longer than kPhBins steps, whose
// far entries hold a vanishing share of the photons) take one global
// atomic per run of equal keys.
template <int PASS>
__global__ __launch_bounds__(kBlock) void k_ph_pass(GapDev* __restrict__ gaps,
                                                    const long long* __restrict__ qwi, int B) {
  __shared__ int32_t s_hist[kPhBins];
  const int lane = lane_id();
  const long long total = qwi[B];
  long long w0, w1;
  xcd_range(total, w0, w1);
  for (long long w = w0; w < w1;) {
    const int g = find_gap(qwi, B, w);
    const long long wend = qwi[g + 1] < w1 ? qwi[g + 1] : w1;
    GapDev* __restrict__ G = gaps + g;
    const long long nP = (long long)G->n_ph;
    const long long p0 = (w - qwi[g]) * kPhChunk;
    const long long p1 = (wend - qwi[g]) * kPhChunk < nP ? (wend - qwi[g]) * kPhChunk : nP;
    w = wend;
    if (G->status != PIC_OK || G->table_len == 0 || !G->ph_due) continue;
    const int pb = G->phbuf;
    const long long stepn = G->step;
    const int L = G->table_len;
    const int nh = L < kPhBins ? L : kPhBins;  // keys counted in LDS
    gptr<int32_t> bucket = glb(G->ph_bucket);
    gptr<const int32_t> sin = glb<const int32_t>((void*)G->ph_step[pb]);
    for (int k = threadIdx.x; k < nh; k += kBlock) s_hist[k] = 0;
    __syncthreads();
    // one LDS atomic per run of equal keys in a wave (the sorted body of
    // the store holds long runs); far keys count in the global buckets
    for (long long r = p0; r < p1; r += kPhUnroll * kBlock) {
      int key[kPhUnroll];
#pragma unroll
      for (int k = 0; k < kPhUnroll; ++k) {
        const long long i = r + threadIdx.x + (long long)k * kBlock;
        const long long cs = i < p1 ? (long long)sin[i] : (long long)INT32_MIN;
        key[k] = cs >= stepn ? (int)(cs - stepn) : -1;
      }
#pragma unroll
      for (int k = 0; k < kPhUnroll; ++k) {
        int head_lane, run_len;
        wave_runs(key[k], head_lane, run_len);
        if (run_len > 0 && key[k] >= 0) {
          if (key[k] < nh) atomicAdd(&s_hist[key[k]], run_len);
          else if (PASS == 0)
            __hip_atomic_fetch_add(bucket + key[k], run_len, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nh; k += kBlock) {
      const int c = s_hist[k];
      if (c == 0) continue;
      if (PASS == 0)
        __hip_atomic_fetch_add(bucket + k, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else
        s_hist[k] = __hip_atomic_fetch_add(bucket + k, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (PASS == 1) {
      __syncthreads();
      for (long long r = p0; r < p1; r += kPhUnroll * kBlock) {
        int key[kPhUnroll];
        u64x2 rv[kPhUnroll];
#pragma unroll
        for (int k = 0; k < kPhUnroll; ++k) {
          const long long i = r + threadIdx.x + (long long)k * kBlock;
          const long long cs = i < p1 ? (long long)sin[i] : (long long)INT32_MIN;
          key[k] = cs >= stepn ? (int)(cs - stepn) : -1;
        }
        // the kept photons' state is requested before the ranks are taken
#pragma unroll
        for (int k = 0; k < kPhUnroll; ++k) {
          const long long i = r + threadIdx.x + (long long)k * kBlock;
          rv[k] = u64x2{0ull, 0ull};
          if (key[k] >= 0) rv[k] = get_photon(glb<const PhotonRec>((void*)G->ph_rec[pb]), i);
        }
#pragma unroll
        for (int k = 0; k < kPhUnroll; ++k) {
          int head_lane, run_len;
          wave_runs(key[k], head_lane, run_len);
          int b = 0;
          if (run_len > 0 && key[k] >= 0) {
            if (key[k] < nh) b = atomicAdd(&s_hist[key[k]], run_len);
            else
              b = __hip_atomic_fetch_add(bucket + key[k], run_len, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
          }
          b = __shfl(b, head_lane, 64);
          if (key[k] < 0) continue;
          const long long dst = (long long)b + (lane - head_lane);
          *(gptr<u64x2>)(glb(G->ph_rec[pb ^ 1]) + dst) = rv[k];
          G->ph_step[pb ^ 1][dst] = (int32_t)(stepn + key[k]);
        }
      }
    }
    __syncthreads();  // s_hist is read before the next range clears it
  }
}

__global__ __launch_bounds__(1024) void k_ph_scan(GapDev* __restrict__ gaps, int B) {
  __shared__ long long s_sum[1024];
  GapDev* __restrict__ G = gaps + blockIdx.x;
  if (G->status != PIC_OK || G->table_len == 0 || !G->ph_due) return;
  const long long tot = block_scan_counts(G->ph_bucket, G->table_len, s_sum);
  if (threadIdx.x == blockDim.x - 1) G->ph_sorted = (unsigned long long)tot;
}

__global__ __launch_bounds__(1024) void k_sort_finish(GapDev* __restrict__ gaps, int B,
                                                      long long* __restrict__ wi,
                                                      long long* __restrict__ pwi,
                                                      long long* __restrict__ qwi) {
  for (int g = threadIdx.x; g < B; g += blockDim.x) {
    GapDev* G = gaps + g;
    if (G->status != PIC_OK) continue;
    for (int s = 0; s < 2; ++s) {
      G->n[s] = G->sorted_n[s];
      G->live[s] = G->sorted_n[s];
      G->body_n[s] = G->sorted_n[s];
      G->dead[s] = 0;
    }
    G->buf ^= 1;
    if (G->ph_due) {
      G->n_ph = G->ph_sorted;
      G->n_ph_next = G->ph_sorted;
      G->ph_body_n = G->ph_sorted;
      G->ph_base = G->step;
      G->phbuf ^= 1;
    }
  }
  __syncthreads();
  compute_plans(gaps, B, wi, pwi, qwi);
}

// ------------------------------------------------------------------ seed
template <typename T>
__global__ __launch_bounds__(kBlock) void k_seed(GapDev* __restrict__ gaps, int g, int mode,
                                                 long long N, double p0m, double p0p,
                                                 long long base0, long long base1) {
  GapDev* __restrict__ G = gaps + g;
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  int cell;
  uint64_t off24;
  if (mode == PIC_SEED_RANDOM) {
    const U64x4 u = philox4x64_10(0, 0, kTagSeed, 0, (uint64_t)i, G->seed);
    cell = (int)(((u.v[0] >> 32) * (uint64_t)G->n_cells) >> 32);
    off24 = u.v[1] >> 40;
  } else {
    const double x = floor(((double)i + 0.5) * ((double)G->n_cells / (double)N) * 16777216.0);
    const long long X = (long long)x;
    cell = (int)(X >> 24);
    off24 = (uint64_t)(X & 0xFFFFFF);
  }
  const T off = (T)(double)off24 * (T)(1.0 / 16777216.0);
  const int b = G->buf;
  G->cell[b][0][base0 + i] = cell;
  ((T*)G->off[b][0])[base0 + i] = off;
  ((T*)G->p[b][0])[base0 + i] = (T)p0m;
  G->id[b][0][base0 + i] = 2ull * (uint64_t)i;
  G->cell[b][1][base1 + i] = cell;
  ((T*)G->off[b][1])[base1 + i] = off;
  ((T*)G->p[b][1])[base1 + i] = (T)p0p;
  G->id[b][1][base1 + i] = 2ull * (uint64_t)i + 1ull;
}

// ------------------------------------------------------------- rho (diag)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rho(GapDev* __restrict__ gaps, int g,
                                                long long* __restrict__ acc) {
  GapDev* __restrict__ G = gaps + g;
  const int buf = G->buf;
  const T scale = (T)(double)G->one;
  for (int s = 0; s < 2; ++s) {
    const long long q = s == 0 ? -1 : 1;
    const long long nS = (long long)G->n[s];
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nS;
         i += (long long)gridDim.x * kBlock) {
      const int c = G->cell[buf][s][i];
      if (c == kDead) continue;
      const long long oq = (long long)(((const T*)G->off[buf][s])[i] * scale);
      if (G->shape == PIC_SHAPE_QUADRATIC) {
        // the spline's three nodes, folded into [0, n_cells) (periodic) or
        // dropped beyond the wall nodes (absorbing)
        int j;
        long long w0, w1, w2;
        spline_weights<long long>(oq, (long long)G->one, G->K, j, w0, w1, w2);  // any K
        const long long wk[3] = {w0, w1, w2};
        for (int k = 0; k < 3; ++k) {
          int node = c + j - 1 + k;
          if (G->boundary == PIC_BC_PERIODIC)
            node = node < 0 ? node + G->n_cells : (node >= G->n_cells ? node - G->n_cells : node);
          else if (node < 0 || node > G->n_cells)
            continue;  // beyond a wall node
          atomicAdd((unsigned long long*)&acc[node], as_u64(q * wk[k]));
        }
        continue;
      }
      atomicAdd((unsigned long long*)&acc[c], as_u64(q * (G->one - oq)));
      atomicAdd((unsigned long long*)&acc[c + 1], as_u64(q * oq));
    }
  }
}

// ------------------------------------------------------ phase space (diag)
// Histogram of species s over (cell bin, momentum bin): cell c falls in bin
// c * x_bins / n_cells, momentum p in floor((p - p_min) * inv_dp) clamped to
// [0, p_bins), computed in binary64.  Counted in LDS when the bins fit.
constexpr int kPhaseLds = 8192;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_phase(GapDev* __restrict__ gaps, int g, int s, int x_bins,
                                                  int p_bins, double p_min, double inv_dp,
                                                  unsigned long long* __restrict__ out) {
  __shared__ unsigned int h[kPhaseLds];
  const GapDev* __restrict__ G = gaps + g;
  const int nb = x_bins * p_bins;
  const bool lds = nb <= kPhaseLds;
  if (lds) {
    for (int k = threadIdx.x; k < nb; k += kBlock) h[k] = 0u;
    __syncthreads();
  }
  const int buf = G->buf, nc = G->n_cells;
  const long long n = (long long)G->n[s];
  const int32_t* __restrict__ cell = G->cell[buf][s];
  const T* __restrict__ pp = (const T*)G->p[buf][s];
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
    const int c = cell[i];
    if (c == kDead) continue;
    const long long xb = (long long)c * x_bins / nc;
    double q = floor(((double)pp[i] - p_min) * inv_dp);
    q = q >= 0.0 ? q : 0.0;  // also a NaN momentum
    q = q <= (double)(p_bins - 1) ? q : (double)(p_bins - 1);
    const long long bin = xb * p_bins + (long long)q;
    if (lds) atomicAdd(&h[bin], 1u);
    else atomicAdd(out + bin, 1ull);
  }
  if (lds) {
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += kBlock)
      if (h[k]) atomicAdd(out + k, (unsigned long long)h[k]);
  }
}

__global__ void k_zero_ll(long long* __restrict__ a, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    a[i] = 0;
}

// ------------------------------------------------------------- launchers
static int grid_for(long long want, int cap) {
  return (int)(want < 1 ? 1 : (want < cap ? want : cap));
}

// With events, they are recorded by the dispatch itself (its start and end),
// so that the timed span is the kernel's own.
template <typename T, bool kSpread, bool kSpline>
static void push_kernel(const StepLaunch& L, hipEvent_t start, hipEvent_t stop) {
  if (start) {
    hipExtLaunchKernelGGL((k_push<T, kSpread, kSpline>), dim3(kPushGrid), dim3(kBlock), 0, L.stream,
                          start, stop, 0, L.gaps, L.wi, L.B, L.stripes);
    return;
  }
  hipLaunchKernelGGL((k_push<T, kSpread, kSpline>), dim3(kPushGrid), dim3(kBlock), 0, L.stream,
                     L.gaps, L.wi, L.B, L.stripes);
}

template <typename T>
static void push_for(const StepLaunch& L, hipEvent_t start, hipEvent_t stop) {
  if (L.spline) {
    if (L.spread) push_kernel<T, true, true>(L, start, stop);
    else push_kernel<T, false, true>(L, start, stop);
  } else {
    if (L.spread) push_kernel<T, true, false>(L, start, stop);
    else push_kernel<T, false, false>(L, start, stop);
  }
}

hipError_t launch_push(const StepLaunch& L, bool mixed, hipEvent_t start, hipEvent_t stop) {
  if (mixed) push_for<float>(L, start, stop);
  else push_for<double>(L, start, stop);
  return hipGetLastError();
}

hipError_t launch_step_after_push(const StepLaunch& L, bool mixed) {
  const int nf = grid_for(L.cell_items, 1 << 30);
  const int nfold = (4 * L.B * kStripes + kBlock - 1) / kBlock;
  const int grid = nf + L.emit_grid + L.conv_grid + nfold;
  if (mixed)
    hipLaunchKernelGGL(k_post<float>, dim3(grid), dim3(kBlock), 0, L.stream, L.gaps, L.cwi, L.wi,
                       L.pwi, L.B, nf, L.emit_grid, L.conv_grid, L.emit_cnt, L.emit_ent, L.wg_emit,
                       L.stripes);
  else
    hipLaunchKernelGGL(k_post<double>, dim3(grid), dim3(kBlock), 0, L.stream, L.gaps, L.cwi, L.wi,
                       L.pwi, L.B, nf, L.emit_grid, L.conv_grid, L.emit_cnt, L.emit_ent, L.wg_emit,
                       L.stripes);
  hipLaunchKernelGGL(k_finalize, dim3((L.B + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0, L.stream,
                     L.gaps, L.B, L.wi, L.items);
  hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(1024), 0, L.stream, L.B, L.items, L.wi, L.pwi, L.qwi);
  return hipGetLastError();
}

hipError_t launch_step(const StepLaunch& L, bool mixed) {
  hipError_t e = launch_push(L, mixed, nullptr, nullptr);
  if (e != hipSuccess) return e;
  return launch_step_after_push(L, mixed);
}

hipError_t launch_sort(const StepLaunch& L, bool mixed) {
  hipLaunchKernelGGL(k_sort_zero, dim3(grid_for(L.cell_items, 1 << 30)), dim3(kBlock), 0, L.stream, L.gaps, L.cwi, L.B);
  hipLaunchKernelGGL(k_ph_zero, dim3(L.B), dim3(kBlock), 0, L.stream, L.gaps, L.B);
  if (mixed) hipLaunchKernelGGL((k_sort_pass<0, float, false>), dim3(L.push_grid), dim3(kBlock), 0, L.stream, L.gaps, L.wi, L.B);
  else hipLaunchKernelGGL((k_sort_pass<0, double, false>), dim3(L.push_grid), dim3(kBlock), 0, L.stream, L.gaps, L.wi, L.B);
  hipLaunchKernelGGL(k_ph_pass<0>, dim3(L.ph_sort_grid), dim3(kBlock), 0, L.stream, L.gaps, L.qwi, L.B);
  hipLaunchKernelGGL(k_sort_scan<false>, dim3(2 * L.B), dim3(1024), 0, L.stream, L.gaps, L.B);
  hipLaunchKernelGGL(k_ph_scan, dim3(L.B), dim3(1024), 0, L.stream, L.gaps, L.B);
  if (mixed) hipLaunchKernelGGL((k_sort_pass<1, float, false>), dim3(L.push_grid), dim3(kBlock), 0, L.stream, L.gaps, L.wi, L.B);
  else hipLaunchKernelGGL((k_sort_pass<1, double, false>), dim3(L.push_grid), dim3(kBlock), 0, L.stream, L.gaps, L.wi, L.B);
  hipLaunchKernelGGL(k_ph_pass<1>, dim3(L.ph_sort_grid), dim3(kBlock), 0, L.stream, L.gaps, L.qwi, L.B);
  hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(1024), 0, L.stream, L.gaps, L.B, L.wi, L.pwi, L.qwi);
  return hipGetLastError();
}

// The tails are a small part of the leptons, so their passes take a quarter
// of the full sort's grid (which also keeps the launches cheap when there is
// nothing to sort).
template <typename T>
static void tail_sort_for(const StepLaunch& L) {
  const int grid = L.push_grid / 4;
  hipLaunchKernelGGL(k_tail_plan, dim3(1), dim3(1024), 0, L.stream, L.gaps, L.B, L.twi);
  hipLaunchKernelGGL(k_tail_zero, dim3(grid_for(L.cell_items, 1 << 30)), dim3(kBlock), 0, L.stream, L.gaps, L.cwi, L.B);
  hipLaunchKernelGGL((k_sort_pass<0, T, true>), dim3(grid), dim3(kBlock), 0, L.stream, L.gaps, L.twi, L.B);
  hipLaunchKernelGGL(k_sort_scan<true>, dim3(2 * L.B), dim3(1024), 0, L.stream, L.gaps, L.B);
  hipLaunchKernelGGL((k_sort_pass<1, T, true>), dim3(grid), dim3(kBlock), 0, L.stream, L.gaps, L.twi, L.B);
  hipLaunchKernelGGL(k_tail_copy<T>, dim3(grid), dim3(kBlock), 0, L.stream, L.gaps, L.twi, L.B);
}

hipError_t launch_tail_sort(const StepLaunch& L, bool mixed) {
  if (mixed) tail_sort_for<float>(L);
  else tail_sort_for<double>(L);
  return hipGetLastError();
}

hipError_t launch_plan(const StepLaunch& L) {
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, L.stream, L.gaps, L.B, L.wi, L.pwi, L.qwi);
  return hipGetLastError();
}

hipError_t launch_seed(GapDev* gaps, int g, int mode, long long N, double p0m, double p0p,
                       long long base0, long long base1, bool mixed, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  const int grid = (int)((N + kBlock - 1) / kBlock);
  if (mixed) hipLaunchKernelGGL(k_seed<float>, dim3(grid), dim3(kBlock), 0, st, gaps, g, mode, N, p0m, p0p, base0, base1);
  else hipLaunchKernelGGL(k_seed<double>, dim3(grid), dim3(kBlock), 0, st, gaps, g, mode, N, p0m, p0p, base0, base1);
  return hipGetLastError();
}

hipError_t launch_phase(GapDev* gaps, int g, int s, int x_bins, int p_bins, double p_min, double inv_dp,
                        unsigned long long* out, bool mixed, hipStream_t st) {
  if (mixed) hipLaunchKernelGGL(k_phase<float>, dim3(1024), dim3(kBlock), 0, st, gaps, g, s, x_bins, p_bins, p_min, inv_dp, out);
  else hipLaunchKernelGGL(k_phase<double>, dim3(1024), dim3(kBlock), 0, st, gaps, g, s, x_bins, p_bins, p_min, inv_dp, out);
  return hipGetLastError();
}

hipError_t launch_zero(long long* a, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_ll, dim3(256), dim3(256), 0, st, a, n);
  return hipGetLastError();
}

hipError_t launch_rho(GapDev* gaps, int g, long long* rho_acc, long long n_nodes, bool mixed,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_zero_ll, dim3(64), dim3(256), 0, st, rho_acc, n_nodes);
  if (mixed) hipLaunchKernelGGL(k_rho<float>, dim3(1024), dim3(kBlock), 0, st, gaps, g, rho_acc);
  else hipLaunchKernelGGL(k_rho<double>, dim3(1024), dim3(kBlock), 0, st, gaps, g, rho_acc);
  return hipGetLastError();
}

// ------------------------------------------------- static node scratch
// The node-charge accumulators of pic_read_fields_noalloc: one array per
// GPU the library runs on, held until the process ends, shared by every
// call on that GPU.  Host code never passes `scratch` itself to a kernel
// (in host code the name stands for a host-side placeholder); it uses the
// device address that hipGetSymbolAddress returns, looked up once per
// device with that device current.
__device__ __align__(256) long long scratch[kStaticNodes];

hipError_t static_scratch(int device, long long** out) {
  static std::mutex lock;
  static long long* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> guard(lock);
  if (!addr[device]) {
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) {
      const hipError_t e2 = hipSetDevice(prev);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    addr[device] = static_cast<long long*>(p);
  }
  *out = addr[device];
  return hipSuccess;
}

}  // namespace pic
