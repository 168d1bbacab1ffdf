// HIP kernels (gfx950) of the pair-cascade PIC step.
//
// One step of a gap (arXiv:2012.05587, sections 2-3):
//   k_push     gather E at each lepton, relativistic push, move with an exact
//              integer charge-conserving flux (per-workgroup LDS tile reduced
//              into the global int64 grid), absorb/wrap, and the threshold
//              test: the emitter loses k * gamma_pair and is listed;
//   k_emit     listed emitters draw their photons (or in-place pairs) from
//              Philox and append them;
//   k_field    Ampere's law E -= w 2^-K F (Eq. 4 in normalised units) and the
//              field diagnostics;
//   k_convert  photons due this step become pairs (appended);
//   k_finalize counters, history row and the work plan of the next step.
// Every S steps the leptons are re-sorted by cell and the photon store by
// conversion step (counting sorts), which drops absorbed leptons and
// converted photons.
//
// All kernels take the gaps of a batch at once: work items are chunks of
// particles, photons or cells, numbered across gaps by prefix arrays that
// the device itself maintains, so a sequence of steps needs no host
// synchronisation and can be captured in a graph.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pic_device.hpp"
#include "pic_kernels.hpp"

namespace pic {

__device__ __forceinline__ int wrap_or_clamp(const GapDev& G, int c) {
  if (G.boundary == PIC_BC_PERIODIC) {
    if (c < 0) c += G.n_cells;
    else if (c >= G.n_cells) c -= G.n_cells;
  } else {
    if (c < 0) c = 0;
    else if (c >= G.n_cells) c = G.n_cells - 1;
  }
  return c;
}

__device__ __forceinline__ unsigned long long as_u64(long long v) { return (unsigned long long)v; }

// n_conv = min{k >= 1 : u >= T_k} over the decreasing integer table T
// (T_{len-1} = 0).  T_k ~ q^k 2^32, so k ~ ln(u 2^-32) / ln q; the estimate
// only picks where to look: the answer is decided by the table entries.
__device__ __forceinline__ int conv_steps(const uint32_t* __restrict__ table, int len, uint32_t u,
                                         float inv_lnq) {
  int k;
  if (u == 0u) {
    k = len - 1;
  } else {
    const float est = __logf((float)u * 2.3283064365386963e-10f) * inv_lnq;
    k = (int)ceilf(est);
  }
  k = k < 1 ? 1 : (k > len - 1 ? len - 1 : k);
  // walk to the exact answer; the estimate is within a step or two
  for (int it = 0; it < 4; ++it) {
    if (u >= table[k]) {
      if (k > 1 && u >= table[k - 1]) { --k; continue; }
      return k;
    }
    ++k;
  }
  // fall back to bisection (not reached for tables built by the runtime)
  int lo = 1, hi = len - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (u >= table[mid]) hi = mid; else lo = mid + 1;
  }
  return lo;
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

// Block-wide exclusive prefix sum (256 threads); `total` gets the sum.
__device__ __forceinline__ unsigned long long block_excl_scan(unsigned long long x,
                                                              unsigned long long* s_tmp,
                                                              unsigned long long& total) {
  const unsigned long long incl = wave_incl_scan(x);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (lane_id() == 63) s_tmp[w] = incl;
  __syncthreads();
  unsigned long long off = 0, t = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; ++k) {
    const unsigned long long v = s_tmp[k];
    if (k < w) off += v;
    t += v;
  }
  total = t;
  return off + incl - x;
}

// ------------------------------------------------------------------ push
// Sums of one workgroup over the work items of one gap, flushed with one
// atomic each when the workgroup moves to another gap or finishes.
struct PushTally {
  double ke, lost;
  unsigned long long absorbed[2];
};

__device__ __forceinline__ void flush_tally(double* __restrict__ stripes, int g, PushTally& t,
                                            bool diag, double* s_d, unsigned long long* s_u) {
  const double ke = wave_sum(t.ke), lost = wave_sum(t.lost);
  const unsigned long long a0 = wave_sum(t.absorbed[0]), a1 = wave_sum(t.absorbed[1]);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (lane_id() == 0) {
    s_d[w] = ke; s_d[4 + w] = lost;
    s_u[w] = a0; s_u[4 + w] = a1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double k = (s_d[0] + s_d[1]) + (s_d[2] + s_d[3]);
    const double l = (s_d[4] + s_d[5]) + (s_d[6] + s_d[7]);
    const unsigned long long b0 = s_u[0] + s_u[1] + s_u[2] + s_u[3];
    const unsigned long long b1 = s_u[4] + s_u[5] + s_u[6] + s_u[7];
    const int st = blockIdx.x & (kStripes - 1);
    if (diag && k != 0.0) atomicAdd(stripe_slot(stripes, g, 0, st), k);
    if (l != 0.0) atomicAdd(stripe_slot(stripes, g, 1, st), l);
    if (b0) atomicAdd((unsigned long long*)stripe_slot(stripes, g, 2, st), b0);
    if (b1) atomicAdd((unsigned long long*)stripe_slot(stripes, g, 3, st), b1);
  }
  t.ke = 0.0; t.lost = 0.0; t.absorbed[0] = 0; t.absorbed[1] = 0;
}

// One work item is a chunk of kChunk leptons of one species of one gap.
// Leptons are sorted by cell (between re-sorts they drift by a few cells),
// so a chunk touches a short range of cells: its current is summed in a
// per-workgroup LDS tile over that range and added to the grid with one
// atomic per touched cell.  Chunks spread over more than kTile cells (the
// sparse early cascade, unsorted appended leptons) add to the grid directly.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_push(GapDev* __restrict__ gaps,
                                                 const long long* __restrict__ wi, int B,
                                                 int32_t* __restrict__ emit_cnt,
                                                 uint32_t* __restrict__ emit_ent,
                                                 double* __restrict__ stripes) {
  using I = typename Fixed<T>::I;
  __shared__ long long s_flux[kTile];
  __shared__ uint32_t s_emit[kChunk];  // chunk-local index << 8 | k
  __shared__ int s_red[8];
  __shared__ double s_d[8];
  __shared__ unsigned long long s_u[8];
  __shared__ int s_emit_n;

  const long long total = wi[B];
  long long w0, w1;
  xcd_range(total, w0, w1);
  const int tid = threadIdx.x;
  const int lane = lane_id();
  PushTally tally = {0.0, 0.0, {0, 0}};
  int cur_g = -1;
  bool cur_diag = false;

  for (long long w = w0; w < w1; ++w) {
    const int g = find_gap(wi, B, w);
    GapDev* __restrict__ G = gaps + g;
    if (g != cur_g) {
      if (cur_g >= 0) flush_tally(stripes, cur_g, tally, cur_diag, s_d, s_u);
      cur_g = g;
      cur_diag = (G->step % G->diag_every) == 0;
    }
    if (G->status != PIC_OK) continue;
    const int buf = G->buf;
    const long long chunks0 = ((long long)G->n[0] + kChunk - 1) / kChunk;
    const long long local = w - wi[g];
    const int s = local < chunks0 ? 0 : 1;
    const long long i0 = (s == 0 ? local : local - chunks0) * kChunk;
    const long long nS = (long long)G->n[s];
    const long long i1 = i0 + kChunk < nS ? i0 + kChunk : nS;
    if (tid == 0) emit_cnt[w] = 0;

    gptr<int32_t> cellA = glb(G->cell[buf][s]);
    gptr<T> offA = glb<T>(G->off[buf][s]);
    gptr<T> pA = glb<T>(G->p[buf][s]);
    gptr<const double> E = glb<const double>(G->E);
    gptr<unsigned long long> F = glb<unsigned long long>((void*)G->F);
    const int nc = G->n_cells;
    const bool periodic = G->boundary == PIC_BC_PERIODIC;
    const I ONE = (I)G->one;
    const T scale = (T)(double)G->one;
    const T inv_scale = (T)(1.0 / (double)G->one);
    const T qdt = s == 0 ? -(T)G->dt : (T)G->dt;
    const T dtdx = (T)G->dtdx;
    const T gthr = (T)G->gthr, gpair = (T)G->gpair;
    const T one_t = (T)1, half_t = (T)0.5;
    const double w_d = G->weight;

    int cl[kItems];
    T ov[kItems], pv[kItems];
    int mn = INT32_MAX, mx = INT32_MIN;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const long long i = i0 + tid + (long long)j * kBlock;
      cl[j] = i < i1 ? cellA[i] : kDead;
      ov[j] = (T)0;
      pv[j] = (T)0;
      if (cl[j] != kDead) {
        ov[j] = offA[i];
        pv[j] = pA[i];
        mn = min(mn, cl[j]);
        mx = max(mx, cl[j]);
      }
    }
    if (tid == 0) s_emit_n = 0;
    block_minmax(mn, mx, s_red);
    if (mx < mn) continue;  // no live lepton in this chunk (uniform)
    const int base = mn - 1;
    const int span = mx - mn + 3;
    const bool lds = span <= kTile;
    if (lds) {
      for (int k = tid; k < span; k += kBlock) s_flux[k] = 0;
      __syncthreads();
    }

    bool bad = false, emit_bad = false;

#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const long long i = i0 + tid + (long long)j * kBlock;
      const int c = cl[j];
      if (c == kDead) continue;
      int cm = c - 1, cp = c + 1;
      if (periodic) { cm = cm < 0 ? nc - 1 : cm; cp = cp >= nc ? 0 : cp; }
      else { cm = cm < 0 ? 0 : cm; cp = cp >= nc ? nc - 1 : cp; }
      const T Em = (T)E[cm], Ec = (T)E[c], Ep = (T)E[cp];
      const T o = ov[j];
      const I oq = (I)(o * scale);
      // gather: node averages, then linear in the offset
      const T el = half_t * (Em + Ec);
      const T er = half_t * (Ec + Ep);
      const T Epart = el + o * (er - el);
      // push and move
      T pn = pv[j] + qdt * Epart;
      const T gam = sqrt(one_t + pn * pn);
      const T v = pn / gam;
      const T d = v * dtdx;
      const I dq = (I)rint(d * scale);
      I nq = oq + dq;
      I a1, a2 = 0;  // flux of a positive charge through this cell and the next
      int cross = 0;  // -1, 0, +1: node crossed to the left / none / right
      int c2 = c;
      bool keep = true;
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
      if (!isfinite(pn) || !isfinite(gam)) bad = true;
      if (keep) {
        // emission: repeated subtraction of gamma_pair while at or above threshold
        int k = 0;
        T gm = gam;
        while (gm >= gthr && k <= kMaxEmit) {
          gm = gm - gpair;
          ++k;
        }
        if (k > kMaxEmit) { emit_bad = true; k = 0; }
        T gnew = gam;
        if (k > 0) {
          const T mag = sqrt(gm * gm - one_t);
          pn = pn > (T)0 ? mag : -mag;
          gnew = sqrt(one_t + pn * pn);
          const int pos = atomicAdd(&s_emit_n, 1);
          s_emit[pos] = ((uint32_t)(i - i0) << 8) | (uint32_t)k;
        }
        pA[i] = pn;
        offA[i] = (T)nq * inv_scale;
        if (c2 != c) cellA[i] = c2;
        // energy: the Lorentz factor in the particle precision, summed in binary64
        if (cur_diag) tally.ke += w_d * (double)gnew;
      } else {
        tally.lost += w_d * (double)gam;
        tally.absorbed[s] += 1;
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
          int cc = base + k;
          if (cc < 0) cc += nc;
          else if (cc >= nc) cc -= nc;
          gadd(F + cc, as_u64(f));
        }
      }
    }
    // ---- emitters of this chunk, in the chunk's own slice of the list
    const int ne = s_emit_n;
    if (ne > 0) {
      if (tid == 0) emit_cnt[w] = ne;
      gptr<uint32_t> el = glb(emit_ent + w * (long long)kChunk);
      for (int k = tid; k < ne; k += kBlock) el[k] = s_emit[k];
    }
    __syncthreads();
  }
  if (cur_g >= 0) flush_tally(stripes, cur_g, tally, cur_diag, s_d, s_u);
}

// ------------------------------------------------------------------ emit
// Chunk x of the current plan lists its emitters in emit_ent[x * kChunk ..]
// (chunk-local index << 8 | number of emissions k).
__device__ __forceinline__ void chunk_origin(const GapDev* G, long long local, int& s,
                                             long long& i0) {
  const long long chunks0 = ((long long)G->n[0] + kChunk - 1) / kChunk;
  s = local < chunks0 ? 0 : 1;
  i0 = (s == 0 ? local : local - chunks0) * kChunk;
}

// Sum over the block of x (256 threads); every thread gets it.
__device__ __forceinline__ unsigned long long block_sum(unsigned long long x,
                                                        unsigned long long* s_tmp) {
  const unsigned long long v = wave_sum(x);
  __syncthreads();
  if (lane_id() == 0) s_tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  return (s_tmp[0] + s_tmp[1]) + (s_tmp[2] + s_tmp[3]);
}

template <typename T>
__device__ void emit_role(GapDev* __restrict__ gaps, const long long* __restrict__ wi, int B,
                          const int32_t* __restrict__ emit_cnt,
                          const uint32_t* __restrict__ emit_ent, int vb, int nvb,
                          unsigned long long* s_tmp, unsigned long long* s_base) {
  const int lane = lane_id();
  const long long total = wi[B];
  long long w0, w1;
  xcd_range(total, w0, w1, vb, nvb);
  for (long long w = w0; w < w1;) {
    const int g = find_gap(wi, B, w);
    const long long wend = wi[g + 1] < w1 ? wi[g + 1] : w1;
    GapDev* __restrict__ G = gaps + g;
    if (G->status != PIC_OK) { w = wend; continue; }
    // pass 1: emissions of this workgroup's chunks of gap g, for one reservation
    unsigned long long cnt = 0;
    for (long long x = w; x < wend; ++x) {
      const int ne = emit_cnt[x];
      for (int e = threadIdx.x; e < ne; e += kBlock) cnt += emit_ent[x * kChunk + e] & 255u;
    }
    const unsigned long long tot = block_sum(cnt, s_tmp);
    if (tot == 0) { w = wend; continue; }
    const bool in_place = G->table_len == 0;
    if (threadIdx.x == 0) {
      atomicAdd(&G->photons_emitted, tot);
      if (in_place) {
        const unsigned long long be = atomicAdd(&G->n_next[0], tot);
        const unsigned long long bp = atomicAdd(&G->n_next[1], tot);
        atomicAdd(&G->pairs_created, tot);
        if (be + tot > (unsigned long long)G->cap || bp + tot > (unsigned long long)G->cap)
          G->overflow = 1;
        s_base[0] = be;
        s_base[1] = bp;
      } else {
        const unsigned long long b = atomicAdd(&G->n_ph_next, tot);
        atomicAdd(&G->inflight, tot);
        if (b + tot > (unsigned long long)G->ph_cap) G->overflow = 1;
        s_base[0] = b;
        s_base[1] = 0;
      }
    }
    __syncthreads();
    const unsigned long long base0 = s_base[0], base1 = s_base[1];
    const int buf = G->buf;
    const uint64_t stepn = (uint64_t)G->step;
    const uint64_t seed = G->seed;
    const bool absorbing = G->boundary == PIC_BC_ABSORBING;
    const bool diag = (G->step % G->diag_every) == 0;
    const long long ONE = G->one;
    const T pchild = (T)G->pchild;
    const T scale = (T)(double)ONE;
    const unsigned long long cap = (unsigned long long)G->cap;
    const unsigned long long ph_cap = (unsigned long long)G->ph_cap;
    const int pb = G->phbuf;
    unsigned long long run = 0, esc = 0;
    double ke = 0.0;
    // pass 2: write the photons (or pairs) at base + running offset
    for (long long x = w; x < wend; ++x) {
      const int ne = emit_cnt[x];
      if (ne == 0) continue;
      int s;
      long long i0;
      chunk_origin(G, x - wi[g], s, i0);
      for (int r = 0; r < ne; r += kBlock) {
        const int e = r + threadIdx.x;
        int k = 0;
        long long i = 0;
        if (e < ne) {
          const uint32_t en = emit_ent[x * kChunk + e];
          k = (int)(en & 255u);
          i = i0 + (long long)(en >> 8);
        }
        unsigned long long rt;
        const unsigned long long ex = run + block_excl_scan((unsigned long long)k, s_tmp, rt);
        run += rt;
        if (k == 0) continue;
        const int c = G->cell[buf][s][i];
        const long long oq = (long long)(((const T*)G->off[buf][s])[i] * scale);
        const T pv = ((const T*)G->p[buf][s])[i];
        const uint64_t id = G->id[buf][s][i];
        const int dir = pv > (T)0 ? 1 : -1;
        if (in_place) {
          // pair made in place (the paper's zero mean free path)
          const T pc = dir > 0 ? pchild : -pchild;
          const T offn = (T)oq * ((T)1 / scale);
          for (int jj = 0; jj < k; ++jj) {
            const U64x4 u = philox4x64_10(stepn, (uint64_t)jj, kTagPhoton, 0, id, seed);
            const uint64_t child = u.v[1] & ~(uint64_t)1;
            const unsigned long long se = base0 + ex + jj, sp = base1 + ex + jj;
            if (se < cap) {
              G->cell[buf][0][se] = c; ((T*)G->off[buf][0])[se] = offn;
              ((T*)G->p[buf][0])[se] = pc; G->id[buf][0][se] = child;
            }
            if (sp < cap) {
              G->cell[buf][1][sp] = c; ((T*)G->off[buf][1])[sp] = offn;
              ((T*)G->p[buf][1])[sp] = pc; G->id[buf][1][sp] = child | 1u;
            }
          }
          if (diag) ke += (double)k * 2.0 * G->weight * G->child_gamma64;
        } else {
          const long long X0 = (long long)c * ONE + oq;
          for (int jj = 0; jj < k; ++jj) {
            const U64x4 u = philox4x64_10(stepn, (uint64_t)jj, kTagPhoton, 0, id, seed);
            const uint64_t child = u.v[1] & ~(uint64_t)1;
            const int ncv = conv_steps(G->table, G->table_len, (uint32_t)(u.v[0] >> 32), G->inv_lnq);
            long long X = X0 + (long long)dir * (long long)ncv * G->photon_step;
            int cstep = (int)((long long)stepn + ncv);
            if (absorbing) {
              if (X < 0 || X >= G->domain) { cstep = INT32_MIN; ++esc; }
            } else {
              X %= G->domain;
              if (X < 0) X += G->domain;
            }
            const unsigned long long slot = base0 + ex + jj;
            if (slot < ph_cap) {
              G->ph_x[pb][slot] = X;
              G->ph_step[pb][slot] = cstep;
              G->ph_child[pb][slot] = child | (dir > 0 ? 1u : 0u);
            }
          }
        }
      }
    }
    const unsigned long long esc_b = block_sum(esc, s_tmp);
    const double ke_w = wave_sum(ke);
    if (lane == 0 && ke_w != 0.0) atomicAdd(&G->ke_acc, ke_w);
    if (threadIdx.x == 0 && esc_b > 0) {
      atomicAdd(&G->photons_escaped, esc_b);
      atomicAdd(&G->inflight, (unsigned long long)(-(long long)esc_b));
      atomicAdd(&G->lost_energy, (double)esc_b * G->weight * G->gpair64);
    }
    __syncthreads();  // s_base and s_tmp are reused by the next gap
    w = wend;
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
  const double wq = G->wq, dxh = G->dx;
  double fe = 0.0, es = 0.0;
  for (int k = threadIdx.x; k < kCellChunk; k += kBlock) {
    const long long c = c0 + k;
    if (c >= nc) break;
    const long long f = G->F[c];
    const double e = G->E[c] - wq * (double)f;
    G->E[c] = e;
    G->F_last[c] = f;
    G->F[c] = 0;
    fe += e * e * dxh * 0.5;
    es += e;
  }
  fe = wave_sum(fe);
  es = wave_sum(es);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) { s_red[w] = fe; s_red[4 + w] = es; }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&G->fe_acc, (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]));
    atomicAdd(&G->es_acc, (s_red[4] + s_red[5]) + (s_red[6] + s_red[7]));
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

__device__ __forceinline__ long long convert_items(const GapDev* G) {
  long long b0, b1, t0, t1;
  photon_ranges(G, b0, b1, t0, t1);
  return (b1 - b0 + kPhChunk - 1) / kPhChunk + (t1 - t0 + kPhChunk - 1) / kPhChunk;
}

__device__ __forceinline__ void convert_item(const GapDev* G, long long local, long long& i0,
                                             long long& i1) {
  long long b0, b1, t0, t1;
  photon_ranges(G, b0, b1, t0, t1);
  const long long nb = (b1 - b0 + kPhChunk - 1) / kPhChunk;
  if (local < nb) {
    i0 = b0 + local * kPhChunk;
    i1 = i0 + kPhChunk < b1 ? i0 + kPhChunk : b1;
  } else {
    i0 = t0 + (local - nb) * kPhChunk;
    i1 = i0 + kPhChunk < t1 ? i0 + kPhChunk : t1;
  }
}

template <typename T>
__device__ void convert_role(GapDev* __restrict__ gaps, const long long* __restrict__ pwi, int B,
                             int vb, int nvb, unsigned long long* s_tmp,
                             unsigned long long* s_base) {
  const long long total = pwi[B];
  long long w0, w1;
  xcd_range(total, w0, w1, vb, nvb);
  for (long long w = w0; w < w1;) {
    const int g = find_gap(pwi, B, w);
    const long long wend = pwi[g + 1] < w1 ? pwi[g + 1] : w1;
    GapDev* __restrict__ G = gaps + g;
    if (G->status != PIC_OK) { w = wend; continue; }
    const int pb = G->phbuf, buf = G->buf;
    const int stepn = (int)G->step;
    gptr<const int32_t> phs = glb<const int32_t>((void*)G->ph_step[pb]);
    // pass 1: due photons of this workgroup's items, for one reservation
    unsigned long long cnt = 0;
    for (long long x = w; x < wend; ++x) {
      long long i0, i1;
      convert_item(G, x - pwi[g], i0, i1);
      for (long long i = i0 + threadIdx.x; i < i1; i += kBlock) cnt += phs[i] == stepn ? 1u : 0u;
    }
    const unsigned long long tot = block_sum(cnt, s_tmp);
    if (tot == 0) { w = wend; continue; }
    const bool diag = ((long long)stepn % G->diag_every) == 0;
    const unsigned long long cap = (unsigned long long)G->cap;
    if (threadIdx.x == 0) {
      const unsigned long long be = atomicAdd(&G->n_next[0], tot);
      const unsigned long long bp = atomicAdd(&G->n_next[1], tot);
      atomicAdd(&G->pairs_created, tot);
      atomicAdd(&G->inflight, (unsigned long long)(-(long long)tot));
      if (be + tot > cap || bp + tot > cap) G->overflow = 1;
      if (diag) atomicAdd(&G->ke_acc, (double)tot * 2.0 * G->weight * G->child_gamma64);
      s_base[0] = be;
      s_base[1] = bp;
    }
    __syncthreads();
    const unsigned long long be = s_base[0], bp = s_base[1];
    const long long ONE = G->one;
    const T inv_scale = (T)(1.0 / (double)ONE);
    const T pchild = (T)G->pchild;
    unsigned long long run = 0;
    // pass 2: write the pairs at base + running offset
    for (long long x = w; x < wend; ++x) {
      long long i0, i1;
      convert_item(G, x - pwi[g], i0, i1);
      for (long long r = i0; r < i1; r += kBlock) {
        const long long i = r + threadIdx.x;
        const bool due = i < i1 && phs[i] == stepn;
        unsigned long long rt;
        const unsigned long long ex = run + block_excl_scan(due ? 1ull : 0ull, s_tmp, rt);
        run += rt;
        if (!due) continue;
        const long long X = G->ph_x[pb][i];
        const uint64_t ch = G->ph_child[pb][i];
        const int c = (int)(X / ONE);
        const T offn = (T)(X % ONE) * inv_scale;
        const T pc = (ch & 1u) ? pchild : -pchild;
        const uint64_t child = ch & ~(uint64_t)1;
        const unsigned long long se = be + ex, sp = bp + ex;
        if (se < cap) {
          G->cell[buf][0][se] = c; ((T*)G->off[buf][0])[se] = offn;
          ((T*)G->p[buf][0])[se] = pc; G->id[buf][0][se] = child;
        }
        if (sp < cap) {
          G->cell[buf][1][sp] = c; ((T*)G->off[buf][1])[sp] = offn;
          ((T*)G->p[buf][1])[sp] = pc; G->id[buf][1][sp] = child | 1u;
        }
      }
    }
    __syncthreads();
    w = wend;
  }
}

// ------------------------------------------------------------ plans
// Work-item prefixes of the next launches: particle chunks per gap (both
// species) and due-photon chunks per gap; frozen gaps get none.
__device__ void compute_plans(GapDev* __restrict__ gaps, int B, long long* __restrict__ wi,
                              long long* __restrict__ pwi) {
  __shared__ long long s_a[1024], s_b[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (B + nt - 1) / nt;
  long long sa = 0, sb = 0;
  for (int g = tid * per; g < (tid + 1) * per && g < B; ++g) {
    const GapDev* G = gaps + g;
    if (G->status == PIC_OK) {
      sa += ((long long)G->n[0] + kChunk - 1) / kChunk + ((long long)G->n[1] + kChunk - 1) / kChunk;
      sb += convert_items(G);
    }
  }
  s_a[tid] = sa; s_b[tid] = sb;
  __syncthreads();
  for (int d = 1; d < nt; d <<= 1) {
    long long ya = tid >= d ? s_a[tid - d] : 0, yb = tid >= d ? s_b[tid - d] : 0;
    __syncthreads();
    s_a[tid] += ya; s_b[tid] += yb;
    __syncthreads();
  }
  long long ra = s_a[tid] - sa, rb = s_b[tid] - sb;
  for (int g = tid * per; g < (tid + 1) * per && g < B; ++g) {
    const GapDev* G = gaps + g;
    wi[g] = ra; pwi[g] = rb;
    if (G->status == PIC_OK) {
      ra += ((long long)G->n[0] + kChunk - 1) / kChunk + ((long long)G->n[1] + kChunk - 1) / kChunk;
      rb += convert_items(G);
    }
  }
  if (tid == nt - 1) { wi[B] = s_a[nt - 1]; pwi[B] = s_b[nt - 1]; }
}

__global__ __launch_bounds__(1024) void k_plan(GapDev* __restrict__ gaps, int B,
                                               long long* __restrict__ wi,
                                               long long* __restrict__ pwi) {
  compute_plans(gaps, B, wi, pwi);
}

// Ends a step for every gap: freeze on error, roll the counters, write the
// history row, and plan the next step.
constexpr int kFoldMax = 1024;  // gaps whose stripes finalize folds with the whole block

__device__ void finalize_body(GapDev* __restrict__ gaps, int B, long long* __restrict__ wi,
                              long long* __restrict__ pwi, double* __restrict__ stripes) {
  __shared__ unsigned long long s_fold[kFoldMax * 4];
  // fold the striped push tallies: 32 lanes sum the stripes of one
  // (gap, accumulator) pair; accumulators 2 and 3 hold integer counts
  const bool wide = B <= kFoldMax;
  if (wide) {
    const int lane = lane_id();
    const int pairs = B * 4;
    for (int base = (threadIdx.x >> 6) * 2; base < pairs; base += (blockDim.x >> 6) * 2) {
      const int pair = base + (lane >> 5);
      const int st = lane & 31;
      unsigned long long bits = 0;
      if (pair < pairs) {
        unsigned long long* slot = (unsigned long long*)stripe_slot(stripes, pair >> 2, pair & 3, st);
        bits = *slot;
        *slot = 0ull;
      }
      double dv = __longlong_as_double((long long)bits);
      unsigned long long uv = bits;
#pragma unroll
      for (int d = 16; d >= 1; d >>= 1) {
        dv += __shfl_xor(dv, d, 64);
        uv += __shfl_xor(uv, d, 64);
      }
      if (st == 0 && pair < pairs)
        s_fold[pair] = (pair & 3) < 2 ? (unsigned long long)__double_as_longlong(dv) : uv;
    }
    __syncthreads();
  }
  for (int g = threadIdx.x; g < B; g += blockDim.x) {
    GapDev* G = gaps + g;
    double ke = 0.0, lost = 0.0;
    unsigned long long ab[2] = {0, 0};
    if (wide) {
      ke = __longlong_as_double((long long)s_fold[g * 4 + 0]);
      lost = __longlong_as_double((long long)s_fold[g * 4 + 1]);
      ab[0] = s_fold[g * 4 + 2];
      ab[1] = s_fold[g * 4 + 3];
    } else {
      for (int st = 0; st < kStripes; ++st) {
        ke += *stripe_slot(stripes, g, 0, st);
        lost += *stripe_slot(stripes, g, 1, st);
        ab[0] += *(unsigned long long*)stripe_slot(stripes, g, 2, st);
        ab[1] += *(unsigned long long*)stripe_slot(stripes, g, 3, st);
        for (int a = 0; a < 4; ++a) *(unsigned long long*)stripe_slot(stripes, g, a, st) = 0ull;
      }
    }
    G->ke_acc += ke;
    G->lost_energy += lost;
    for (int s = 0; s < 2; ++s) {
      G->absorbed[s] += ab[s];
      G->dead[s] += ab[s];
    }
    if (G->status == PIC_OK) {
      int st = PIC_OK;
      if (G->nonfinite) st = PIC_ERR_NONFINITE;
      else if (G->overflow) st = PIC_ERR_CAPACITY;
      else if (G->emit_err) st = PIC_ERR_EMISSION;
      if (st != PIC_OK) {
        G->status = st;
      } else {
        G->pushes = G->pushes + G->live[0] + G->live[1];
        for (int s = 0; s < 2; ++s) {
          G->n[s] = G->n_next[s];
          G->live[s] = G->n[s] - G->dead[s];
        }
        G->n_ph = G->n_ph_next;
        const long long done = G->step;
        G->step = done + 1;
        if (done % G->diag_every == 0) {
          pic_history_row r;
          r.step = done;
          r.n_minus = (int64_t)G->live[0];
          r.n_plus = (int64_t)G->live[1];
          r.n_photons = (int64_t)G->inflight;
          r.pairs_created = (int64_t)G->pairs_created;
          r.photons_emitted = (int64_t)G->photons_emitted;
          r.photons_escaped = (int64_t)G->photons_escaped;
          r.absorbed_minus = (int64_t)G->absorbed[0];
          r.absorbed_plus = (int64_t)G->absorbed[1];
          r.kinetic = G->ke_acc;
          r.field = G->fe_acc;
          r.photon_energy = (double)G->inflight * G->weight * G->gpair64;
          r.lost_energy = G->lost_energy;
          r.e_mean = G->es_acc / (double)G->n_cells;
          G->hist[G->hist_count % (unsigned long long)G->hist_rows] = r;
          G->hist_count = G->hist_count + 1;
          G->last = r;
        }
      }
    }
    G->ke_acc = 0.0;
    G->fe_acc = 0.0;
    G->es_acc = 0.0;
  }
  __syncthreads();
  compute_plans(gaps, B, wi, pwi);
}

// Everything of a step between the push and the finalize: the Ampere update
// (blocks [0, n_field)), the emission draws (next n_emit blocks) and the
// conversions (last n_conv blocks) are independent of each other.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_post(GapDev* __restrict__ gaps,
                                                 const long long* __restrict__ cwi,
                                                 const long long* __restrict__ wi,
                                                 const long long* __restrict__ pwi, int B,
                                                 int n_field, int n_emit, int n_conv,
                                                 const int32_t* __restrict__ emit_cnt,
                                                 const uint32_t* __restrict__ emit_ent) {
  __shared__ double s_red[8];
  __shared__ unsigned long long s_tmp[kBlock / 64];
  __shared__ unsigned long long s_base[2];
  const int b = blockIdx.x;
  if (b < n_field) field_role(gaps, cwi, B, b, s_red);
  else if (b < n_field + n_emit)
    emit_role<T>(gaps, wi, B, emit_cnt, emit_ent, b - n_field, n_emit, s_tmp, s_base);
  else convert_role<T>(gaps, pwi, B, b - n_field - n_emit, n_conv, s_tmp, s_base);
}

__global__ __launch_bounds__(1024) void k_finalize(GapDev* __restrict__ gaps, int B,
                                                   long long* __restrict__ wi,
                                                   long long* __restrict__ pwi,
                                                   double* __restrict__ stripes) {
  finalize_body(gaps, B, wi, pwi, stripes);
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

__global__ __launch_bounds__(kBlock) void k_sort_zero(GapDev* __restrict__ gaps,
                                                      const long long* __restrict__ cwi, int B) {
  const int g = find_gap(cwi, B, blockIdx.x);
  GapDev* __restrict__ G = gaps + g;
  const long long c0 = (blockIdx.x - cwi[g]) * (long long)kCellChunk;
  for (int k = threadIdx.x; k < kCellChunk; k += kBlock) {
    const long long c = c0 + k;
    if (c >= G->n_cells) break;
    G->sort_cnt[0][c] = 0;
    G->sort_cnt[1][c] = 0;
  }
  if (blockIdx.x == cwi[g] && threadIdx.x == 0) { G->sorted_n[0] = 0; G->sorted_n[1] = 0; }
}

template <int PASS>
__global__ __launch_bounds__(kBlock) void k_sort_pass(GapDev* __restrict__ gaps,
                                                      const long long* __restrict__ wi, int B,
                                                      int elem_bytes) {
  const long long total = wi[B];
  long long w0, w1;
  xcd_range(total, w0, w1);
  const int lane = lane_id();
  for (long long w = w0; w < w1; ++w) {
    const int g = find_gap(wi, B, w);
    GapDev* __restrict__ G = gaps + g;
    if (G->status != PIC_OK) continue;
    const int buf = G->buf;
    const long long chunks0 = ((long long)G->n[0] + kChunk - 1) / kChunk;
    const long long local = w - wi[g];
    const int s = local < chunks0 ? 0 : 1;
    const long long i0 = (s == 0 ? local : local - chunks0) * kChunk;
    const long long nS = (long long)G->n[s];
    const long long i1 = i0 + kChunk < nS ? i0 + kChunk : nS;
    gptr<int32_t> cnt = glb(G->sort_cnt[s]);
    const int nb = buf ^ 1;
    gptr<const int32_t> cin = glb<const int32_t>((void*)G->cell[buf][s]);
    int cvs[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const long long i = i0 + threadIdx.x + (long long)j * kBlock;
      cvs[j] = i < i1 ? cin[i] : kDead;
    }
    if (PASS == 0) {
#pragma unroll
      for (int j = 0; j < kItems; ++j) {
        const int cv = cvs[j];
        int head_lane, run_len;
        wave_runs(cv, head_lane, run_len);
        if (run_len > 0 && cv != kDead)
          __hip_atomic_fetch_add(cnt + cv, run_len, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      continue;
    }
    // destinations of all items first (one returning atomic per run), then the moves
    long long dst[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int cv = cvs[j];
      int head_lane, run_len;
      wave_runs(cv, head_lane, run_len);
      int b = 0;
      if (run_len > 0 && cv != kDead)
        b = __hip_atomic_fetch_add(cnt + cv, run_len, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      b = __shfl(b, head_lane, 64);
      dst[j] = (long long)b + (lane - head_lane);
    }
    gptr<int32_t> cout = glb(G->cell[nb][s]);
    gptr<const uint64_t> iin = glb<const uint64_t>((void*)G->id[buf][s]);
    gptr<uint64_t> iout = glb(G->id[nb][s]);
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const long long i = i0 + threadIdx.x + (long long)j * kBlock;
      const int cv = cvs[j];
      if (cv == kDead) continue;
      const long long d = dst[j];
      cout[d] = cv;
      iout[d] = iin[i];
      if (elem_bytes == 8) {
        glb<double>(G->off[nb][s])[d] = glb<const double>(G->off[buf][s])[i];
        glb<double>(G->p[nb][s])[d] = glb<const double>(G->p[buf][s])[i];
      } else {
        glb<float>(G->off[nb][s])[d] = glb<const float>(G->off[buf][s])[i];
        glb<float>(G->p[nb][s])[d] = glb<const float>(G->p[buf][s])[i];
      }
    }
  }
}

// Exclusive scan of n int32 counts in place by one 1024-thread block; returns the total.
__device__ long long block_scan_counts(int32_t* __restrict__ cnt, int n, long long* s_sum) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (n + nt - 1) / nt;
  long long loc = 0;
  for (int c = tid * per; c < (tid + 1) * per && c < n; ++c) loc += cnt[c];
  s_sum[tid] = loc;
  __syncthreads();
  for (int d = 1; d < nt; d <<= 1) {
    long long y = tid >= d ? s_sum[tid - d] : 0;
    __syncthreads();
    s_sum[tid] += y;
    __syncthreads();
  }
  long long run = s_sum[tid] - loc;
  for (int c = tid * per; c < (tid + 1) * per && c < n; ++c) {
    const int v = cnt[c];
    cnt[c] = (int32_t)run;
    run += v;
  }
  return s_sum[nt - 1];
}

// Exclusive scan of the per-cell counts of one (gap, species) in place.
__global__ __launch_bounds__(1024) void k_sort_scan(GapDev* __restrict__ gaps, int B) {
  __shared__ long long s_sum[1024];
  const int g = blockIdx.x >> 1, s = blockIdx.x & 1;
  GapDev* __restrict__ G = gaps + g;
  if (G->status != PIC_OK) return;
  const long long tot = block_scan_counts(G->sort_cnt[s], G->n_cells, s_sum);
  if (threadIdx.x == blockDim.x - 1) G->sorted_n[s] = (unsigned long long)tot;
}

// ---- photon store: counting sort by conversion step, dropping the photons
// that converted or escaped.
__global__ __launch_bounds__(kBlock) void k_ph_zero(GapDev* __restrict__ gaps, int B) {
  GapDev* __restrict__ G = gaps + blockIdx.x;
  for (int k = threadIdx.x; k <= G->table_len; k += kBlock) G->ph_bucket[k] = 0;
  if (threadIdx.x == 0) G->ph_sorted = 0;
}

template <int PASS>
__global__ __launch_bounds__(kBlock) void k_ph_pass(GapDev* __restrict__ gaps, int B) {
  const int lane = lane_id();
  for (int g = 0; g < B; ++g) {
    GapDev* __restrict__ G = gaps + g;
    if (G->status != PIC_OK || G->table_len == 0) continue;
    const long long nP = (long long)G->n_ph;
    if (nP == 0) continue;
    long long i0, i1;
    xcd_range(nP, i0, i1);
    const int pb = G->phbuf;
    const long long stepn = G->step;
    int32_t* __restrict__ bucket = G->ph_bucket;
    for (long long r = i0; r < i1; r += kBlock) {
      const long long i = r + threadIdx.x;
      const long long cs = i < i1 ? (long long)G->ph_step[pb][i] : (long long)INT32_MIN;
      const int key = cs >= stepn ? (int)(cs - stepn) : -1;
      int head_lane, run_len;
      wave_runs(key, head_lane, run_len);
      if (PASS == 0) {
        if (run_len > 0 && key >= 0) atomicAdd(&bucket[key], run_len);
      } else {
        int b = 0;
        if (run_len > 0 && key >= 0) b = atomicAdd(&bucket[key], run_len);
        b = __shfl(b, head_lane, 64);
        if (key >= 0) {
          const long long dst = (long long)b + (lane - head_lane);
          G->ph_x[pb ^ 1][dst] = G->ph_x[pb][i];
          G->ph_step[pb ^ 1][dst] = (int32_t)cs;
          G->ph_child[pb ^ 1][dst] = G->ph_child[pb][i];
        }
      }
    }
  }
}

__global__ __launch_bounds__(1024) void k_ph_scan(GapDev* __restrict__ gaps, int B) {
  __shared__ long long s_sum[1024];
  GapDev* __restrict__ G = gaps + blockIdx.x;
  if (G->status != PIC_OK || G->table_len == 0) return;
  const long long tot = block_scan_counts(G->ph_bucket, G->table_len, s_sum);
  if (threadIdx.x == blockDim.x - 1) G->ph_sorted = (unsigned long long)tot;
}

__global__ __launch_bounds__(1024) void k_sort_finish(GapDev* __restrict__ gaps, int B,
                                                      long long* __restrict__ wi,
                                                      long long* __restrict__ pwi) {
  for (int g = threadIdx.x; g < B; g += blockDim.x) {
    GapDev* G = gaps + g;
    if (G->status != PIC_OK) continue;
    for (int s = 0; s < 2; ++s) {
      G->n[s] = G->sorted_n[s];
      G->n_next[s] = G->sorted_n[s];
      G->live[s] = G->sorted_n[s];
      G->dead[s] = 0;
    }
    G->buf ^= 1;
    if (G->table_len > 0) {
      G->n_ph = G->ph_sorted;
      G->n_ph_next = G->ph_sorted;
      G->ph_body_n = G->ph_sorted;
      G->ph_base = G->step;
      G->phbuf ^= 1;
    }
  }
  __syncthreads();
  compute_plans(gaps, B, wi, pwi);
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
__global__ __launch_bounds__(kBlock) void k_rho(GapDev* __restrict__ gaps, int g) {
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
      atomicAdd((unsigned long long*)&G->rho_acc[c], as_u64(q * (G->one - oq)));
      atomicAdd((unsigned long long*)&G->rho_acc[c + 1], as_u64(q * oq));
    }
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

hipError_t launch_push(const StepLaunch& L, bool mixed) {
  if (mixed)
    hipLaunchKernelGGL(k_push<float>, dim3(L.push_grid), dim3(kBlock), 0, L.stream, L.gaps, L.wi, L.B,
                       L.emit_cnt, L.emit_ent, L.stripes);
  else
    hipLaunchKernelGGL(k_push<double>, dim3(L.push_grid), dim3(kBlock), 0, L.stream, L.gaps, L.wi, L.B,
                       L.emit_cnt, L.emit_ent, L.stripes);
  return hipGetLastError();
}

hipError_t launch_step_after_push(const StepLaunch& L, bool mixed) {
  const int nf = grid_for(L.cell_items, 1 << 30);
  const int grid = nf + L.emit_grid + L.conv_grid;
  if (mixed)
    hipLaunchKernelGGL(k_post<float>, dim3(grid), dim3(kBlock), 0, L.stream, L.gaps, L.cwi, L.wi,
                       L.pwi, L.B, nf, L.emit_grid, L.conv_grid, L.emit_cnt, L.emit_ent);
  else
    hipLaunchKernelGGL(k_post<double>, dim3(grid), dim3(kBlock), 0, L.stream, L.gaps, L.cwi, L.wi,
                       L.pwi, L.B, nf, L.emit_grid, L.conv_grid, L.emit_cnt, L.emit_ent);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, L.stream, L.gaps, L.B, L.wi, L.pwi, L.stripes);
  return hipGetLastError();
}

hipError_t launch_step(const StepLaunch& L, bool mixed) {
  hipError_t e = launch_push(L, mixed);
  if (e != hipSuccess) return e;
  return launch_step_after_push(L, mixed);
}

hipError_t launch_sort(const StepLaunch& L, bool mixed) {
  const int eb = mixed ? 4 : 8;
  hipLaunchKernelGGL(k_sort_zero, dim3(grid_for(L.cell_items, 1 << 30)), dim3(kBlock), 0, L.stream, L.gaps, L.cwi, L.B);
  hipLaunchKernelGGL(k_ph_zero, dim3(L.B), dim3(kBlock), 0, L.stream, L.gaps, L.B);
  hipLaunchKernelGGL(k_sort_pass<0>, dim3(L.push_grid), dim3(kBlock), 0, L.stream, L.gaps, L.wi, L.B, eb);
  hipLaunchKernelGGL(k_ph_pass<0>, dim3(L.conv_grid), dim3(kBlock), 0, L.stream, L.gaps, L.B);
  hipLaunchKernelGGL(k_sort_scan, dim3(2 * L.B), dim3(1024), 0, L.stream, L.gaps, L.B);
  hipLaunchKernelGGL(k_ph_scan, dim3(L.B), dim3(1024), 0, L.stream, L.gaps, L.B);
  hipLaunchKernelGGL(k_sort_pass<1>, dim3(L.push_grid), dim3(kBlock), 0, L.stream, L.gaps, L.wi, L.B, eb);
  hipLaunchKernelGGL(k_ph_pass<1>, dim3(L.conv_grid), dim3(kBlock), 0, L.stream, L.gaps, L.B);
  hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(1024), 0, L.stream, L.gaps, L.B, L.wi, L.pwi);
  return hipGetLastError();
}

hipError_t launch_plan(const StepLaunch& L) {
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, L.stream, L.gaps, L.B, L.wi, L.pwi);
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

hipError_t launch_rho(GapDev* gaps, int g, long long* rho_acc, long long n_nodes, bool mixed,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_zero_ll, dim3(64), dim3(256), 0, st, rho_acc, n_nodes);
  if (mixed) hipLaunchKernelGGL(k_rho<float>, dim3(1024), dim3(kBlock), 0, st, gaps, g);
  else hipLaunchKernelGGL(k_rho<double>, dim3(1024), dim3(kBlock), 0, st, gaps, g);
  return hipGetLastError();
}

}  // namespace pic
