// HIP kernels (gfx950) of the pair-cascade PIC step.
//
// One step of a gap (arXiv:2012.05587, sections 2-3):
//   k_push     gather E at each lepton, relativistic push, move with an exact
//              integer charge-conserving flux (per-workgroup LDS tile reduced
//              into the global int64 grid), absorb/wrap, threshold emission
//              with wave-aggregated appends of photons or in-place pairs;
//   k_field    Ampere's law E -= w 2^-K F (Eq. 4 in normalised units) and the
//              field diagnostics;
//   k_convert  photons due this step become pairs (appended);
//   k_finalize counters, history row and the work plan of the next step.
// Every S steps the particles are re-sorted by cell (counting sort) and
// dead slots and converted photons are dropped.
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

template <typename T>
struct Prec;
template <>
struct Prec<double> { static constexpr int K = 40; };
template <>
struct Prec<float> { static constexpr int K = 24; };

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

// min{k >= 1 : u >= T_k} over the decreasing table T (T_{len-1} = 0).
__device__ __forceinline__ int conv_steps(const uint32_t* __restrict__ table, int len, uint32_t u) {
  int lo = 1, hi = len - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
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

// ------------------------------------------------------------------ push
template <typename T>
__global__ __launch_bounds__(kBlock) void k_push(GapDev* __restrict__ gaps,
                                                 const long long* __restrict__ wi, int B) {
  __shared__ long long s_flux[kTile + 4];
  __shared__ T s_E[kTile + 4];
  __shared__ int s_red[8];

  const long long total = wi[B];
  long long w0, w1;
  xcd_range(total, w0, w1);
  const int tid = threadIdx.x;
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

    int32_t* __restrict__ cellA = G->cell[buf][s];
    T* __restrict__ offA = (T*)G->off[buf][s];
    T* __restrict__ pA = (T*)G->p[buf][s];
    const int nc = G->n_cells;
    const int absorbing = G->boundary == PIC_BC_ABSORBING;
    const double* __restrict__ E = G->E;
    const long long ONE = G->one;
    const T scale = (T)(double)ONE;
    const T inv_scale = (T)(1.0 / (double)ONE);
    const T qdt = s == 0 ? -(T)G->dt : (T)G->dt;
    const long long q = s == 0 ? -1 : 1;
    const T dtdx = (T)G->dtdx;
    const T gthr = (T)G->gthr, gpair = (T)G->gpair, pchild = (T)G->pchild;
    const T one_t = (T)1, half_t = (T)0.5;
    const long long stepn = G->step;
    const bool diag = (stepn % G->diag_every) == 0;
    const double w_d = G->weight;

    int cell[kItems];
    int mn = INT32_MAX, mx = INT32_MIN;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const long long i = i0 + tid + (long long)j * kBlock;
      cell[j] = i < i1 ? cellA[i] : kDead;
      if (cell[j] != kDead) { mn = min(mn, cell[j]); mx = max(mx, cell[j]); }
    }
    block_minmax(mn, mx, s_red);
    if (mx < mn) continue;  // no live lepton in this chunk (uniform)
    const int base = mn - 1;
    const bool lds = (mx - mn + 3) <= kTile;
    if (lds) {
      const int span = mx - mn + 3;
      for (int k = tid; k < span; k += kBlock) {
        s_flux[k] = 0;
        s_E[k] = (T)E[wrap_or_clamp(*G, base + k)];
      }
      __syncthreads();
    }

    double ke = 0.0, lost = 0.0;
    unsigned long long n_abs = 0;
    bool bad = false;

#pragma unroll 1
    for (int j = 0; j < kItems; ++j) {
      const long long i = i0 + tid + (long long)j * kBlock;
      int c = cell[j];
      const bool act = c != kDead;
      int k = 0;
      T pn = (T)0, gam = (T)0;
      long long nq = 0;
      bool keep = false;
      if (act) {
        const T o = offA[i];
        const long long oq = (long long)(o * scale);
        T Em, Ec, Ep;
        if (lds) {
          Em = s_E[c - base - 1]; Ec = s_E[c - base]; Ep = s_E[c - base + 1];
        } else {
          Em = (T)E[wrap_or_clamp(*G, c - 1)];
          Ec = (T)E[c];
          Ep = (T)E[wrap_or_clamp(*G, c + 1)];
        }
        // gather: node averages, then linear in the offset
        const T el = half_t * (Em + Ec);
        const T er = half_t * (Ec + Ep);
        const T Epart = el + o * (er - el);
        // push and move
        pn = pA[i] + qdt * Epart;
        gam = sqrt(one_t + pn * pn);
        const T v = pn / gam;
        const T d = v * dtdx;
        const long long dq = (long long)rint(d * scale);
        nq = oq + dq;
        long long f1, f2 = 0;
        int cross = 0;  // -1, 0, +1: node crossed to the left / none / right
        int c2 = c;
        keep = true;
        if (nq >= ONE) {
          f1 = q * (ONE - oq);
          cross = 1;
          c2 = c + 1;
          nq -= ONE;
          f2 = q * nq;
          if (c2 >= nc) { if (absorbing) keep = false; else c2 = 0; }
        } else if (nq < 0) {
          f1 = q * (0 - oq);
          cross = -1;
          c2 = c - 1;
          nq += ONE;
          f2 = q * (nq - ONE);
          if (c2 < 0) { if (absorbing) keep = false; else c2 = nc - 1; }
        } else {
          f1 = q * dq;
        }
        const bool second = cross != 0 && keep;
        if (lds) {
          // tile indices are unwrapped: c - 1 .. c + 1 all lie in [base, base + span)
          atomicAdd((unsigned long long*)&s_flux[c - base], as_u64(f1));
          if (second) atomicAdd((unsigned long long*)&s_flux[c + cross - base], as_u64(f2));
        } else {
          atomicAdd((unsigned long long*)&G->F[c], as_u64(f1));
          if (second) atomicAdd((unsigned long long*)&G->F[c2], as_u64(f2));
        }
        if (!isfinite(pn) || !isfinite(gam)) bad = true;
        if (keep) {
          c = c2;
          // emission: repeated subtraction of gamma_pair while at or above threshold
          T gm = gam;
          while (gm >= gthr) {
            gm = gm - gpair;
            ++k;
            if (k > kMaxEmit) break;
          }
          if (k > kMaxEmit) { G->emit_err = 1; k = 0; }
          if (k > 0) {
            const T mag = sqrt(gm * gm - one_t);
            pn = pn > (T)0 ? mag : -mag;
          }
          pA[i] = pn;
          offA[i] = (T)nq * inv_scale;
          if (c != cell[j]) cellA[i] = c;
          if (diag) {
            const double pd = (double)pn;
            ke += w_d * sqrt(1.0 + pd * pd);
          }
        } else {
          const double pd = (double)pn;
          lost += w_d * sqrt(1.0 + pd * pd);
          ++n_abs;
          pA[i] = pn;
          cellA[i] = kDead;
        }
      }

      // ---- emission appends, aggregated per wave (wave-uniform section)
      const unsigned long long emitters = __ballot(k > 0);
      if (emitters) {
        const int incl = wave_incl_scan(k);
        const int excl = incl - k;
        const int tot = __shfl(incl, 63, 64);
        const int dir = pn > (T)0 ? 1 : -1;
        const uint64_t my_id = k > 0 ? G->id[buf][s][i] : 0;
        if (G->table_len == 0) {
          // pair made in place (the paper's zero mean free path)
          unsigned long long be = 0, bp = 0;
          if (lane == 63) {
            be = atomicAdd(&G->n_next[0], (unsigned long long)tot);
            bp = atomicAdd(&G->n_next[1], (unsigned long long)tot);
            atomicAdd(&G->photons_emitted, (unsigned long long)tot);
            atomicAdd(&G->pairs_created, (unsigned long long)tot);
            if (be + tot > (unsigned long long)G->cap || bp + tot > (unsigned long long)G->cap)
              G->overflow = 1;
          }
          be = __shfl(be, 63, 64);
          bp = __shfl(bp, 63, 64);
          const unsigned long long cap = (unsigned long long)G->cap;
          const T pc = dir > 0 ? pchild : -pchild;
          const T offn = (T)nq * inv_scale;
          for (int jj = 0; jj < k; ++jj) {
            const U64x4 u = philox4x64_10((uint64_t)stepn, (uint64_t)jj, kTagPhoton, 0, my_id, G->seed);
            const uint64_t child = u.v[1] & ~(uint64_t)1;
            const unsigned long long se = be + excl + jj, sp = bp + excl + jj;
            const int nb = buf;
            if (se < cap) {
              G->cell[nb][0][se] = c; ((T*)G->off[nb][0])[se] = offn;
              ((T*)G->p[nb][0])[se] = pc; G->id[nb][0][se] = child;
            }
            if (sp < cap) {
              G->cell[nb][1][sp] = c; ((T*)G->off[nb][1])[sp] = offn;
              ((T*)G->p[nb][1])[sp] = pc; G->id[nb][1][sp] = child | 1u;
            }
          }
          if (diag) ke += (double)k * 2.0 * w_d * G->child_gamma64;
        } else {
          unsigned long long bph = 0;
          if (lane == 63) {
            bph = atomicAdd(&G->n_ph_next, (unsigned long long)tot);
            atomicAdd(&G->photons_emitted, (unsigned long long)tot);
            atomicAdd(&G->inflight, (unsigned long long)tot);
            if (bph + tot > (unsigned long long)G->ph_cap) G->overflow = 1;
          }
          bph = __shfl(bph, 63, 64);
          const unsigned long long cap = (unsigned long long)G->ph_cap;
          const int pb = G->phbuf;
          unsigned long long esc = 0;
          const long long X0 = (long long)c * ONE + nq;
          for (int jj = 0; jj < k; ++jj) {
            const U64x4 u = philox4x64_10((uint64_t)stepn, (uint64_t)jj, kTagPhoton, 0, my_id, G->seed);
            const uint64_t child = u.v[1] & ~(uint64_t)1;
            const int ncv = conv_steps(G->table, G->table_len, (uint32_t)(u.v[0] >> 32));
            long long X = X0 + (long long)dir * (long long)ncv * G->photon_step;
            int cstep = (int)(stepn + ncv);
            if (absorbing) {
              if (X < 0 || X >= G->domain) { cstep = INT32_MIN; ++esc; }
            } else {
              X %= G->domain;
              if (X < 0) X += G->domain;
            }
            const unsigned long long slot = bph + excl + jj;
            if (slot < cap) {
              G->ph_x[pb][slot] = X;
              G->ph_step[pb][slot] = cstep;
              G->ph_child[pb][slot] = child | (dir > 0 ? 1u : 0u);
            }
          }
          const unsigned long long esc_w = wave_sum(esc);
          if (esc > 0) lost += (double)esc * w_d * G->gpair64;
          if (lane == 63 && esc_w > 0) {
            atomicAdd(&G->photons_escaped, esc_w);
            atomicAdd(&G->inflight, (unsigned long long)(-(long long)esc_w));
          }
        }
      }
    }

    // ---- per-wave tallies
    const double ke_w = wave_sum(ke);
    const double lost_w = wave_sum(lost);
    const unsigned long long abs_w = wave_sum(n_abs);
    const unsigned long long bad_w = __ballot(bad);
    if (lane == 0) {
      if (diag && ke_w != 0.0) atomicAdd(&G->ke_acc, ke_w);
      if (abs_w) {
        atomicAdd(&G->absorbed[s], abs_w);
        atomicAdd(&G->dead[s], abs_w);
      }
      if (lost_w != 0.0) atomicAdd(&G->lost_energy, lost_w);
      if (bad_w) G->nonfinite = 1;
    }

    if (lds) {
      __syncthreads();
      const int span = mx - mn + 3;
      for (int k = tid; k < span; k += kBlock) {
        const long long f = s_flux[k];
        if (f != 0) {
          int cc = base + k;
          if (cc < 0) cc += nc;
          else if (cc >= nc) cc -= nc;
          atomicAdd((unsigned long long*)&G->F[cc], as_u64(f));
        }
      }
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------- field
__global__ __launch_bounds__(kBlock) void k_field(GapDev* __restrict__ gaps,
                                                  const long long* __restrict__ cwi, int B) {
  __shared__ double s_red[8];
  const int g = find_gap(cwi, B, blockIdx.x);
  GapDev* __restrict__ G = gaps + g;
  if (G->status != PIC_OK) return;
  const long long c0 = (blockIdx.x - cwi[g]) * (long long)kCellChunk;
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
template <typename T>
__global__ __launch_bounds__(kBlock) void k_convert(GapDev* __restrict__ gaps,
                                                    const long long* __restrict__ pwi, int B) {
  const long long total = pwi[B];
  long long w0, w1;
  xcd_range(total, w0, w1);
  const int lane = lane_id();
  for (long long w = w0; w < w1; ++w) {
    const int g = find_gap(pwi, B, w);
    GapDev* __restrict__ G = gaps + g;
    if (G->status != PIC_OK) continue;
    const int pb = G->phbuf, buf = G->buf;
    const long long i0 = (w - pwi[g]) * (long long)kPhChunk;
    const long long nP = (long long)G->n_ph;
    const long long i1 = i0 + kPhChunk < nP ? i0 + kPhChunk : nP;
    const int stepn = (int)G->step;
    const bool diag = ((long long)stepn % G->diag_every) == 0;
    const long long ONE = G->one;
    const T inv_scale = (T)(1.0 / (double)ONE);
    const T pchild = (T)G->pchild;
    const unsigned long long cap = (unsigned long long)G->cap;
    for (long long i = i0 + threadIdx.x; i - threadIdx.x < i1; i += kBlock) {
      const bool due = i < i1 && G->ph_step[pb][i] == stepn;
      const unsigned long long m = __ballot(due);
      if (!m) continue;
      const int cnt = __popcll(m);
      const int rank = __popcll(m & ((1ull << lane) - 1ull));
      unsigned long long be = 0, bp = 0;
      if (lane == 0) {
        be = atomicAdd(&G->n_next[0], (unsigned long long)cnt);
        bp = atomicAdd(&G->n_next[1], (unsigned long long)cnt);
        atomicAdd(&G->pairs_created, (unsigned long long)cnt);
        atomicAdd(&G->inflight, (unsigned long long)(-(long long)cnt));
        if (be + cnt > cap || bp + cnt > cap) G->overflow = 1;
        if (diag) atomicAdd(&G->ke_acc, (double)cnt * 2.0 * G->weight * G->child_gamma64);
      }
      be = __shfl(be, 0, 64);
      bp = __shfl(bp, 0, 64);
      if (due) {
        const long long X = G->ph_x[pb][i];
        const uint64_t ch = G->ph_child[pb][i];
        const int c = (int)(X / ONE);
        const T offn = (T)(X % ONE) * inv_scale;
        const T pc = (ch & 1u) ? pchild : -pchild;
        const uint64_t child = ch & ~(uint64_t)1;
        const unsigned long long se = be + rank, sp = bp + rank;
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
  }
}

// ------------------------------------------------------------ plans
// Work-item prefixes of the next launches: particle chunks per gap (both
// species) and photon chunks per gap; frozen gaps get none.
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
      sb += ((long long)G->n_ph + kPhChunk - 1) / kPhChunk;
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
      rb += ((long long)G->n_ph + kPhChunk - 1) / kPhChunk;
    }
  }
  if (tid == nt - 1) { wi[B] = s_a[nt - 1]; pwi[B] = s_b[nt - 1]; }
}

__global__ __launch_bounds__(1024) void k_plan(GapDev* __restrict__ gaps, int B,
                                               long long* __restrict__ wi,
                                               long long* __restrict__ pwi) {
  compute_plans(gaps, B, wi, pwi);
}

__global__ __launch_bounds__(1024) void k_finalize(GapDev* __restrict__ gaps, int B,
                                                   long long* __restrict__ wi,
                                                   long long* __restrict__ pwi) {
  for (int g = threadIdx.x; g < B; g += blockDim.x) {
    GapDev* G = gaps + g;
    if (G->status == PIC_OK) {
      int st = PIC_OK;
      if (G->nonfinite) st = PIC_ERR_NONFINITE;
      else if (G->overflow) st = PIC_ERR_CAPACITY;
      else if (G->emit_err) st = PIC_ERR_EMISSION;
      if (st != PIC_OK) {
        G->status = st;
      } else {
        G->pushes += G->live[0] + G->live[1];
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
          G->hist_count += 1;
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

// ------------------------------------------------------------------ sort
// Lanes holding the same cell in a row of a wave form a run; the first lane
// of a run (its head) does one atomic for the whole run.
__device__ __forceinline__ void wave_runs(int cv, unsigned long long& heads, int& head_lane,
                                          int& run_len) {
  const int lane = lane_id();
  const int prev = __shfl_up(cv, 1, 64);
  const bool head = lane == 0 || cv != prev;
  heads = __ballot(head);
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
  if (blockIdx.x == cwi[g] && threadIdx.x == 0) { G->sorted_n[0] = 0; G->sorted_n[1] = 0; G->ph_sorted = 0; }
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
    int32_t* __restrict__ cnt = G->sort_cnt[s];
    for (int j = 0; j < kItems; ++j) {
      const long long i = i0 + threadIdx.x + (long long)j * kBlock;
      const int cv = i < i1 ? G->cell[buf][s][i] : kDead;
      unsigned long long heads;
      int head_lane, run_len;
      wave_runs(cv, heads, head_lane, run_len);
      if (PASS == 0) {
        if (run_len > 0 && cv != kDead) atomicAdd(&cnt[cv], run_len);
      } else {
        int b = 0;
        if (run_len > 0 && cv != kDead) b = atomicAdd(&cnt[cv], run_len);
        b = __shfl(b, head_lane, 64);
        if (cv != kDead) {
          const long long dst = (long long)b + (lane - head_lane);
          const int nb = buf ^ 1;
          G->cell[nb][s][dst] = cv;
          G->id[nb][s][dst] = G->id[buf][s][i];
          if (elem_bytes == 8) {
            ((double*)G->off[nb][s])[dst] = ((const double*)G->off[buf][s])[i];
            ((double*)G->p[nb][s])[dst] = ((const double*)G->p[buf][s])[i];
          } else {
            ((float*)G->off[nb][s])[dst] = ((const float*)G->off[buf][s])[i];
            ((float*)G->p[nb][s])[dst] = ((const float*)G->p[buf][s])[i];
          }
        }
      }
    }
  }
}

// Exclusive scan of the per-cell counts of one (gap, species) in place.
__global__ __launch_bounds__(1024) void k_sort_scan(GapDev* __restrict__ gaps, int B) {
  __shared__ long long s_sum[1024];
  const int g = blockIdx.x >> 1, s = blockIdx.x & 1;
  GapDev* __restrict__ G = gaps + g;
  if (G->status != PIC_OK) return;
  const int nc = G->n_cells, tid = threadIdx.x, nt = blockDim.x;
  const int per = (nc + nt - 1) / nt;
  int32_t* __restrict__ cnt = G->sort_cnt[s];
  long long loc = 0;
  for (int c = tid * per; c < (tid + 1) * per && c < nc; ++c) loc += cnt[c];
  s_sum[tid] = loc;
  __syncthreads();
  for (int d = 1; d < nt; d <<= 1) {
    long long y = tid >= d ? s_sum[tid - d] : 0;
    __syncthreads();
    s_sum[tid] += y;
    __syncthreads();
  }
  long long run = s_sum[tid] - loc;
  for (int c = tid * per; c < (tid + 1) * per && c < nc; ++c) {
    const int v = cnt[c];
    cnt[c] = (int32_t)run;
    run += v;
  }
  if (tid == nt - 1) G->sorted_n[s] = (unsigned long long)s_sum[nt - 1];
}

__global__ __launch_bounds__(kBlock) void k_photon_compact(GapDev* __restrict__ gaps,
                                                           const long long* __restrict__ pwi, int B) {
  const long long total = pwi[B];
  long long w0, w1;
  xcd_range(total, w0, w1);
  const int lane = lane_id();
  for (long long w = w0; w < w1; ++w) {
    const int g = find_gap(pwi, B, w);
    GapDev* __restrict__ G = gaps + g;
    if (G->status != PIC_OK) continue;
    const int pb = G->phbuf;
    const long long i0 = (w - pwi[g]) * (long long)kPhChunk;
    const long long nP = (long long)G->n_ph;
    const long long i1 = i0 + kPhChunk < nP ? i0 + kPhChunk : nP;
    const long long stepn = G->step;
    for (long long i = i0 + threadIdx.x; i - threadIdx.x < i1; i += kBlock) {
      const bool keep = i < i1 && (long long)G->ph_step[pb][i] >= stepn;
      const unsigned long long m = __ballot(keep);
      if (!m) continue;
      const int cnt = __popcll(m);
      const int rank = __popcll(m & ((1ull << lane) - 1ull));
      unsigned long long b = 0;
      if (lane == 0) b = atomicAdd(&G->ph_sorted, (unsigned long long)cnt);
      b = __shfl(b, 0, 64);
      if (keep) {
        const unsigned long long d = b + rank;
        G->ph_x[pb ^ 1][d] = G->ph_x[pb][i];
        G->ph_step[pb ^ 1][d] = G->ph_step[pb][i];
        G->ph_child[pb ^ 1][d] = G->ph_child[pb][i];
      }
    }
  }
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
    G->n_ph = G->ph_sorted;
    G->n_ph_next = G->ph_sorted;
    G->phbuf ^= 1;
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
  if (mixed) hipLaunchKernelGGL(k_push<float>, dim3(L.push_grid), dim3(kBlock), 0, L.stream, L.gaps, L.wi, L.B);
  else hipLaunchKernelGGL(k_push<double>, dim3(L.push_grid), dim3(kBlock), 0, L.stream, L.gaps, L.wi, L.B);
  return hipGetLastError();
}

hipError_t launch_step(const StepLaunch& L, bool mixed) {
  hipError_t e = launch_push(L, mixed);
  if (e != hipSuccess) return e;
  return launch_step_after_push(L, mixed);
}

hipError_t launch_step_after_push(const StepLaunch& L, bool mixed) {
  hipLaunchKernelGGL(k_field, dim3(grid_for(L.cell_items, 1 << 30)), dim3(kBlock), 0, L.stream, L.gaps, L.cwi, L.B);
  if (mixed) hipLaunchKernelGGL(k_convert<float>, dim3(L.conv_grid), dim3(kBlock), 0, L.stream, L.gaps, L.pwi, L.B);
  else hipLaunchKernelGGL(k_convert<double>, dim3(L.conv_grid), dim3(kBlock), 0, L.stream, L.gaps, L.pwi, L.B);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, L.stream, L.gaps, L.B, L.wi, L.pwi);
  return hipGetLastError();
}

hipError_t launch_sort(const StepLaunch& L, bool mixed) {
  const int eb = mixed ? 4 : 8;
  hipLaunchKernelGGL(k_sort_zero, dim3(grid_for(L.cell_items, 1 << 30)), dim3(kBlock), 0, L.stream, L.gaps, L.cwi, L.B);
  hipLaunchKernelGGL(k_sort_pass<0>, dim3(L.push_grid), dim3(kBlock), 0, L.stream, L.gaps, L.wi, L.B, eb);
  hipLaunchKernelGGL(k_sort_scan, dim3(2 * L.B), dim3(1024), 0, L.stream, L.gaps, L.B);
  hipLaunchKernelGGL(k_sort_pass<1>, dim3(L.push_grid), dim3(kBlock), 0, L.stream, L.gaps, L.wi, L.B, eb);
  hipLaunchKernelGGL(k_photon_compact, dim3(L.conv_grid), dim3(kBlock), 0, L.stream, L.gaps, L.pwi, L.B);
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
