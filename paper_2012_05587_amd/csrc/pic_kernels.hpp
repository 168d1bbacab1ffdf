// Launchers of the device kernels, called by the host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include "pic_device.hpp"

namespace pic {

struct StepLaunch {
  GapDev* gaps;        // device array of B descriptors
  long long* wi;       // particle work-item prefix, B + 1 entries (device)
  long long* pwi;      // due-photon work-item prefix, B + 1 entries (device)
  long long* qwi;      // photon-store work-item prefix (re-sort), B + 1 entries (device)
  long long* twi;      // work-item prefix of the tail sort, B + 1 entries (device)
  long long* cwi;      // cell work-item prefix, B + 1 entries (device, static)
  long long* items;    // the finalize's per-gap item counts of the next step, 3 x B (device)
  long long cell_items;
  int B;
  int push_grid, conv_grid, emit_grid, ph_sort_grid;
  int32_t* emit_cnt;   // emitters per chunk of the current plan (device)
  uint32_t* emit_ent;  // kChunk entries per chunk (device)
  uint32_t* wg_emit;   // emitters listed by each push workgroup, kPushGrid entries (device)
  unsigned long long* stripes;  // striped push tallies, B x 4 x kStripes x kStripeStride (device)
  hipStream_t stream;
  bool spread;         // some gap draws per-lepton thresholds (gamma_thr_spread > 0)
  bool spline;         // the batch's leptons have the quadratic-spline shape
};

hipError_t launch_step(const StepLaunch& L, bool mixed);
// start/stop (both or neither): events recorded by the push dispatch itself
hipError_t launch_push(const StepLaunch& L, bool mixed, hipEvent_t start, hipEvent_t stop);
hipError_t launch_step_after_push(const StepLaunch& L, bool mixed);
hipError_t launch_sort(const StepLaunch& L, bool mixed);
hipError_t launch_tail_sort(const StepLaunch& L, bool mixed);
hipError_t launch_plan(const StepLaunch& L);
hipError_t launch_seed(GapDev* gaps, int g, int mode, long long N, double p0m, double p0p,
                       long long base0, long long base1, bool mixed, hipStream_t st);
hipError_t launch_phase(GapDev* gaps, int g, int s, int x_bins, int p_bins, double p_min, double inv_dp,
                        unsigned long long* out, bool mixed, hipStream_t st);
hipError_t launch_zero(long long* a, long long n, hipStream_t st);
hipError_t launch_rho(GapDev* gaps, int g, long long* rho_acc, long long n_nodes, bool mixed,
                      hipStream_t st);
// Static node scratch (kStaticNodes int64 per GPU): its device address on
// `device`, looked up on first use.
constexpr long long kStaticNodes = (1 << 20) + 1;
constexpr int kMaxDevices = 64;
hipError_t static_scratch(int device, long long** out);

}  // namespace pic
