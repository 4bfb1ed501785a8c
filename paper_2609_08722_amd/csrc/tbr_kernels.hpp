// tbr_kernels.hpp -- kernel argument blocks and launch-facing declarations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tbr_device.hpp"

namespace tbr {

struct KProgram {
  int n, k;
  const float *cx, *cy, *angle, *length, *half_width, *logits, *palette;
};

struct KOpts {
  float tau, tau_min, tau_c, eps;
  const float* coupling;  // [N][3] c_1..c_3 of the calibrated coupling, or null (uniform)
};

// Replay tape (all device memory, pixel-minor so a wave's accesses coalesce).
struct KTape {
  double2* ckpt_xy;    // [n_ckpt][P]: position of states x_0, x_k, x_2k, ... (FP64)
  float2* ckpt_t;      // [n_ckpt][P]: their transmittance (Tm, Te), T = Tm 2^Te
  int32_t* nrec;       // [P] records pushed per pixel
  int32_t* side_idx;   // [side_slots][P] stroke index of each record
  double2* side_xy;    // [side_slots][P] position x_i at the record (FP64)
  int32_t* status;     // [1] max records over pixels (atomicMax)
  int ckpt_interval;   // k (0: only the final state)
  int side_slots;      // per-pixel capacity
};

// Optional L2 seed computed at the end of the soft trace (fit step).
struct KSeed {
  const float* target;  // [P*3] or null
  float* grad_rgb;      // [P*3] dL/dR
  float* loss_part;     // [n_blocks] sum of squared errors per block
};

struct KGrad {
  float *cx, *cy, *angle, *length, *half_width, *logits, *palette;
};

// One admitted serving request (device copy, read by k_serve).
struct ServeDesc {
  const StrokeRec* recs;  // prepared records of the request's program and options
  const float* palette;   // [K*3]
  float* rgb;             // [H*W*3] or null (hard)
  int32_t* label;         // [H*W] or null
  int32_t* owner;         // [H*W] or null
  int n, width, height, tiles_x;
  int soft;               // 1 soft composite, 0 hard
  int pad[3];
};

// Stroke preparation of one request of a serving tick (read by k_serve_prep).
struct ServePrep {
  KProgram prog;
  KOpts opts;
  StrokeRec* out;  // the request's records in the arena
  int block0;      // first block of this request in the tick's prep launch
  int pad;
};

// One job of the fused multi-job fit (passed by value in the kernel arguments).
struct FitJobK {
  const StrokeRec* recs;
  const float4* coup;   // profile cubics (coupled launches only)
  const float* palette;
  const float* target;  // [P*3]
  float* partial;       // [tiles][n + 1][8]
  float* loss_part;     // [tiles]
  KTape tape;
  int n, width, height, tiles_x, item0;
};
constexpr int kMaxFitJobs = 16;
struct FitJobsK {
  FitJobK job[kMaxFitJobs];
  int n_jobs, n_items;
};

struct KAdam {
  float lr_centre, lr_angle, lr_length, lr_width, lr_logits, lr_palette;
  float beta1, beta2, eps, bc1, bc2;
  float r_lo, r_hi, l_max;
};

// Parameter windows of the fitting loop (derived from tbr_window_opts).
struct KWindow {
  float a_lo, a_span, l_max;
  float r0_first, r0_log_ratio;  // r0_i = r0_first exp(r0_log_ratio i / (N - 1))
  float r_lo_frac, r_span_frac;
  float lambda_length, lambda_area;
};

__global__ void k_stroke_prep(KProgram p, KOpts o, StrokeRec* out, int32_t* status, float4* coup);
__global__ void k_window_map(const float* th, float* nat, int n, int kpal, KWindow w);
__global__ void k_reg_loss(const float* nat, int n, KWindow w, float* loss);
__global__ void k_window_adam(float* th, const float* g_nat, float* m, float* v, int n, int kpal,
                              KWindow w, KAdam a, const int32_t* records, int capacity);
// Transport variants of the per-pixel kernels (the values of
// tbr_render_opts.transport): the capsule map, its calibrated coupling (coup
// = per-stroke profile cubics), the inert-mark model (no displacement), and
// the sixteen drops of R_D.
constexpr int kCapsule = 0, kCoupled = 1, kInert = 2, kDrops = 3;

template <int kT>
__global__ void k_trace_soft(const StrokeRec* recs, const float4* coup, int n, int width,
                             int height, const float* palette, float* rgb, KTape tape, KSeed seed);
template <int kT>
__global__ void k_trace_hard(const StrokeRec* recs, const float4* coup, int n, int width,
                             int height, const float* palette, float* rgb, int32_t* label,
                             int32_t* owner);
template <int kT>
__global__ void k_replay(const StrokeRec* recs, const float4* coup, int n, int width, int height,
                         const float* palette, const float* grad_rgb, KTape tape, float* partial);
__global__ void k_sum_tiles(const float* partial, int rows8, int n_tiles, int tiles_per_group,
                            double* out);
__global__ void k_finalize(const double* groups, int n_groups, KProgram p, KOpts o, KGrad grad,
                           float* gcol, float* pal_terms);
__global__ void k_palette_grad(const float* pal_terms, int n, int kpal, const float* gcol,
                               float* gpal);
__global__ void k_loss_final(const float* part, int n_part, float inv_count, float* loss);
__global__ void k_adam(float* prm, const float* grd, float* m, float* v, int n, int kpal, KAdam a,
                       const int32_t* records, int capacity);
// Waves per SIMD of the fused fit kernel (its launch bound). The forward and
// the replay share one register allocation there, so the bound trades
// registers for occupancy per transport, as measured at 1024^2 x 2000
// (bitwise the same results at every bound). The capsule map at 7 waves
// (72 VGPRs; its spills are of values that live across a tile or a
// 16-stroke chunk, and one reload in the forward's checkpoint store) runs
// 1.6-1.9% faster than at 6 (80 VGPRs), 4-5% faster than at 4 or 5 (98 / 96
// VGPRs, no spill) and 5% faster than at 8 (64 VGPRs, spills in the stroke
// loops). Programs of long strokes put many more steps on the flank's and
// the general map's far steps, which need more registers: the fitting loop
// of Table hyper (offsets up to 0.3 per component) runs 4.7% faster at 6
// waves than at 7 at every stage of its annealing, so the capsule map has a
// 6-wave instantiation for such programs (kFusedWavesLong). The coupled map,
// with more live values, is fastest at 5; R_U and R_D run at 7.
template <int kT>
constexpr int kFusedWaves = kT == kCoupled ? 5 : 7;
constexpr int kFusedWavesLong = 6;
template <int kT, int kW>
__global__ void k_fit_fused(FitJobsK jobs, int* cursor);
__global__ void k_serve(const ServeDesc* descs, const uint2* items, int n_items, int* cursor);
__global__ void k_serve_prep(const ServePrep* preps, int n_req);
__global__ void k_fill_i32(int32_t* p, int n, int v);
constexpr int kCompThreadsK = 1024;  // the compensation's one workgroup
__global__ void k_compensate(KProgram p, float eps, int endpoint, int skip, double2* pts,
                             float* ocx, float* ocy, float* oangle, float* olength,
                             int32_t* blocked);

}  // namespace tbr
