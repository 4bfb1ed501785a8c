// tbr_api.hip -- host side of the C ABI declared in include/tbr.h:
// argument validation, workspace layout and kernel launches.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "tbr.h"
#include "tbr_kernels.hpp"

using namespace tbr;

namespace tbr {
thread_local std::string g_err;  // last error message of this thread (all entry points)
}  // namespace tbr

namespace {

tbr_status fail(tbr_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
tbr_status fail(tbr_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

tbr_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(TBR_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return TBR_OK;
}

// Benchmark timing hook (tbr_set_timing_events).
thread_local std::string g_timed_kernel;
thread_local hipEvent_t g_ev_begin = nullptr, g_ev_end = nullptr;

struct Timed {
  bool on;
  hipStream_t st;
  Timed(const char* name, hipStream_t s) : on(g_ev_begin && g_timed_kernel == name), st(s) {
    if (on) (void)hipEventRecord(g_ev_begin, st);
  }
  ~Timed() {
    if (on) (void)hipEventRecord(g_ev_end, st);
  }
};

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

constexpr int kTile = 16;  // pixels per block side (4 waves of 8x8)

int tiles_x(const tbr_render_opts* o) { return (o->width + kTile - 1) / kTile; }
int tiles_y(const tbr_render_opts* o) { return (o->height + kTile - 1) / kTile; }
size_t n_tiles(const tbr_render_opts* o) { return (size_t)tiles_x(o) * tiles_y(o); }
size_t n_pixels(const tbr_render_opts* o) { return (size_t)o->width * o->height; }

int n_ckpt(const tbr_render_opts* o, int n) {
  if (o->ckpt_interval <= 0 || n <= 1) return 1;
  return 1 + (n - 1) / o->ckpt_interval;
}

bool coupled(const tbr_render_opts* o) { return o->transport == TBR_TRANSPORT_COUPLED; }

// Render workspace: [recs][status][coup][tape: nrec | ckpt | side_idx | side_xy]
// (coup: the strokes' profile cubics, coupled transport only)
struct RenderLayout {
  size_t recs, status, coup, nrec, ckpt_xy, ckpt_t, side_idx, side_xy, total;
};

RenderLayout render_layout(const tbr_render_opts* o, int n, bool tape) {
  RenderLayout L{};
  size_t off = 0;
  L.recs = off;
  off = align_up(off + (size_t)(n > 0 ? n : 1) * sizeof(StrokeRec));
  L.status = off;
  off = align_up(off + 64);
  if (coupled(o)) {
    L.coup = off;
    off = align_up(off + (size_t)(n > 0 ? n : 1) * sizeof(float4));
  }
  if (tape) {
    size_t P = n_pixels(o);
    L.nrec = off;
    off = align_up(off + P * sizeof(int32_t));
    L.ckpt_xy = off;
    off = align_up(off + (size_t)n_ckpt(o, n) * P * sizeof(double2));
    L.ckpt_t = off;
    off = align_up(off + (size_t)n_ckpt(o, n) * P * sizeof(float2));
    L.side_idx = off;
    off = align_up(off + (size_t)o->side_slots * P * sizeof(int32_t));
    L.side_xy = off;
    off = align_up(off + (size_t)o->side_slots * P * sizeof(double2));
  }
  L.total = off;
  return L;
}

constexpr int kGroups = 32;  // first-stage groups of the tile sum

struct BackLayout {
  size_t partial, groups, gcol, pal_terms, total;
};

BackLayout back_layout(const tbr_render_opts* o, int n, int k) {
  BackLayout L{};
  size_t rows8 = (size_t)(n + 1) * 8, off = 0;
  L.partial = off;
  off = align_up(off + n_tiles(o) * rows8 * sizeof(float));
  L.groups = off;
  off = align_up(off + (size_t)kGroups * rows8 * sizeof(double));
  L.gcol = off;
  off = align_up(off + (size_t)(n + 1) * 3 * sizeof(float));
  L.pal_terms = off;
  off = align_up(off + (size_t)(n > 0 ? n : 1) * k * 3 * sizeof(float));
  L.total = off;
  return L;
}

struct FitLayout {
  RenderLayout r;
  BackLayout b;
  size_t base_r, base_b, loss_part, grads, cursor, seed, total;
};

size_t packed_len(int n, int k) { return (size_t)5 * n + (size_t)n * k + (size_t)3 * k; }

FitLayout fit_layout(const tbr_render_opts* o, int n, int k) {
  FitLayout L{};
  L.r = render_layout(o, n, true);
  L.b = back_layout(o, n, k);
  size_t off = 0;
  L.base_r = off;
  off = align_up(off + L.r.total);
  L.base_b = off;
  off = align_up(off + L.b.total);
  L.loss_part = off;
  off = align_up(off + n_tiles(o) * sizeof(float));
  L.grads = off;
  off = align_up(off + packed_len(n, k) * sizeof(float));
  L.cursor = off;  // work cursor of the fused launch (single-job step)
  off = align_up(off + sizeof(int));
  if (o->transport == TBR_TRANSPORT_INERT) {  // dL/dR between the two kernels (no fused launch)
    L.seed = off;
    off = align_up(off + n_pixels(o) * 3 * sizeof(float));
  }
  L.total = off;
  return L;
}

tbr_status check_opts(const tbr_render_opts* o, bool soft, bool tape) {
  if (!o) return fail(TBR_E_INVALID, "opts is NULL");
  if (o->width < 1 || o->width > 16384 || o->height < 1 || o->height > 16384)
    return fail(TBR_E_INVALID, "canvas %dx%d outside 1..16384", o->width, o->height);
  if (!(o->tau >= 0.f) || !std::isfinite(o->tau)) return fail(TBR_E_INVALID, "tau must be >= 0");
  if (soft && !(o->tau_min > 0.f)) return fail(TBR_E_INVALID, "tau_min must be > 0 for soft renders");
  if (!(o->tau_c >= 0.f) || !std::isfinite(o->tau_c)) return fail(TBR_E_INVALID, "tau_c must be >= 0");
  if (!(o->eps_floor > 0.f) || !std::isfinite(o->eps_floor))
    return fail(TBR_E_INVALID, "eps_floor must be > 0");
  if (o->ckpt_interval < 0) return fail(TBR_E_INVALID, "ckpt_interval must be >= 0");
  if (tape && o->side_slots < 1) return fail(TBR_E_INVALID, "side_slots must be >= 1 with a tape");
  if (o->side_slots < 0) return fail(TBR_E_INVALID, "side_slots must be >= 0");
  if (o->transport < TBR_TRANSPORT_CAPSULE || o->transport > TBR_TRANSPORT_DROPS16)
    return fail(TBR_E_INVALID, "transport %d is not a TBR_TRANSPORT_* value", o->transport);
  if (coupled(o) && !o->coupling)
    return fail(TBR_E_INVALID, "the coupled transport needs the coupling coefficients");
  return TBR_OK;
}

tbr_status check_prog(const tbr_program* p) {
  if (!p) return fail(TBR_E_INVALID, "program is NULL");
  if (p->n_strokes < 0) return fail(TBR_E_INVALID, "n_strokes = %d < 0", p->n_strokes);
  if (p->n_palette < 1 || p->n_palette > 64)
    return fail(TBR_E_INVALID, "n_palette = %d outside 1..64", p->n_palette);
  if (!p->palette) return fail(TBR_E_INVALID, "palette is NULL");
  if (p->n_strokes > 0 && (!p->cx || !p->cy || !p->angle || !p->length || !p->half_width || !p->logits))
    return fail(TBR_E_INVALID, "a stroke array is NULL");
  return TBR_OK;
}

KProgram kprog(const tbr_program* p) {
  return KProgram{p->n_strokes, p->n_palette, p->cx, p->cy, p->angle, p->length,
                  p->half_width, p->logits, p->palette};
}
KOpts kopts(const tbr_render_opts* o) {
  return KOpts{o->tau, o->tau_min, o->tau_c, o->eps_floor, coupled(o) ? o->coupling : nullptr};
}

float4* coup_of(char* ws, const RenderLayout& L, const tbr_render_opts* o) {
  return coupled(o) ? reinterpret_cast<float4*>(ws + L.coup) : nullptr;
}

KTape ktape(char* ws, const RenderLayout& L, const tbr_render_opts* o, bool tape) {
  KTape t{};
  t.status = reinterpret_cast<int32_t*>(ws + L.status);
  t.ckpt_interval = o->ckpt_interval;
  t.side_slots = o->side_slots;
  if (tape) {
    t.ckpt_xy = reinterpret_cast<double2*>(ws + L.ckpt_xy);
    t.ckpt_t = reinterpret_cast<float2*>(ws + L.ckpt_t);
    t.nrec = reinterpret_cast<int32_t*>(ws + L.nrec);
    t.side_idx = reinterpret_cast<int32_t*>(ws + L.side_idx);
    t.side_xy = reinterpret_cast<double2*>(ws + L.side_xy);
  }
  return t;
}

tbr_status launch_prep(const tbr_program* p, const tbr_render_opts* o, StrokeRec* recs,
                       int32_t* status, float4* coup, hipStream_t st) {
  int nb = (p->n_strokes + 255) / 256;
  if (nb < 1) nb = 1;
  k_stroke_prep<<<nb, 256, 0, st>>>(kprog(p), kopts(o), recs, status, coup);
  return check_launch("stroke_prep");
}

// Deterministic reduction of the tiles' partial rows and the chain rule to
// the program arrays (shared by the backward and both fit steps).
tbr_status launch_reduce(const tbr_program* p, const tbr_render_opts* o, const tbr_program_grad* g,
                         char* ws, const BackLayout& BL, hipStream_t st) {
  const int n = p->n_strokes;
  float* partial = reinterpret_cast<float*>(ws + BL.partial);
  double* groups = reinterpret_cast<double*>(ws + BL.groups);
  float* gcol = reinterpret_cast<float*>(ws + BL.gcol);
  int rows8 = (n + 1) * 8;
  int nt = (int)n_tiles(o);
  int tpg = (nt + kGroups - 1) / kGroups;
  k_sum_tiles<<<dim3((rows8 + 255) / 256, kGroups), 256, 0, st>>>(partial, rows8, nt, tpg, groups);
  tbr_status s = check_launch("sum_tiles");
  if (s) return s;
  KGrad kg{g->cx, g->cy, g->angle, g->length, g->half_width, g->logits, g->palette};
  float* pal_terms = reinterpret_cast<float*>(ws + BL.pal_terms);
  k_finalize<<<(n + 1 + 255) / 256, 256, 0, st>>>(groups, kGroups, kprog(p), kopts(o), kg, gcol,
                                                  pal_terms);
  if ((s = check_launch("finalize"))) return s;
  k_palette_grad<<<p->n_palette * 3, 256, 0, st>>>(pal_terms, n, p->n_palette, gcol, g->palette);
  return check_launch("palette_grad");
}

// The fused fit kernel over the jobs' (job, tile) items; the cursor is
// cleared by a fill kernel (no memset node if the caller captures a graph).
// long_strokes selects the capsule map's 6-wave instantiation (programs
// whose strokes may be long; see kFusedWavesLong).
tbr_status launch_fused(const FitJobsK& K, int* cursor, int transport, bool long_strokes,
                        hipStream_t st) {
  k_fill_i32<<<1, 64, 0, st>>>(cursor, 1, 0);
  tbr_status s = check_launch("fill");
  if (s) return s;
  {
    Timed tm("fit_fused", st);
    const int grid = std::min(K.n_items, 256 * 8);
    switch (transport) {
      case kCoupled:
        k_fit_fused<kCoupled, kFusedWaves<kCoupled>><<<grid, 256, 0, st>>>(K, cursor);
        break;
      case kInert: k_fit_fused<kInert, kFusedWaves<kInert>><<<grid, 256, 0, st>>>(K, cursor); break;
      case kDrops: k_fit_fused<kDrops, kFusedWaves<kDrops>><<<grid, 256, 0, st>>>(K, cursor); break;
      default:
        if (long_strokes)
          k_fit_fused<kCapsule, kFusedWavesLong><<<grid, 256, 0, st>>>(K, cursor);
        else
          k_fit_fused<kCapsule, kFusedWaves<kCapsule>><<<grid, 256, 0, st>>>(K, cursor);
        break;
    }
  }
  return check_launch("fit_fused");
}

tbr_status launch_backward(const tbr_program* p, const tbr_render_opts* o, const char* tape_ws,
                           const RenderLayout& RL, const float* grad_rgb, const tbr_program_grad* g,
                           char* ws, const BackLayout& BL, hipStream_t st) {
  const int n = p->n_strokes;
  KTape t = ktape(const_cast<char*>(tape_ws), RL, o, true);
  float* partial = reinterpret_cast<float*>(ws + BL.partial);
  const StrokeRec* recs = reinterpret_cast<const StrokeRec*>(tape_ws + RL.recs);
  const float4* coup = coup_of(const_cast<char*>(tape_ws), RL, o);
  dim3 grid(tiles_x(o), tiles_y(o));
  {
    Timed tm("replay", st);
    const int W = o->width, H = o->height;
    switch (o->transport) {
      case kCoupled:
        k_replay<kCoupled><<<grid, 256, 0, st>>>(recs, coup, n, W, H, p->palette, grad_rgb, t,
                                                 partial);
        break;
      case kInert:
        k_replay<kInert><<<grid, 256, 0, st>>>(recs, nullptr, n, W, H, p->palette, grad_rgb, t,
                                               partial);
        break;
      case kDrops:
        k_replay<kDrops><<<grid, 256, 0, st>>>(recs, nullptr, n, W, H, p->palette, grad_rgb, t,
                                               partial);
        break;
      default:
        k_replay<kCapsule><<<grid, 256, 0, st>>>(recs, nullptr, n, W, H, p->palette, grad_rgb,
                                                 t, partial);
    }
  }
  tbr_status s = check_launch("replay");
  if (s) return s;
  return launch_reduce(p, o, g, ws, BL, st);
}

KWindow kwindow_of(const tbr_window_opts* o) {
  return KWindow{o->a_lo, o->a_hi - o->a_lo, o->l_max, o->r0_first,
                 (float)std::log((double)o->r0_last / (double)o->r0_first), o->r_lo_frac,
                 o->r_hi_frac - o->r_lo_frac, o->lambda_length, o->lambda_area};
}

tbr_status kwindow(const tbr_window_opts* o, KWindow* out) {
  if (!o) return fail(TBR_E_INVALID, "window opts are NULL");
  if (!(o->a_hi > o->a_lo) || !(o->l_max > 0.f) || !(o->r0_first > 0.f) || !(o->r0_last > 0.f) ||
      !(o->r_lo_frac > 0.f) || !(o->r_hi_frac > o->r_lo_frac) || !(o->lambda_length >= 0.f) ||
      !(o->lambda_area >= 0.f))
    return fail(TBR_E_INVALID, "window opts out of range");
  *out = kwindow_of(o);
  return TBR_OK;
}

KAdam kadam(const tbr_adam_opts* adam) {
  return KAdam{adam->lr_centre, adam->lr_angle, adam->lr_length, adam->lr_width, adam->lr_logits,
               adam->lr_palette, adam->beta1, adam->beta2, adam->eps,
               (float)(1.0 - std::pow((double)adam->beta1, adam->step)),
               (float)(1.0 - std::pow((double)adam->beta2, adam->step)),
               adam->r_lo, adam->r_hi, adam->l_max};
}

tbr_status check_adam(const tbr_adam_opts* adam) {
  if (!adam) return fail(TBR_E_INVALID, "adam opts are NULL");
  if (adam->step < 1) return fail(TBR_E_INVALID, "adam step must be >= 1");
  if (!(adam->beta1 >= 0.f && adam->beta1 < 1.f && adam->beta2 >= 0.f && adam->beta2 < 1.f &&
        adam->eps > 0.f && adam->r_lo > 0.f && adam->r_hi >= adam->r_lo && adam->l_max >= 0.f))
    return fail(TBR_E_INVALID, "bad Adam settings");
  return TBR_OK;
}

// Multi-job workspace: [cursor 256 B][job 0 fit layout][job 1 ...]
size_t multi_offset(const tbr_fit_job* jobs, int j) {
  size_t off = kAlign;
  for (int q = 0; q < j; ++q)
    off = align_up(off + fit_layout(&jobs[q].opts, jobs[q].n_strokes, jobs[q].n_palette).total);
  return off;
}

// The fit step up to its gradient: stroke prep, the fused forward + seed +
// replay launch, the loss and the fixed-order reduction to the natural
// parameters' gradient (*g_out; grads or the workspace copy). *records is the
// side-table high-water mark on the device.
tbr_status fit_core(int32_t n_strokes, int32_t n_palette, float* params, float* grads,
                    const tbr_render_opts* opts, const float* target_rgb, float* loss,
                    void* workspace, size_t workspace_bytes, hipStream_t st, float** g_out,
                    const int32_t** records, bool long_strokes = false) {
  tbr_status s;
  if (n_strokes < 0 || n_palette < 1 || n_palette > 64)
    return fail(TBR_E_INVALID, "n_strokes %d / n_palette %d out of range", n_strokes, n_palette);
  if (!params || !target_rgb || !loss || !workspace) return fail(TBR_E_INVALID, "null argument");
  if ((s = check_opts(opts, true, true))) return s;
  FitLayout FL = fit_layout(opts, n_strokes, n_palette);
  if (workspace_bytes < FL.total)
    return fail(TBR_E_INVALID, "workspace %zu bytes < required %zu", workspace_bytes, FL.total);
  char* ws = static_cast<char*>(workspace);
  char* rws = ws + FL.base_r;
  char* bws = ws + FL.base_b;
  const int N = n_strokes, K = n_palette;
  float* g = grads ? grads : reinterpret_cast<float*>(ws + FL.grads);
  tbr_program prog{N, K, params, params + N, params + 2 * N, params + 3 * N, params + 4 * N,
                   params + 5 * N, params + 5 * N + (size_t)N * K};
  tbr_program_grad pg{g, g + N, g + 2 * N, g + 3 * N, g + 4 * N, g + 5 * N,
                      g + 5 * N + (size_t)N * K};
  StrokeRec* recs = reinterpret_cast<StrokeRec*>(rws + FL.r.recs);
  KTape t = ktape(rws, FL.r, opts, true);
  float4* coup = coup_of(rws, FL.r, opts);
  if ((s = launch_prep(&prog, opts, recs, t.status, coup, st))) return s;
  float* lpart = reinterpret_cast<float*>(ws + FL.loss_part);
  if (opts->transport == TBR_TRANSPORT_INERT) {
    // R_U's per-stroke work is too light to hide memory latency at the
    // fused kernel's occupancy: the soft trace with tape and L2 seed, then
    // the replay, as two launches (same per-pixel code, same sums)
    float* grad_rgb = reinterpret_cast<float*>(ws + FL.seed);
    dim3 grid(tiles_x(opts), tiles_y(opts));
    k_trace_soft<kInert><<<grid, 256, 0, st>>>(recs, nullptr, N, opts->width, opts->height,
                                               prog.palette, nullptr, t,
                                               KSeed{target_rgb, grad_rgb, lpart});
    if ((s = check_launch("trace_soft"))) return s;
    k_replay<kInert><<<grid, 256, 0, st>>>(recs, nullptr, N, opts->width, opts->height,
                                           prog.palette, grad_rgb, t,
                                           reinterpret_cast<float*>(bws + FL.b.partial));
    if ((s = check_launch("replay"))) return s;
    k_loss_final<<<1, 256, 0, st>>>(lpart, (int)n_tiles(opts),
                                    1.0f / (3.0f * (float)n_pixels(opts)), loss);
    if ((s = check_launch("loss_final"))) return s;
    if ((s = launch_reduce(&prog, opts, &pg, bws, FL.b, st))) return s;
    *g_out = g;
    *records = t.status;
    return TBR_OK;
  }
  // soft forward with tape, L2 seed and replay adjoint of each tile in one
  // persistent launch (one drain of the GPU per step instead of two)
  FitJobsK KJ{};
  KJ.n_jobs = 1;
  FitJobK& D = KJ.job[0];
  D.recs = recs;
  D.coup = coup;
  D.palette = prog.palette;
  D.target = target_rgb;
  D.partial = reinterpret_cast<float*>(bws + FL.b.partial);
  D.loss_part = lpart;
  D.tape = t;
  D.n = N;
  D.width = opts->width;
  D.height = opts->height;
  D.tiles_x = tiles_x(opts);
  D.item0 = 0;
  KJ.n_items = (int)n_tiles(opts);
  if ((s = launch_fused(KJ, reinterpret_cast<int*>(ws + FL.cursor), opts->transport,
                        long_strokes, st)))
    return s;
  k_loss_final<<<1, 256, 0, st>>>(lpart, (int)n_tiles(opts), 1.0f / (3.0f * (float)n_pixels(opts)),
                                  loss);
  if ((s = check_launch("loss_final"))) return s;
  if ((s = launch_reduce(&prog, opts, &pg, bws, FL.b, st))) return s;
  *g_out = g;
  *records = t.status;
  return TBR_OK;
}

tbr_status check_render(const tbr_program* prog, const tbr_render_opts* opts, int32_t mode,
                        bool tape) {
  tbr_status s;
  if ((s = check_prog(prog))) return s;
  const bool soft = mode & TBR_SOFT, hard = mode & TBR_HARD;
  if (!(soft || hard) || (mode & ~(TBR_SOFT | TBR_HARD)))
    return fail(TBR_E_INVALID, "mode %d is not TBR_SOFT and/or TBR_HARD", mode);
  if (tape && !soft) return fail(TBR_E_INVALID, "a tape needs TBR_SOFT");
  return check_opts(opts, soft, tape);
}

// Stroke preparation and the trace kernels of one render, on the records,
// status word, profile cubics and tape that layout L places in ws.
tbr_status render_launch(const tbr_program* prog, const tbr_render_opts* opts, int32_t mode,
                         float* rgb, int32_t* label, int32_t* owner, char* ws,
                         const RenderLayout& L, bool tape, hipStream_t st) {
  tbr_status s;
  const bool soft = mode & TBR_SOFT, hard = mode & TBR_HARD;
  StrokeRec* recs = reinterpret_cast<StrokeRec*>(ws + L.recs);
  KTape t = ktape(ws, L, opts, tape);
  float4* coup = coup_of(ws, L, opts);
  if ((s = launch_prep(prog, opts, recs, t.status, coup, st))) return s;
  dim3 grid(tiles_x(opts), tiles_y(opts));
  const int n = prog->n_strokes, W = opts->width, H = opts->height;
  if (soft) {
    {
      Timed tm("trace_soft", st);
      const KSeed none{nullptr, nullptr, nullptr};
      switch (opts->transport) {
        case kCoupled:
          k_trace_soft<kCoupled><<<grid, 256, 0, st>>>(recs, coup, n, W, H, prog->palette, rgb, t,
                                                       none);
          break;
        case kInert:
          k_trace_soft<kInert><<<grid, 256, 0, st>>>(recs, nullptr, n, W, H, prog->palette, rgb,
                                                     t, none);
          break;
        case kDrops:
          k_trace_soft<kDrops><<<grid, 256, 0, st>>>(recs, nullptr, n, W, H, prog->palette, rgb,
                                                     t, none);
          break;
        default:
          k_trace_soft<kCapsule><<<grid, 256, 0, st>>>(recs, nullptr, n, W, H, prog->palette,
                                                       rgb, t, none);
      }
    }
    if ((s = check_launch("trace_soft"))) return s;
  }
  if (hard && (label || owner || (!soft && rgb))) {
    {
      Timed tm("trace_hard", st);
      float* hrgb = soft ? nullptr : rgb;
      switch (opts->transport) {
        case kCoupled:
          k_trace_hard<kCoupled><<<grid, 256, 0, st>>>(recs, coup, n, W, H, prog->palette, hrgb,
                                                       label, owner);
          break;
        case kInert:
          k_trace_hard<kInert><<<grid, 256, 0, st>>>(recs, nullptr, n, W, H, prog->palette, hrgb,
                                                     label, owner);
          break;
        case kDrops:
          k_trace_hard<kDrops><<<grid, 256, 0, st>>>(recs, nullptr, n, W, H, prog->palette, hrgb,
                                                     label, owner);
          break;
        default:
          k_trace_hard<kCapsule><<<grid, 256, 0, st>>>(recs, nullptr, n, W, H, prog->palette,
                                                       hrgb, label, owner);
      }
    }
    if ((s = check_launch("trace_hard"))) return s;
  }
  return TBR_OK;
}


// The allocation-free render (tbr_render_static) keeps its prepared stroke
// records, status word and profile cubics in this array instead of a
// workspace: one copy per device, held until the process ends. Host code
// uses only the per-device address from hipGetSymbolAddress.
constexpr size_t kScratchBytes = size_t(1) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_dev[kMaxDevices];

// The address of `scratch` on the current device, looked up once per device.
tbr_status scratch_here(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(TBR_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(TBR_E_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(TBR_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_dev[dev];
  return TBR_OK;
}

}  // namespace

extern "C" {

size_t tbr_render_workspace_bytes(const tbr_render_opts* opts, int32_t n_strokes, int32_t mode,
                                  int32_t with_tape) {
  if (!opts || n_strokes < 0) return 0;
  return render_layout(opts, n_strokes, with_tape && (mode & TBR_SOFT)).total;
}

tbr_status tbr_render(const tbr_program* prog, const tbr_render_opts* opts, int32_t mode,
                      float* rgb, int32_t* label, int32_t* owner, void* workspace,
                      size_t workspace_bytes, int32_t with_tape, void* stream) {
  tbr_status s;
  if ((s = check_render(prog, opts, mode, with_tape != 0))) return s;
  if (!workspace) return fail(TBR_E_INVALID, "workspace is NULL");
  RenderLayout L = render_layout(opts, prog->n_strokes, with_tape != 0);
  if (workspace_bytes < L.total)
    return fail(TBR_E_INVALID, "workspace %zu bytes < required %zu", workspace_bytes, L.total);
  return render_launch(prog, opts, mode, rgb, label, owner, static_cast<char*>(workspace), L,
                       with_tape != 0, reinterpret_cast<hipStream_t>(stream));
}

tbr_status tbr_render_static(const tbr_program* prog, const tbr_render_opts* opts, int32_t mode,
                             float* rgb, int32_t* label, int32_t* owner, void* stream) {
  tbr_status s;
  if ((s = check_render(prog, opts, mode, false))) return s;
  if (prog->n_strokes > TBR_STATIC_MAX_STROKES)
    return fail(TBR_E_CAPACITY, "n_strokes = %d exceeds the allocation-free render's %d",
                prog->n_strokes, TBR_STATIC_MAX_STROKES);
  RenderLayout L = render_layout(opts, prog->n_strokes, false);
  if (L.total > kScratchBytes)
    return fail(TBR_E_CAPACITY, "scratch %zu bytes < required %zu", kScratchBytes, L.total);
  char* ws = nullptr;
  if ((s = scratch_here(&ws))) return s;
  return render_launch(prog, opts, mode, rgb, label, owner, ws, L, false,
                       reinterpret_cast<hipStream_t>(stream));
}

tbr_status tbr_tape_records(const void* workspace, size_t workspace_bytes,
                            const tbr_render_opts* opts, int32_t n_strokes,
                            int32_t* max_records, void* stream) {
  if (!workspace || !opts || !max_records || n_strokes < 0)
    return fail(TBR_E_INVALID, "null argument");
  RenderLayout L = render_layout(opts, n_strokes, false);
  if (workspace_bytes < L.total) return fail(TBR_E_INVALID, "workspace too small");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int32_t v = 0;
  hipError_t e = hipMemcpyAsync(&v, static_cast<const char*>(workspace) + L.status, sizeof v,
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(TBR_E_DEVICE, "tape_records: %s", hipGetErrorString(e));
  *max_records = v;
  if (v > opts->side_slots)
    return fail(TBR_E_OVERFLOW, "side table needs %d slots per pixel, has %d", v, opts->side_slots);
  return TBR_OK;
}

size_t tbr_backward_workspace_bytes(const tbr_render_opts* opts, int32_t n_strokes,
                                    int32_t n_palette) {
  if (!opts || n_strokes < 0 || n_palette < 1) return 0;
  return back_layout(opts, n_strokes, n_palette).total;
}

tbr_status tbr_render_backward(const tbr_program* prog, const tbr_render_opts* opts,
                               const void* tape_ws, size_t tape_bytes, const float* grad_rgb,
                               const tbr_program_grad* grad, void* workspace,
                               size_t workspace_bytes, void* stream) {
  tbr_status s;
  if ((s = check_prog(prog))) return s;
  if ((s = check_opts(opts, true, true))) return s;
  if (!tape_ws || !grad_rgb || !grad || !workspace) return fail(TBR_E_INVALID, "null argument");
  if (!grad->palette || (prog->n_strokes > 0 && (!grad->cx || !grad->cy || !grad->angle ||
                                                 !grad->length || !grad->half_width || !grad->logits)))
    return fail(TBR_E_INVALID, "a gradient array is NULL");
  RenderLayout RL = render_layout(opts, prog->n_strokes, true);
  if (tape_bytes < RL.total) return fail(TBR_E_INVALID, "tape %zu bytes < %zu", tape_bytes, RL.total);
  BackLayout BL = back_layout(opts, prog->n_strokes, prog->n_palette);
  if (workspace_bytes < BL.total)
    return fail(TBR_E_INVALID, "workspace %zu bytes < required %zu", workspace_bytes, BL.total);
  return launch_backward(prog, opts, static_cast<const char*>(tape_ws), RL, grad_rgb, grad,
                         static_cast<char*>(workspace), BL, reinterpret_cast<hipStream_t>(stream));
}

size_t tbr_fit_workspace_bytes(const tbr_render_opts* opts, int32_t n_strokes, int32_t n_palette) {
  if (!opts || n_strokes < 0 || n_palette < 1) return 0;
  return fit_layout(opts, n_strokes, n_palette).total;
}

tbr_status tbr_fit_step(int32_t n_strokes, int32_t n_palette, float* params, float* grads,
                        float* adam_m, float* adam_v, const tbr_adam_opts* adam,
                        const tbr_render_opts* opts, const float* target_rgb, float* loss,
                        void* workspace, size_t workspace_bytes, void* stream) {
  tbr_status s;
  if (!params || !adam_m || !adam_v || !adam || !target_rgb || !loss || !workspace)
    return fail(TBR_E_INVALID, "null argument");
  if ((s = check_adam(adam))) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  float* g = nullptr;
  const int32_t* records = nullptr;
  if ((s = fit_core(n_strokes, n_palette, params, grads, opts, target_rgb, loss, workspace,
                    workspace_bytes, st, &g, &records)))
    return s;
  const int N = n_strokes, K = n_palette;
  int total = (int)packed_len(N, K);
  k_adam<<<(total + 255) / 256, 256, 0, st>>>(params, g, adam_m, adam_v, N, K, kadam(adam),
                                              records, opts->side_slots);
  return check_launch("adam");
}

tbr_status tbr_window_map(int32_t n_strokes, int32_t n_palette, const float* theta, float* params,
                          const tbr_window_opts* window, void* stream) {
  tbr_status s;
  if (n_strokes < 0 || n_palette < 1 || n_palette > 64)
    return fail(TBR_E_INVALID, "n_strokes %d / n_palette %d out of range", n_strokes, n_palette);
  if (!theta || !params) return fail(TBR_E_INVALID, "null argument");
  KWindow w;
  if ((s = kwindow(window, &w))) return s;
  const int total = (int)packed_len(n_strokes, n_palette);
  k_window_map<<<(total + 255) / 256, 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(
      theta, params, n_strokes, n_palette, w);
  return check_launch("window_map");
}

// A window whose offset bound per component exceeds this (canvas units)
// admits long strokes: the fused launch then takes kFusedWavesLong.
constexpr float kLongOffset = 0.1f;

tbr_status tbr_fit_loop_step(int32_t n_strokes, int32_t n_palette, float* theta, float* params,
                             float* grads, float* adam_m, float* adam_v,
                             const tbr_window_opts* window, const tbr_adam_opts* adam,
                             const tbr_render_opts* opts, const float* target_rgb, float* loss,
                             void* workspace, size_t workspace_bytes, void* stream) {
  tbr_status s;
  if (!theta || !params || !adam_m || !adam_v || !adam || !target_rgb || !loss || !workspace)
    return fail(TBR_E_INVALID, "null argument");
  if ((s = check_adam(adam))) return s;
  KWindow w;
  if ((s = kwindow(window, &w))) return s;
  // every argument is checked before the first launch, so a rejected call
  // leaves params untouched
  if (n_strokes < 0 || n_palette < 1 || n_palette > 64)
    return fail(TBR_E_INVALID, "n_strokes %d / n_palette %d out of range", n_strokes, n_palette);
  if ((s = check_opts(opts, true, true))) return s;
  if (workspace_bytes < fit_layout(opts, n_strokes, n_palette).total)
    return fail(TBR_E_INVALID, "workspace %zu bytes < required %zu", workspace_bytes,
                fit_layout(opts, n_strokes, n_palette).total);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int N = n_strokes, K = n_palette;
  const int total = (int)packed_len(N, K);
  if ((s = tbr_window_map(N, K, theta, params, window, stream))) return s;
  float* g = nullptr;
  const int32_t* records = nullptr;
  // offsets beyond a tenth of the canvas per component allow long strokes
  if ((s = fit_core(N, K, params, grads, opts, target_rgb, loss, workspace, workspace_bytes, st,
                    &g, &records, window->l_max > kLongOffset)))
    return s;
  k_reg_loss<<<1, 256, 0, st>>>(params, N, w, loss);
  if ((s = check_launch("reg_loss"))) return s;
  k_window_adam<<<(total + 255) / 256, 256, 0, st>>>(theta, g, adam_m, adam_v, N, K, w,
                                                     kadam(adam), records, opts->side_slots);
  return check_launch("window_adam");
}

size_t tbr_compensate_workspace_bytes(int32_t n_strokes, int32_t endpoint) {
  if (n_strokes < 0) return 0;
  return align_up((size_t)(n_strokes > 0 ? n_strokes : 1) * (endpoint ? 2 : 1) * sizeof(double2));
}

tbr_status tbr_compensate(const tbr_program* inert, float eps_floor, int32_t endpoint,
                          int32_t skip_blocked, float* cx, float* cy, float* angle, float* length,
                          int32_t* blocked, void* workspace, size_t workspace_bytes, void* stream) {
  tbr_status s;
  if ((s = check_prog(inert))) return s;
  if (!(eps_floor > 0.f) || !std::isfinite(eps_floor))
    return fail(TBR_E_INVALID, "eps_floor must be > 0");
  if (inert->n_strokes == 0) return TBR_OK;  // nothing to write (outputs may be NULL)
  if (!cx || !cy || !angle || !length || !blocked || !workspace)
    return fail(TBR_E_INVALID, "null argument");
  const size_t need = tbr_compensate_workspace_bytes(inert->n_strokes, endpoint);
  if (workspace_bytes < need)
    return fail(TBR_E_INVALID, "workspace %zu bytes < required %zu", workspace_bytes, need);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  {
    Timed tm("compensate", st);
    k_compensate<<<1, kCompThreadsK, 0, st>>>(kprog(inert), eps_floor, endpoint ? 1 : 0,
                                               skip_blocked ? 1 : 0,
                                               static_cast<double2*>(workspace), cx, cy, angle,
                                               length, blocked);
  }
  return check_launch("compensate");
}

tbr_status tbr_coupling_check(const float* coupling, int32_t n_strokes, float* min_g) {
  if (!coupling || n_strokes < 0) return fail(TBR_E_INVALID, "null argument");
  // g in W = cos(4 pi v) is the cubic a0 + a1 W + a2 W^2 + a3 W^3 on [-1, 1]:
  // its minimum is at an end or at a real root of g'(W) inside.
  double worst = INFINITY;
  int32_t bad = -1;
  for (int32_t i = 0; i < n_strokes; ++i) {
    const double c1 = coupling[3 * i], c2 = coupling[3 * i + 1], c3 = coupling[3 * i + 2];
    if (!std::isfinite(c1) || !std::isfinite(c2) || !std::isfinite(c3)) {
      worst = -INFINITY;
      bad = i;
      break;
    }
    const double a0 = 1.0 - c2, a1 = c1 - 3.0 * c3, a2 = 2.0 * c2, a3 = 4.0 * c3;
    auto g = [&](double W) { return a0 + W * (a1 + W * (a2 + W * a3)); };
    double m = std::min(g(-1.0), g(1.0));
    // g'(W) = a1 + 2 a2 W + 3 a3 W^2
    double roots[2];
    int nr = 0;
    if (a3 != 0.0) {
      const double A = 3.0 * a3, B = 2.0 * a2, D = B * B - 4.0 * A * a1;
      if (D >= 0.0) {
        const double q = -0.5 * (B + std::copysign(std::sqrt(D), B));
        if (q != 0.0) roots[nr++] = q / A;
        if (q != 0.0) roots[nr++] = a1 / q;
        else roots[nr++] = 0.0;  // B = D = 0: a double root at 0
      }
    } else if (a2 != 0.0) {
      roots[nr++] = -a1 / (2.0 * a2);
    }
    for (int k = 0; k < nr; ++k)
      if (roots[k] > -1.0 && roots[k] < 1.0) m = std::min(m, g(roots[k]));
    if (m < worst) {
      worst = m;
      bad = i;
    }
  }
  if (min_g) *min_g = n_strokes > 0 ? (float)worst : 1.0f;
  if (n_strokes > 0 && !(worst > 0.0))
    return fail(TBR_E_INVALID, "profile of stroke %d is not positive (min g = %g)", bad, worst);
  return TBR_OK;
}

void tbr_schedule_at(int32_t step, int32_t total_steps, float tau_first, float tau_last,
                     float tau_c_first, float tau_c_last, float* tau, float* tau_c,
                     float* lr_scale) {
  const double T = total_steps > 1 ? (double)total_steps : 1.0;
  const double f = total_steps > 1 ? (double)step / (T - 1.0) : 0.0;
  if (tau) *tau = (float)((double)tau_first * std::pow((double)tau_last / tau_first, f));
  if (tau_c)
    *tau_c = (float)((double)tau_c_first * std::pow((double)tau_c_last / tau_c_first, f));
  if (lr_scale) *lr_scale = (float)(0.5 * (1.0 + std::cos(3.14159265358979323846 * step / T)));
}

size_t tbr_fit_multi_workspace_bytes(const tbr_fit_job* jobs, int32_t n_jobs) {
  if (!jobs || n_jobs < 1 || n_jobs > kMaxFitJobs) return 0;
  for (int j = 0; j < n_jobs; ++j)
    if (jobs[j].n_strokes < 0 || jobs[j].n_palette < 1) return 0;
  return multi_offset(jobs, n_jobs);
}

tbr_status tbr_fit_multi_step(const tbr_fit_job* jobs, int32_t n_jobs, void* workspace,
                              size_t workspace_bytes, void* stream) {
  tbr_status s;
  if (!jobs || n_jobs < 1 || n_jobs > kMaxFitJobs)
    return fail(TBR_E_INVALID, "n_jobs = %d outside 1..%d", n_jobs, kMaxFitJobs);
  if (!workspace) return fail(TBR_E_INVALID, "workspace is NULL");
  for (int j = 0; j < n_jobs; ++j) {
    const tbr_fit_job& J = jobs[j];
    if (J.n_strokes < 0 || J.n_palette < 1 || J.n_palette > 64)
      return fail(TBR_E_INVALID, "job %d: n_strokes %d / n_palette %d out of range", j,
                  J.n_strokes, J.n_palette);
    if (!J.params || !J.adam_m || !J.adam_v || !J.target_rgb || !J.loss)
      return fail(TBR_E_INVALID, "job %d: null argument", j);
    if ((s = check_opts(&J.opts, true, true))) return s;
    if ((s = check_adam(&J.adam))) return s;
    if (J.opts.transport != jobs[0].opts.transport)
      return fail(TBR_E_INVALID, "job %d: every job of one step must use the same transport", j);
  }
  const size_t need = multi_offset(jobs, n_jobs);
  if (workspace_bytes < need)
    return fail(TBR_E_INVALID, "workspace %zu bytes < required %zu", workspace_bytes, need);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  // jobs in decreasing cost order, so the largest jobs' tiles are taken first
  int order[kMaxFitJobs];
  for (int j = 0; j < n_jobs; ++j) order[j] = j;
  std::sort(order, order + n_jobs, [&](int a, int b) {
    double ca = (double)n_pixels(&jobs[a].opts) * jobs[a].n_strokes;
    double cb = (double)n_pixels(&jobs[b].opts) * jobs[b].n_strokes;
    return ca > cb || (ca == cb && a < b);
  });
  FitJobsK K{};
  K.n_jobs = n_jobs;
  int items = 0;
  std::vector<tbr_program> progs(n_jobs);
  std::vector<tbr_program_grad> pgrads(n_jobs);
  std::vector<FitLayout> layouts(n_jobs);
  for (int q = 0; q < n_jobs; ++q) {
    const int j = order[q];
    const tbr_fit_job& J = jobs[j];
    const int N = J.n_strokes, Kp = J.n_palette;
    FitLayout FL = fit_layout(&J.opts, N, Kp);
    layouts[j] = FL;
    char* base = ws + multi_offset(jobs, j);
    char* rws = base + FL.base_r;
    float* g = J.grads ? J.grads : reinterpret_cast<float*>(base + FL.grads);
    float* pr = J.params;
    progs[j] = tbr_program{N, Kp, pr, pr + N, pr + 2 * N, pr + 3 * N, pr + 4 * N, pr + 5 * N,
                           pr + 5 * N + (size_t)N * Kp};
    pgrads[j] = tbr_program_grad{g, g + N, g + 2 * N, g + 3 * N, g + 4 * N, g + 5 * N,
                                 g + 5 * N + (size_t)N * Kp};
    StrokeRec* recs = reinterpret_cast<StrokeRec*>(rws + FL.r.recs);
    KTape t = ktape(rws, FL.r, &J.opts, true);
    float4* coup = coup_of(rws, FL.r, &J.opts);
    if ((s = launch_prep(&progs[j], &J.opts, recs, t.status, coup, st))) return s;
    FitJobK& D = K.job[q];
    D.recs = recs;
    D.coup = coup;
    D.palette = progs[j].palette;
    D.target = J.target_rgb;
    D.partial = reinterpret_cast<float*>(base + FL.base_b + FL.b.partial);
    D.loss_part = reinterpret_cast<float*>(base + FL.loss_part);
    D.tape = t;
    D.n = N;
    D.width = J.opts.width;
    D.height = J.opts.height;
    D.tiles_x = tiles_x(&J.opts);
    D.item0 = items;
    items += (int)n_tiles(&J.opts);
  }
  K.n_items = items;
  if ((s = launch_fused(K, reinterpret_cast<int*>(ws), jobs[0].opts.transport, false, st)))
    return s;
  for (int j = 0; j < n_jobs; ++j) {
    const tbr_fit_job& J = jobs[j];
    const FitLayout& FL = layouts[j];
    char* base = ws + multi_offset(jobs, j);
    k_loss_final<<<1, 256, 0, st>>>(reinterpret_cast<float*>(base + FL.loss_part),
                                    (int)n_tiles(&J.opts),
                                    1.0f / (3.0f * (float)n_pixels(&J.opts)), J.loss);
    if ((s = check_launch("loss_final"))) return s;
    if ((s = launch_reduce(&progs[j], &J.opts, &pgrads[j], base + FL.base_b, FL.b, st))) return s;
    int total = (int)packed_len(J.n_strokes, J.n_palette);
    const int32_t* recmax = reinterpret_cast<const int32_t*>(base + FL.base_r + FL.r.status);
    k_adam<<<(total + 255) / 256, 256, 0, st>>>(J.params, pgrads[j].cx, J.adam_m, J.adam_v,
                                                J.n_strokes, J.n_palette, kadam(&J.adam), recmax,
                                                J.opts.side_slots);
    if ((s = check_launch("adam"))) return s;
  }
  return TBR_OK;
}

tbr_status tbr_fit_multi_records(const tbr_fit_job* jobs, int32_t n_jobs, const void* workspace,
                                 size_t workspace_bytes, int32_t* max_records, void* stream) {
  if (!jobs || n_jobs < 1 || n_jobs > kMaxFitJobs || !workspace || !max_records)
    return fail(TBR_E_INVALID, "null argument or bad n_jobs");
  if (workspace_bytes < multi_offset(jobs, n_jobs)) return fail(TBR_E_INVALID, "workspace too small");
  tbr_status worst = TBR_OK;
  for (int j = 0; j < n_jobs; ++j) {
    FitLayout FL = fit_layout(&jobs[j].opts, jobs[j].n_strokes, jobs[j].n_palette);
    const char* base = static_cast<const char*>(workspace) + multi_offset(jobs, j) + FL.base_r;
    tbr_status s = tbr_tape_records(base, FL.r.total, &jobs[j].opts, jobs[j].n_strokes,
                                    &max_records[j], stream);
    if (s == TBR_E_OVERFLOW) worst = s;
    else if (s != TBR_OK) return s;
  }
  if (worst == TBR_E_OVERFLOW) return fail(TBR_E_OVERFLOW, "a job's side table overflowed");
  return TBR_OK;
}

tbr_status tbr_set_timing_events(const char* kernel, void* begin, void* end) {
  if (!kernel) {
    g_timed_kernel.clear();
    g_ev_begin = g_ev_end = nullptr;
    return TBR_OK;
  }
  if (!begin || !end) return fail(TBR_E_INVALID, "timing events are NULL");
  g_timed_kernel = kernel;
  g_ev_begin = reinterpret_cast<hipEvent_t>(begin);
  g_ev_end = reinterpret_cast<hipEvent_t>(end);
  return TBR_OK;
}

const char* tbr_last_error(void) { return g_err.c_str(); }

const char* tbr_version(void) { return "tbr 0.1.0 (gfx950)"; }

}  // extern "C"
