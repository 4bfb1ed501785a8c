// tbr_kernels.hip -- HIP kernels for gfx950 (CDNA4), wave64, FP32 VALU.
//
// Pixel layout: a block of 256 threads is 4 waves; each wave owns an 8x8
// pixel tile (lane l -> (l & 7, l >> 3)), the block a 16x16 tile. Pixel
// centres are ((j + .5) / W, (i + .5) / H), row-major. Stroke records are
// read with wave-uniform addresses: scalar loads into SGPRs in the trace
// kernels, vector loads where a loop holds a barrier (the replay, the fused
// and serving kernels). No stroke data is staged through LDS: it measured
// no faster (see load_rec).
//
// Paper references (TBR, arxiv 2609.08722): Eq. chain and Eq. render
// (Sec. 3), the operator (Sec. 4), Eq. relax (Sec. 5.1), Eq. state, the
// regeneration Eqs. rpos / rT, the floor and record rule, log-space
// transmittance with the alpha clamp, periodic checkpoints, Eq. adjstep and
// Eq. adjparam (Sec. 5.2).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "tbr_device.hpp"
#include "tbr_kernels.hpp"

namespace tbr {

// ---------------------------------------------------------------------------
// Stroke preparation: the per-stroke constants of one record.
// ---------------------------------------------------------------------------
__device__ __forceinline__ StrokeRec prep_stroke(const KProgram& p, const KOpts& o, int i) {
  StrokeRec g;
  g.mx = (double)p.cx[i];
  g.my = (double)p.cy[i];
  float phi = p.angle[i];
  g.ce = cosf(phi);
  g.se = sinf(phi);
  float ell = fabsf(p.length[i]);
  g.ell = ell;
  g.hl = 0.5f * ell;
  g.two_ell = ell + ell;
  float r = p.half_width[i];
  g.r = r;
  g.ar = r * fmaf(kPi, r, ell + ell);
  g.per_r = fmaf(kTwoPi, r, ell + ell);
  float tr = o.tau * r;
  bool rel = tr > o.tau_min;
  float wd = rel ? tr : o.tau_min;
  g.inv_wd = 1.0f / wd;
  g.dwd_dr = rel ? o.tau : 0.f;
  float er = o.eps * r;
  g.floor_c = er * er;
  // beyond far_sig a wave skips coverage, and psi's floor cannot bind there
  // on any leaf: C = (sigma - rl)(pi (sigma + rl) + 2 l) >= pi (sigma - rl)^2
  // exceeds (eps r)^2 once sigma - rl > eps r / sqrt(pi) (with a margin for
  // the kernels' FP32 C); at the usual eps that is far inside 28 wd
  g.far_sig = r + fmaxf(-kFarZ * wd, er * (1.001f / sqrtf(kPi)));
  // colour: softmax(z / tau_c) P, or P[argmax z] when tau_c == 0
  const float* z = p.logits + (size_t)i * p.k;
  int best = 0;
  float zmax = z[0];
  for (int j = 1; j < p.k; ++j)
    if (z[j] > zmax) {
      zmax = z[j];
      best = j;
    }
  g.label = best;
  float cr = 0.f, cg = 0.f, cb = 0.f;
  if (o.tau_c > 0.f) {
    float inv_tc = 1.0f / o.tau_c, tot = 0.f;
    for (int j = 0; j < p.k; ++j) tot += expf((z[j] - zmax) * inv_tc);
    float inv_tot = 1.0f / tot;
    for (int j = 0; j < p.k; ++j) {
      float s = expf((z[j] - zmax) * inv_tc) * inv_tot;
      cr = fmaf(s, p.palette[3 * j + 0], cr);
      cg = fmaf(s, p.palette[3 * j + 1], cg);
      cb = fmaf(s, p.palette[3 * j + 2], cb);
    }
  } else {
    cr = p.palette[3 * best + 0];
    cg = p.palette[3 * best + 1];
    cb = p.palette[3 * best + 2];
  }
  g.cr = cr;
  g.cg = cg;
  g.cb = cb;
  return g;
}

// One thread per stroke of one program.
__global__ void __launch_bounds__(256)
    k_stroke_prep(KProgram p, KOpts o, StrokeRec* __restrict__ out, int32_t* __restrict__ status,
                  float4* __restrict__ coup) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && status) *status = 0;  // tape record high-water mark of this launch
  if (i >= p.n) return;
  out[i] = prep_stroke(p, o, i);
  if (coup) {  // Eq. profile as a cubic in cos(4 pi w) (see coupled_leaf)
    const float c1 = o.coupling[3 * i], c2 = o.coupling[3 * i + 1], c3 = o.coupling[3 * i + 2];
    coup[i] = make_float4(1.f - c2, fmaf(-3.f, c3, c1), 2.f * c2, 4.f * c3);
  }
}

// Every request of a serving tick in one launch: request j owns the blocks
// [preps[j].block0, preps[j].block0 + ceil(n_j / 256)), one thread per
// stroke (requests of empty programs own no block).
__global__ void __launch_bounds__(256) k_serve_prep(const ServePrep* __restrict__ preps, int n_req) {
  const int b = blockIdx.x;
  int j = 0;
  while (j + 1 < n_req && b >= preps[j + 1].block0) ++j;
  j = __builtin_amdgcn_readfirstlane(j);
  const ServePrep q = preps[j];
  const int i = (b - q.block0) * 256 + (int)threadIdx.x;
  if (b >= q.block0 && i < q.prog.n) q.out[i] = prep_stroke(q.prog, q.opts, i);
}

// Wave-uniform load of a stroke record. The compiler issues scalar loads
// where it can prove that no store of the launch changes the record (the
// trace kernels' barrier-free loops) and vector loads otherwise. Forcing
// either kind measured slower: scalar loads in the replay and fused kernels
// (at their occupancy the scalar cache's latency shows), the records staged
// through LDS per chunk, and vector loads in the trace kernels (more VGPRs,
// fewer waves).
__device__ __forceinline__ StrokeRec load_rec(const StrokeRec* __restrict__ recs, int i) {
  i = __builtin_amdgcn_readfirstlane(i);
  return recs[i];
}

// Wave-uniform load of a stroke's profile coefficients (coupled variant).
__device__ __forceinline__ float4 load_coup(const float4* __restrict__ coup, int i) {
  i = __builtin_amdgcn_readfirstlane(i);
  return coup[i];
}

template <bool kC>
__device__ __forceinline__ Leaf leaf_at(const Chart& c, const StrokeRec& g,
                                        const float4* __restrict__ coup, int i) {
  if constexpr (kC) {
    return coupled_leaf(c.w, g, load_coup(coup, i));
  } else {
    return uniform_leaf(g);
  }
}

struct PixelId {
  int px, py;
  bool active;
  int p;  // flat index (clamped inside the canvas for inactive lanes)
};

__device__ __forceinline__ PixelId pixel_of_tile(int tx, int ty, int width, int height) {
  PixelId id;
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  id.px = tx * 16 + (wave & 1) * 8 + (lane & 7);
  id.py = ty * 16 + (wave >> 1) * 8 + (lane >> 3);
  id.active = id.px < width && id.py < height;
  int cx = min(id.px, width - 1), cy = min(id.py, height - 1);
  id.p = cy * width + cx;
  return id;
}

// ---------------------------------------------------------------------------
// Soft forward trace (Eq. chain + Eq. render with Eq. relax) of one pixel
// per lane, optionally writing the replay tape. Shared by the render, the
// fit step and the serving kernel, so a pixel's result does not depend on
// which launch computed it.
// ---------------------------------------------------------------------------
struct SoftOut {
  float cr, cg, cb;  // composite R = C_0 + T_0 c_0
  int nrec;          // records pushed (floor bound)
};

template <bool kTape, int kT = kCapsule>
__device__ __forceinline__ SoftOut soft_pixel(const StrokeRec* __restrict__ recs,
                                              const float4* __restrict__ coup, int n,
                                              const PixelId& id, int width, int height,
                                              const float* __restrict__ palette,
                                              const KTape& tape) {
  const int P = width * height;
  double x = (id.px + 0.5) / (double)width;
  double y = (id.py + 0.5) / (double)height;
  float cr = 0.f, cg = 0.f, cb = 0.f;
  float tm = 1.0f;
  int te = 0;
  int nrec = 0;
  const bool write_tape = kTape && id.active;
  const int k = kTape ? tape.ckpt_interval : 0;
  // states x_k, x_2k, ... (< x_n) are checkpointed; x_{i+1} is the input of
  // stroke i, so the first one met going down is at i = floor((n-1)/k) k - 1
  int next_ck = k > 0 ? ((n - 1) / k) * k - 1 : -1;
  // A far point is never floored (far_sig), so the far steps run psi
  // without the floor and record no side-table entry.
  // psi (or R_D's drops) and the advance of one step, with the floor and its
  // record when kFloor
  auto transport = [&](int i, const Chart& c, const StrokeRec& g, const Leaf& lf, auto floor_tag) {
    constexpr bool kFloor = decltype(floor_tag)::value;
    if constexpr (kT == kDrops) {
      // R_D: the tape records x_i wherever a drop's floor binds (far steps
      // included: a drop may reach past the capsule's far margin)
      const double x0 = x, y0 = y;
      if (drops_backward(x, y, g)) {
        if (write_tape && nrec < tape.side_slots) {
          size_t o = (size_t)nrec * P + id.p;
          tape.side_idx[o] = i;
          tape.side_xy[o] = make_double2(x0, y0);
        }
        ++nrec;
      }
    } else if constexpr (kT != kInert) {
      if constexpr (kFloor) {
        Move mv = displace<false, true>(c, g, true, lf);
        if (mv.floored) {  // record where the floor binds
          if (write_tape && nrec < tape.side_slots) {
            size_t o = (size_t)nrec * P + id.p;
            tape.side_idx[o] = i;
            tape.side_xy[o] = make_double2(x, y);
          }
          ++nrec;
        }
        advance(x, y, c, mv, g);
      } else {
        psi_far_advance<kT == kCoupled>(x, y, c, kT == kCoupled ? c.th : far_theta(c), g, lf);
      }
    }
  };
  int i = n - 1;
  while (i >= 0) {
    // Strokes far from every pixel of the wave, up to the next one that is
    // not: alpha < 7e-13, so 1 - alpha rounds to 1 and T and C are
    // unchanged to FP32 rounding. Lanes past a ragged canvas edge trace a
    // point just outside the canvas and vote too: that can only keep the
    // exact path. The near stroke leaves the loop with its chart.
    StrokeRec g;
    Chart c;
    Leaf lf;
    bool near = false;
    for (; i >= 0; --i) {
      g = load_rec(recs, i);
      if (__builtin_expect(kTape && i == next_ck, 0)) {
        if (write_tape) {
          size_t o = (size_t)((i + 1) / k) * P + id.p;
          tape.ckpt_xy[o] = make_double2(x, y);
          tape.ckpt_t[o] = make_float2(tm, (float)te);
        }
        next_ck -= k;
      }
      if constexpr (kT == kCoupled) {  // the far vote needs the leaf's edge
        c = chart(x, y, g);
        lf = leaf_at<true>(c, g, coup, i);
        if (!wave_all(is_far<true>(c.sig, lf, g))) {
          near = true;
          break;
        }
      } else {
        lf = uniform_leaf(g);
        chart_dist(x, y, g, c);
        if (__builtin_expect(!wave_all(is_far<false>(c.sig, lf, g)), 0)) {
          chart_angle(g, c);
          near = true;
          break;
        }
      }
      transport(i, c, g, lf, std::integral_constant<bool, false>{});
    }
    if (!near) break;
    // a near stroke: coverage and compositing, then psi with the floor
    Cover v = cover(c.sig, g, lf.r);
    float t = trans_value(tm, te);
    float ta = t * v.alpha;
    cr = fmaf(ta, g.cr, cr);
    cg = fmaf(ta, g.cg, cg);
    cb = fmaf(ta, g.cb, cb);
    tm *= v.q;
    renorm(tm, te);
    transport(i, c, g, lf, std::integral_constant<bool, true>{});
    --i;
  }
  float t = trans_value(tm, te);
  SoftOut o;
  o.cr = fmaf(t, palette[0], cr);  // background c_0 = P[0]
  o.cg = fmaf(t, palette[1], cg);
  o.cb = fmaf(t, palette[2], cb);
  o.nrec = nrec;
  if (write_tape) {  // state x_0
    tape.ckpt_xy[id.p] = make_double2(x, y);
    tape.ckpt_t[id.p] = make_float2(tm, (float)te);
    tape.nrec[id.p] = nrec;
  }
  return o;
}

// Hard trace of one pixel per lane: first footprint hit going N -> 1; lanes
// retire on a hit and the wave leaves the stroke loop once all have retired.
template <int kT = kCapsule>
__device__ __forceinline__ void hard_pixel(const StrokeRec* __restrict__ recs,
                                           const float4* __restrict__ coup, int n,
                                           const PixelId& id, int width, int height, int& own,
                                           int& lab) {
  double x = (id.px + 0.5) / (double)width;
  double y = (id.py + 0.5) / (double)height;
  bool done = !id.active;
  own = -1;
  lab = 0;
  for (int i = n - 1; i >= 0; --i) {
    if (__builtin_expect(wave_all(done), 0)) break;
    const StrokeRec g = load_rec(recs, i);
    if (!done) {
      Chart c;
      Leaf lf;
      if constexpr (kT == kCoupled) {
        c = chart(x, y, g);
        lf = leaf_at<true>(c, g, coup, i);
      } else {
        lf = uniform_leaf(g);
        chart_dist(x, y, g, c);
      }
      if constexpr (kT == kCapsule || kT == kCoupled) {
        // Every lane still tracing lies beyond the stroke's far margin: none
        // can hit it, and psi's floor cannot bind there.
        if (__builtin_expect(wave_all(is_far<kT == kCoupled>(c.sig, lf, g)), 1)) {
          psi_far_advance<kT == kCoupled>(x, y, c, kT == kCoupled ? c.th : far_theta(c), g, lf);
          continue;
        }
      }
      if constexpr (kT != kCoupled) chart_angle(g, c);
      if (c.sig <= lf.r) {  // closed footprint
        done = true;
        own = i;
        lab = g.label;
      } else if constexpr (kT == kDrops) {
        drops_backward(x, y, g);
      } else if constexpr (kT != kInert) {
        advance(x, y, c, displace(c, g, true, lf), g);
      }
    }
  }
}

template <int kT>
__global__ void __launch_bounds__(256)
    k_trace_soft(const StrokeRec* __restrict__ recs, const float4* __restrict__ coup, int n,
                 int width, int height, const float* __restrict__ palette, float* __restrict__ rgb,
                 KTape tape, KSeed seed) {
  PixelId id = pixel_of_tile(blockIdx.x, blockIdx.y, width, height);
  const int P = width * height;
  SoftOut o = tape.ckpt_xy
                  ? soft_pixel<true, kT>(recs, coup, n, id, width, height, palette, tape)
                  : soft_pixel<false, kT>(recs, coup, n, id, width, height, palette, tape);
  if (id.active && rgb) {
    rgb[3 * (size_t)id.p + 0] = o.cr;
    rgb[3 * (size_t)id.p + 1] = o.cg;
    rgb[3 * (size_t)id.p + 2] = o.cb;
  }
  // L2 seed (fit step): lambda^C_0 = dL/dR = 2 (R - I*) / (3P), loss partials
  if (seed.target) {
    float sq = 0.f;
    if (id.active) {
      float dr = o.cr - seed.target[3 * (size_t)id.p + 0];
      float dg = o.cg - seed.target[3 * (size_t)id.p + 1];
      float db = o.cb - seed.target[3 * (size_t)id.p + 2];
      float sc = 2.0f / (3.0f * (float)P);
      seed.grad_rgb[3 * (size_t)id.p + 0] = sc * dr;
      seed.grad_rgb[3 * (size_t)id.p + 1] = sc * dg;
      seed.grad_rgb[3 * (size_t)id.p + 2] = sc * db;
      sq = fmaf(dr, dr, fmaf(dg, dg, db * db));
    }
    // fixed-order block sum of squared errors
    __shared__ float red[256];
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) seed.loss_part[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
  }
  if (tape.status) {
    // max record count over the wave, one atomic per wave
    int m = id.active ? o.nrec : 0;
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(tape.status, m);
  }
}

template <int kT>
__global__ void __launch_bounds__(256)
    k_trace_hard(const StrokeRec* __restrict__ recs, const float4* __restrict__ coup, int n,
                 int width, int height, const float* __restrict__ palette,
                 float* __restrict__ rgb, int32_t* __restrict__ label,
                 int32_t* __restrict__ owner) {
  PixelId id = pixel_of_tile(blockIdx.x, blockIdx.y, width, height);
  int own, lab;
  hard_pixel<kT>(recs, coup, n, id, width, height, own, lab);
  if (id.active) {
    if (owner) owner[id.p] = own;
    if (label) label[id.p] = lab;
    if (rgb) {
      rgb[3 * (size_t)id.p + 0] = palette[3 * lab + 0];
      rgb[3 * (size_t)id.p + 1] = palette[3 * lab + 1];
      rgb[3 * (size_t)id.p + 2] = palette[3 * lab + 2];
    }
  }
}

// ---------------------------------------------------------------------------
// Serving: one persistent launch per scheduler tick. Blocks pull
// (request, tile) work items through an atomic cursor until the list is
// exhausted (every block exits when the cursor passes n_items), so tiles of
// requests with different programs, resolutions and modes share the device.
// Each tile runs the same per-pixel functions as the single-request kernels.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
    k_serve(const ServeDesc* __restrict__ descs, const uint2* __restrict__ items, int n_items,
            int* __restrict__ cursor) {
  __shared__ int item_s;
  for (;;) {
    if (threadIdx.x == 0) item_s = atomicAdd(cursor, 1);
    __syncthreads();
    const int it = item_s;
    __syncthreads();
    if (it >= n_items) break;
    const uint2 w = items[it];
    const ServeDesc d = descs[__builtin_amdgcn_readfirstlane(w.x)];
    const int tile = __builtin_amdgcn_readfirstlane(w.y);
    PixelId id = pixel_of_tile(tile % d.tiles_x, tile / d.tiles_x, d.width, d.height);
    if (d.soft) {
      KTape none{};
      SoftOut o = soft_pixel<false>(d.recs, nullptr, d.n, id, d.width, d.height, d.palette, none);
      if (id.active) {
        d.rgb[3 * (size_t)id.p + 0] = o.cr;
        d.rgb[3 * (size_t)id.p + 1] = o.cg;
        d.rgb[3 * (size_t)id.p + 2] = o.cb;
      }
    } else {
      int own, lab;
      hard_pixel(d.recs, nullptr, d.n, id, d.width, d.height, own, lab);
      if (id.active) {
        if (d.owner) d.owner[id.p] = own;
        if (d.label) d.label[id.p] = lab;
        if (d.rgb) {
          d.rgb[3 * (size_t)id.p + 0] = d.palette[3 * lab + 0];
          d.rgb[3 * (size_t)id.p + 1] = d.palette[3 * lab + 1];
          d.rgb[3 * (size_t)id.p + 2] = d.palette[3 * lab + 2];
        }
      }
    }
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Cross-lane reduction of 8 per-lane values to 16-lane row sums.
// Three transpose stages halve the value set while exchanging with lane^1,
// lane^2, lane^4; a last exchange with lane^8 adds the row's two halves.
// Afterwards lanes l and l + 8 of each 16-lane row hold the row's sum of
// value index bitrev3(l & 7). The four rows of a wave are added later, in a
// fixed order, together with the block's other waves.
//
// Two ways to exchange, with the same pairwise sums (bitwise the same
// results): DPP (quad permutes, row shifts by 4, a row rotation by 8), or
// ds_swizzle xor patterns, which run on the LDS crossbar so that the adds
// after them are plain vector adds (a DPP add issues at about half the rate
// of a plain one on gfx950) but wait on the crossbar's latency. Measured
// per map at 1024^2 x 2000: the capsule map's fit step (6 waves per SIMD)
// is 1.4% faster with the swizzles, the coupled map's (5 waves) 12% slower,
// so kSwz is set for the capsule map only.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
constexpr int kQuadXor1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int kRowShl4 = 0x104;
constexpr int kRowShr4 = 0x114;
constexpr int kRowRor8 = 0x128;

template <int kXor>
__device__ __forceinline__ float swz_xor(float v) {
  // bit mode: and_mask 0x1F, or_mask 0, xor_mask kXor (within 32 lanes)
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), (kXor << 10) | 0x1F));
}

// The value of lane^1, lane^2, lane^8; and of lane^4 as seen from the lanes
// with bit 2 clear (lo) or set (hi), the only lanes whose result is kept.
template <bool kSwz> __device__ __forceinline__ float xch1(float v) {
  if constexpr (kSwz) return swz_xor<1>(v); else return dpp_mov<kQuadXor1>(v);
}
template <bool kSwz> __device__ __forceinline__ float xch2(float v) {
  if constexpr (kSwz) return swz_xor<2>(v); else return dpp_mov<kQuadXor2>(v);
}
template <bool kSwz> __device__ __forceinline__ float xch4lo(float v) {
  if constexpr (kSwz) return swz_xor<4>(v); else return dpp_mov<kRowShl4>(v);
}
template <bool kSwz> __device__ __forceinline__ float xch4hi(float v) {
  if constexpr (kSwz) return swz_xor<4>(v); else return dpp_mov<kRowShr4>(v);
}
template <bool kSwz> __device__ __forceinline__ float xch8(float v) {
  if constexpr (kSwz) return swz_xor<8>(v); else return dpp_mov<kRowRor8>(v);
}

// One far step by the general map: Phi (Eq. rpos) of the charted point
// x_{i-1} with regenerate, which also takes lanes on the stroke's flank, and
// psi's VJP without the coverage terms (alpha, mu dalpha and the colour
// terms vanish to FP32 beyond the far margin). The coupled map's common
// step; under uniform insertion, the step of a far wave with a lane on the
// flank, which the polar cap-to-cap step does not cover.
template <bool kC>
__device__ __forceinline__ void far_general_step(double& x, double& y, float& lx, float& ly,
                                                 const Chart& ca, const StrokeRec& g,
                                                 const Leaf& lf, float (&v)[5]) {
  Move mv = regenerate(ca, g, lf);
  // unfolded displacement; psi runs from the regenerated x_i back to
  // the chart point x_{i-1}, so its increments are Phi's negated
  const float da = ca.sgs * mv.dS, db = ca.sgh * mv.dH;
  VjpIn vi;
  vi.sgs = ca.sgs;
  vi.sgh = ca.sgh;
  vi.w = ca.w;
  vi.floored = false;
  vi.sig = mv.sig_o;
  vi.th = mv.th_o;
  vi.sn = mv.sn_o;
  vi.cs = mv.cs_o;
  vi.tf = mv.tf_o;
  vi.inv_p1 = mv.inv_per_o;
  vi.rho = ca.sig;
  vi.inv_p0 = ca.inv_per;
  vi.th_o = ca.th;
  vi.sn_o = ca.sn;
  vi.cs_o = ca.cs;
  vi.tf_o = mv.tf;
  vi.dsig = -mv.dsig;
  vi.dth = -mv.dth;
  vi.dsin = -mv.dsin;
  vi.dcos = -mv.dcos;
  vi.dtf = -mv.dtf;
  vi.z = 0.f;
  vi.alpha = 0.f;
  vi.q = 1.f;
  vi.clamped = true;
  step_by(x, y, da, db, g);
  const VjpOut vo = vjp_step<false, kC>(vi, g, lx, ly, 0.f, lf);
  lx = vo.gx;
  ly = vo.gy;
  v[0] = vo.nmx;
  v[1] = vo.nmy;
  v[2] = vo.gphi;
  v[3] = vo.gell;
  v[4] = vo.gr;
}

template <bool kSwz>
__device__ __forceinline__ float row_sums8(const float (&v)[8], int lane) {
  const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
  float u[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float r0 = v[j] + xch1<kSwz>(v[j]);
    float r1 = v[j + 4] + xch1<kSwz>(v[j + 4]);
    u[j] = b0 ? r1 : r0;
  }
  float w[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    float r0 = u[j] + xch2<kSwz>(u[j]);
    float r1 = u[j + 2] + xch2<kSwz>(u[j + 2]);
    w[j] = b1 ? r1 : r0;
  }
  float r0 = w[0] + xch4lo<kSwz>(w[0]);
  float r1 = w[1] + xch4hi<kSwz>(w[1]);
  float t = b2 ? r1 : r0;
  return t + xch8<kSwz>(t);
}

// Same result when values 5..7 are zero (strokes far from the wave). The
// lanes that end with value index 4..7 (lane bit 0 set) only ever combine
// with each other, so the stage-1 sums of values 1..3 may stand in for the
// missing 5..7 there; one select zeroes the lanes of values 5..7 at the end.
template <bool kSwz>
__device__ __forceinline__ float row_sums5(const float (&v)[5], int lane) {
  const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
  float u[4];
  {
    float r0 = v[0] + xch1<kSwz>(v[0]);
    float r1 = v[4] + xch1<kSwz>(v[4]);
    u[0] = b0 ? r1 : r0;
  }
#pragma unroll
  for (int j = 1; j < 4; ++j) u[j] = v[j] + xch1<kSwz>(v[j]);
  float w[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    float r0 = u[j] + xch2<kSwz>(u[j]);
    float r1 = u[j + 2] + xch2<kSwz>(u[j + 2]);
    w[j] = b1 ? r1 : r0;
  }
  float r0 = w[0] + xch4lo<kSwz>(w[0]);
  float r1 = w[1] + xch4hi<kSwz>(w[1]);
  float t = b2 ? r1 : r0;
  t += xch8<kSwz>(t);
  return (b0 && (b1 || b2)) ? 0.f : t;
}

__device__ __forceinline__ int value_index_of_lane(int lane) {
  return ((lane & 1) << 2) | (lane & 2) | ((lane >> 2) & 1);
}

// ---------------------------------------------------------------------------
// Replay adjoint (Sec. 5.2): i = 1..N regenerates x_i = Phi_i(x_{i-1})
// (Eq. rpos) and T_i (Eq. rT, multiplicative form), except where the side
// table holds x_i (the floor bound there in the forward pass) or a
// checkpoint resets the drift; then applies Eq. adjstep and accumulates
// Eq. adjparam. Per stroke, 8 contributions (m_x, m_y, phi, l, r, c_rgb)
// are reduced across each 16-lane row, and the block's 16 row sums are
// then added in a fixed order into the tile's partial row.
// ---------------------------------------------------------------------------
constexpr int kChunk = 16;
// Block reduction buffer: [double buffer][wave * 4 + row][stroke of the
// chunk, padded so the 4 rows of a wave write distinct banks][value].
using ReduceLds = float[2][16][kChunk + 1][8];

// The smallest stroke index at which some lane of the wave pops a side-table
// record (top_idx < 0: the lane has none left), or INT_MAX: wave-uniform, so
// the replay's common steps test it with a scalar compare.
__device__ __forceinline__ int wave_next_pop(int top_idx) {
  int m = top_idx >= 0 ? top_idx : 0x7fffffff;
  for (int off = 32; off > 0; off >>= 1) m = min(m, __shfl_xor(m, off));
  return __builtin_amdgcn_readfirstlane(m);
}

// The replay of one 16x16 tile by the whole block (all 256 threads must
// call it). lcr, lcg, lcb: this lane's dL/dR; prow: the tile's partial row
// [n + 1][8] (row n = background colour gradient).
template <int kT = kCapsule>
__device__ __forceinline__ void replay_tile(const StrokeRec* __restrict__ recs,
                                            const float4* __restrict__ coup, int n,
                                            const PixelId& id, int width, int height,
                                            const float* __restrict__ palette, float lcr,
                                            float lcg, float lcb, const KTape& tape,
                                            float* __restrict__ prow, ReduceLds& lds) {
  const float bgr = palette[0], bgg = palette[1], bgb = palette[2];
  const int P = width * height;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k = tape.ckpt_interval;
  // start from the final state s_0: lambda^C = dL/dR (constant along the
  // chain), lambda^T_0 = lambda^C . c_0, lambda^x_0 = 0
  double x = 0.5, y = 0.5;
  float tm = 1.f;
  int te = 0, top = 0, top_idx = -1;
  if (id.active) {
    double2 s0 = tape.ckpt_xy[id.p];
    float2 t0 = tape.ckpt_t[id.p];
    x = s0.x;
    y = s0.y;
    tm = t0.x;
    te = (int)t0.y;
    top = min(tape.nrec[id.p], tape.side_slots);
    top_idx = top > 0 ? tape.side_idx[(size_t)(top - 1) * P + id.p] : -1;
  } else {
    lcr = lcg = lcb = 0.f;
  }
  float lt = fmaf(lcr, bgr, fmaf(lcg, bgg, lcb * bgb));
  float lx = 0.f, ly = 0.f;
  // background colour gradient: dL/dc_0 = lambda^C T_0
  {
    float t0 = trans_value(tm, te);
    float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, lcr * t0, lcg * t0, lcb * t0};
    float tot = row_sums8<kT == kCapsule>(v, lane);
    __syncthreads();  // lds may still be read by a previous tile of this block
    if (!(lane & 8)) lds[0][wave * 4 + (lane >> 4)][0][value_index_of_lane(lane)] = tot;
    __syncthreads();
    if (threadIdx.x < 8) {
      float s = 0.f;
#pragma unroll
      for (int q = 0; q < 16; ++q) s += lds[0][q][0][threadIdx.x];
      prow[(size_t)n * 8 + threadIdx.x] = s;
    }
    __syncthreads();
  }

  // checkpointed states x_k, x_2k, ... (< x_n); x_{i+1} is the input of stroke i
  int next_ck = (k > 0 && k < n) ? k - 1 : 0x7fffffff;
  if constexpr (kT == kInert) {
    // R_U: the point stays where it is; only T is regenerated (Eq. rT),
    // reset at the checkpoints, and each stroke's coverage differentiated.
    for (int c0 = 0; c0 < n; c0 += kChunk) {
      const int buf = (c0 / kChunk) & 1;
      const int cn = min(kChunk, n - c0);
      for (int j = 0; j < cn; ++j) {
        const int i = c0 + j;
        const StrokeRec g = load_rec(recs, i);
        const bool ck = i == next_ck;
        if (ck) next_ck = next_ck + k + 1 < n ? next_ck + k : 0x7fffffff;
        Chart ca = chart(x, y, g);
        float tot = 0.f;
        if (ck && id.active) {
          const float2 ckt = tape.ckpt_t[(size_t)((i + 1) / k) * P + id.p];
          tm = ckt.x;
          te = (int)ckt.y;
        }
        if (!wave_all(is_far<false>(ca.sig, uniform_leaf(g), g))) {
          Cover cv = cover(ca.sig, g, g.r);
          if (!ck) {
            tm *= cv.inv_q;
            renorm(tm, te);
          }
          float t = trans_value(tm, te);
          float lc = fmaf(lcr, g.cr, fmaf(lcg, g.cg, lcb * g.cb));
          const float dlt = lc - lt;
          float mu = t * dlt;
          float ta = t * cv.alpha;
          lt = fmaf(cv.alpha, dlt, lt);  // (1 - alpha) lt + alpha lc
          VjpOut vo = vjp_cover_only(ca, g, cv, mu);
          float v[8] = {vo.nmx, vo.nmy, vo.gphi, vo.gell, vo.gr, lcr * ta, lcg * ta, lcb * ta};
          tot = row_sums8<kT == kCapsule>(v, lane);
        }
        if (!(lane & 8)) lds[buf][wave * 4 + (lane >> 4)][j][value_index_of_lane(lane)] = tot;
      }
      __syncthreads();
      {
        const int j = threadIdx.x >> 3, vv = threadIdx.x & 7;
        if (j < cn) {
          float s = 0.f;
#pragma unroll
          for (int q = 0; q < 16; ++q) s += lds[buf][q][j][vv];
          prow[(size_t)(c0 + j) * 8 + vv] = vv < 2 ? -s : s;  // the centre's sign
        }
      }
    }
    return;
  }
  if constexpr (kT == kDrops) {
    // R_D: per stroke, the drops' adjoint (which regenerates x_i from
    // x_{i-1}, or starts from x_i where it is loaded), then the capsule
    // coverage at x_i as in the other transports.
    for (int c0 = 0; c0 < n; c0 += kChunk) {
      const int buf = (c0 / kChunk) & 1;
      const int cn = min(kChunk, n - c0);
      for (int j = 0; j < cn; ++j) {
        const int i = c0 + j;
        const StrokeRec g = load_rec(recs, i);
        const bool ck = i == next_ck;
        if (ck) next_ck = next_ck + k + 1 < n ? next_ck + k : 0x7fffffff;
        const bool pop = top_idx == i;
        if (pop) {
          double2 r = tape.side_xy[(size_t)(top - 1) * P + id.p];
          x = r.x;
          y = r.y;
          --top;
          top_idx = top > 0 ? tape.side_idx[(size_t)(top - 1) * P + id.p] : -1;
        }
        if (ck && id.active) {
          const double2 r = tape.ckpt_xy[(size_t)((i + 1) / k) * P + id.p];
          const float2 ckt = tape.ckpt_t[(size_t)((i + 1) / k) * P + id.p];
          x = r.x;
          y = r.y;
          tm = ckt.x;
          te = (int)ckt.y;
        }
        const DropsAdj da = drops_replay(x, y, g, pop || ck, lx, ly);
        float v[8] = {da.nmx, da.nmy, da.gphi, da.gell, da.gr, 0.f, 0.f, 0.f};
        Chart ca;
        chart_dist(x, y, g, ca);
        if (!wave_all(is_far<false>(ca.sig, uniform_leaf(g), g))) {
          chart_angle(g, ca);
          Cover cv = cover(ca.sig, g, g.r);
          if (!ck) {
            tm *= cv.inv_q;
            renorm(tm, te);
          }
          const float t = trans_value(tm, te);
          const float lc = fmaf(lcr, g.cr, fmaf(lcg, g.cg, lcb * g.cb));
          const float dlt = lc - lt;
          const float mu = t * dlt;
          const float ta = t * cv.alpha;
          lt = fmaf(cv.alpha, dlt, lt);  // (1 - alpha) lt + alpha lc
          const VjpOut vo = vjp_cover_only(ca, g, cv, mu);
          lx += vo.nmx;  // + mu d alpha / dx at x_i
          ly += vo.nmy;
          v[0] += vo.nmx;
          v[1] += vo.nmy;
          v[2] += vo.gphi;
          v[3] += vo.gell;
          v[4] += vo.gr;
          v[5] = lcr * ta;
          v[6] = lcg * ta;
          v[7] = lcb * ta;
        }
        const float tot = row_sums8<kT == kCapsule>(v, lane);
        if (!(lane & 8)) lds[buf][wave * 4 + (lane >> 4)][j][value_index_of_lane(lane)] = tot;
      }
      __syncthreads();
      {
        const int j = threadIdx.x >> 3, vv = threadIdx.x & 7;
        if (j < cn) {
          float s = 0.f;
#pragma unroll
          for (int q = 0; q < 16; ++q) s += lds[buf][q][j][vv];
          prow[(size_t)(c0 + j) * 8 + vv] = vv < 2 ? -s : s;  // the centre's sign
        }
      }
    }
    return;
  }
  constexpr bool kC = kT == kCoupled;
  // the next step that some lane of the wave loads (a checkpoint or a pop);
  // the coupled map votes on the lanes' own next pops instead (a wave
  // minimum in its general step costs it registers)
  int next_pop = kC ? 0x7fffffff : wave_next_pop(top_idx);
  int next_stop = min(next_ck, next_pop);
  for (int c0 = 0; c0 < n; c0 += kChunk) {
    const int buf = (c0 / kChunk) & 1;
    const int cn = min(kChunk, n - c0);
    int j = 0;
    while (j < cn) {
      // Common steps, far from every lane of the wave, up to the next step
      // where some lane loads its state (a wave-uniform index: a scalar
      // compare) or the stroke comes near: every lane regenerates x_i =
      // Phi_i(x_{i-1}) (Eq. rpos), and alpha, mu dalpha and the colour terms
      // vanish to FP32. Phi moves a point away from the stroke, so a wave
      // that is far before the step is far after it and the vote can come
      // first. Under uniform insertion the loop takes only waves whose lanes
      // all lie on the stroke's cap (far_cap_step; about 95% of far steps
      // here), and the rest leave it for one step: the loop keeps one path,
      // so the state it carries needs no register copies where paths would
      // join, and the polar step's chain of reciprocals interleaves with its
      // atan. The record is read before the exit tests and handed to the
      // general step: used on both sides of them, all its loads issue at the
      // top of the step (loads used only after the far vote would issue
      // after it, with their latency in the way).
      StrokeRec g;
      for (; j < cn; ++j) {
        const int i = c0 + j;  // stroke index (0-based); its input state is x_{i+1}
        g = load_rec(recs, i);
        if (__builtin_expect(kC ? (i == next_ck || wave_any(top_idx == i)) : i == next_stop, 0)) break;
        Chart ca;
        float v[5];
        if constexpr (kC) {  // the far vote needs the leaf's edge
          ca = chart(x, y, g);
          const Leaf lf = leaf_at<true>(ca, g, coup, i);
          if (!wave_all(is_far<true>(ca.sig, lf, g))) break;
          far_general_step<true>(x, y, lx, ly, ca, g, lf, v);
        } else {
          // one vote: beyond the far margin and on the cap, for every lane
          // (a far wave with a lane on the flank leaves for far_general_step)
          chart_dist(x, y, g, ca);
          if (__builtin_expect(!wave_all2(ca.sig > g.far_sig, ca.E > 0.f), 0)) break;
          far_cap_step(x, y, lx, ly, ca, g, v);
        }
        const float tot = row_sums5<kT == kCapsule>(v, lane);
        if (!(lane & 8)) lds[buf][wave * 4 + (lane >> 4)][j][value_index_of_lane(lane)] = tot;
      }
      if (j == cn) break;
      if constexpr (!kC) {
        // A far wave with a lane on the stroke's flank (about 5% of the
        // steps here, 0.6% being near): the flank-to-flank step when every
        // lane stays on the flank (about 3.5%), else the general map's far
        // step, without the general step's coverage, transmittance and
        // colour terms.
        if (c0 + j != next_stop) {
          Chart ca;
          chart_dist(x, y, g, ca);
          if (wave_all(ca.sig > g.far_sig)) {
            float v[5];
            if (!far_flank_step(x, y, lx, ly, ca, g, v)) {  // flank to flank, or
              chart_angle<true>(g, ca);
              far_general_step<false>(x, y, lx, ly, ca, g, uniform_leaf(g), v);
            }
            const float tot = row_sums5<true>(v, lane);
            if (!(lane & 8)) lds[buf][wave * 4 + (lane >> 4)][j][value_index_of_lane(lane)] = tot;
            ++j;
            continue;
          }
        }
      }
      {
        // The general step: the stroke is near some lane of the wave, or
        // some lane takes x_i from the side table (the floor bound there in
        // the forward pass), or the step is a checkpoint (drift reset).
        const int i = c0 + j;
        const bool ck = i == next_ck;
        if (ck) next_ck = next_ck + k + 1 < n ? next_ck + k : 0x7fffffff;
        const bool pop = top_idx == i;
        float tot;
        if (pop) {
          double2 r = tape.side_xy[(size_t)(top - 1) * P + id.p];
          x = r.x;
          y = r.y;
          --top;
          top_idx = top > 0 ? tape.side_idx[(size_t)(top - 1) * P + id.p] : -1;
        }
        if constexpr (!kC) {
          if (i == next_pop) next_pop = wave_next_pop(top_idx);
          next_stop = min(next_ck, next_pop);
        }
        float2 ckt = make_float2(1.f, 0.f);
        if (ck && id.active) {
          double2 r = tape.ckpt_xy[(size_t)((i + 1) / k) * P + id.p];
          ckt = tape.ckpt_t[(size_t)((i + 1) / k) * P + id.p];
          x = r.x;
          y = r.y;
        }
        const bool loaded = pop || ck;
        // One chart and one displacement serve both directions: for a
        // regenerated lane the chart is at x_{i-1} and Phi_i gives x_i;
        // for a loaded lane the chart is at x_i and psi_i gives the
        // (discarded) x_{i-1}, whose geometry the adjoint needs.
        Chart ca = chart(x, y, g);
        const Leaf lf = leaf_at<kC>(ca, g, coup, i);
        Move mv = displace<true>(ca, g, loaded, lf);
        const float da = ca.sgs * mv.dS, db = ca.sgh * mv.dH;
        VjpIn vi;
        vi.sgs = ca.sgs;
        vi.sgh = ca.sgh;
        vi.w = ca.w;
        vi.floored = mv.floored;
        // psi's increments x_{i-1} - x_i: the map's own for a loaded lane,
        // Phi's negated for a regenerated one
        const float sd = loaded ? 1.f : -1.f;
        vi.dsig = sd * mv.dsig;
        vi.dth = sd * mv.dth;
        vi.dsin = sd * mv.dsin;
        vi.dcos = sd * mv.dcos;
        vi.dtf = sd * mv.dtf;
        if (loaded) {  // in = chart point x_i, out = psi_i(x_i)
          vi.sig = ca.sig;
          vi.th = ca.th;
          vi.sn = ca.sn;
          vi.cs = ca.cs;
          vi.tf = mv.tf;
          vi.inv_p1 = ca.per > 0.f ? ca.inv_per : 0.f;
          vi.rho = mv.sig_o;
          vi.inv_p0 = mv.inv_per_o;
          vi.th_o = mv.th_o;
          vi.sn_o = mv.sn_o;
          vi.cs_o = mv.cs_o;
          vi.tf_o = mv.tf_o;
        } else {  // in = regenerated x_i, out = chart point x_{i-1}
          vi.sig = mv.sig_o;
          vi.th = mv.th_o;
          vi.sn = mv.sn_o;
          vi.cs = mv.cs_o;
          vi.tf = mv.tf_o;
          vi.inv_p1 = mv.inv_per_o;
          vi.rho = ca.sig;
          vi.inv_p0 = ca.inv_per;
          vi.th_o = ca.th;
          vi.sn_o = ca.sn;
          vi.cs_o = ca.cs;
          vi.tf_o = mv.tf;
          step_by(x, y, da, db, g);
        }
        Cover cv = cover(vi.sig, g, lf.r);
        vi.z = cv.z;
        vi.alpha = cv.alpha;
        vi.q = cv.q;
        vi.clamped = cv.clamped;
        if (ck) {
          tm = ckt.x;
          te = (int)ckt.y;
        } else {
          tm *= cv.inv_q;
          renorm(tm, te);
        }
        float t = trans_value(tm, te);
        float lc = fmaf(lcr, g.cr, fmaf(lcg, g.cg, lcb * g.cb));
        const float dlt = lc - lt;
        float mu = t * dlt;
        float ta = t * cv.alpha;
        lt = fmaf(cv.alpha, dlt, lt);  // (1 - alpha) lt + alpha lc
        VjpOut vo = vjp_step<true, kC>(vi, g, lx, ly, mu, lf);
        lx = vo.gx;
        ly = vo.gy;
        float v[8] = {vo.nmx, vo.nmy, vo.gphi, vo.gell, vo.gr, lcr * ta, lcg * ta, lcb * ta};
        tot = row_sums8<kT == kCapsule>(v, lane);
        if (!(lane & 8)) lds[buf][wave * 4 + (lane >> 4)][j][value_index_of_lane(lane)] = tot;
        ++j;
      }
    }
    __syncthreads();
    {
      const int j = threadIdx.x >> 3, vv = threadIdx.x & 7;
      if (j < cn) {
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < 16; ++q) s += lds[buf][q][j][vv];
        prow[(size_t)(c0 + j) * 8 + vv] = vv < 2 ? -s : s;  // the centre's sign
      }
    }
  }
}


template <int kT>
__global__ void __launch_bounds__(256)
    k_replay(const StrokeRec* __restrict__ recs, const float4* __restrict__ coup, int n,
             int width, int height, const float* __restrict__ palette,
             const float* __restrict__ grad_rgb, KTape tape, float* __restrict__ partial) {
  __shared__ ReduceLds lds;
  PixelId id = pixel_of_tile(blockIdx.x, blockIdx.y, width, height);
  const int tile = blockIdx.y * gridDim.x + blockIdx.x;
  float lcr = 0.f, lcg = 0.f, lcb = 0.f;
  if (id.active) {
    lcr = grad_rgb[3 * (size_t)id.p + 0];
    lcg = grad_rgb[3 * (size_t)id.p + 1];
    lcb = grad_rgb[3 * (size_t)id.p + 2];
  }
  replay_tile<kT>(recs, coup, n, id, width, height, palette, lcr, lcg, lcb, tape,
                  partial + (size_t)tile * (n + 1) * 8, lds);
}

// ---------------------------------------------------------------------------
// Fused fit over several jobs: one persistent launch pulls (job, tile) items
// through an atomic cursor (the largest jobs first). Per tile: the soft
// forward with tape, the L2 seed dL/dR = 2 (R - I*) / (3 P) kept in
// registers, the tile's loss partial, and at once the replay of the same
// tile (each lane reads back only its own tape). Partial rows are indexed by
// tile, so the order in which blocks take tiles cannot change any sum.
// ---------------------------------------------------------------------------
// The launch bound kW: kFusedWaves<kT>, or kFusedWavesLong for programs of
// long strokes (tbr_kernels.hpp gives the measurements).
template <int kT, int kW>
__global__ void __launch_bounds__(256, kW) k_fit_fused(FitJobsK jobs, int* __restrict__ cursor) {
  __shared__ ReduceLds lds;
  __shared__ float red[256];
  __shared__ int item_s;
  for (;;) {
    if (threadIdx.x == 0) item_s = atomicAdd(cursor, 1);
    __syncthreads();
    const int it = item_s;
    __syncthreads();
    if (it >= jobs.n_items) break;
    int jb = 0;
    while (jb + 1 < jobs.n_jobs && it >= jobs.job[jb + 1].item0) ++jb;
    const FitJobK& J = jobs.job[jb];
    const int tile = it - J.item0;
    PixelId id = pixel_of_tile(tile % J.tiles_x, tile / J.tiles_x, J.width, J.height);
    const int P = J.width * J.height;
    SoftOut o = soft_pixel<true, kT>(J.recs, J.coup, J.n, id, J.width, J.height, J.palette,
                                     J.tape);
    float lcr = 0.f, lcg = 0.f, lcb = 0.f, sq = 0.f;
    if (id.active) {
      float dr = o.cr - J.target[3 * (size_t)id.p + 0];
      float dg = o.cg - J.target[3 * (size_t)id.p + 1];
      float db = o.cb - J.target[3 * (size_t)id.p + 2];
      float sc = 2.0f / (3.0f * (float)P);
      lcr = sc * dr;
      lcg = sc * dg;
      lcb = sc * db;
      sq = fmaf(dr, dr, fmaf(dg, dg, db * db));
    }
    int m = id.active ? o.nrec : 0;  // side-table high-water mark, one atomic per wave
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(J.tape.status, m);
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) J.loss_part[tile] = red[0];
    replay_tile<kT>(J.recs, J.coup, J.n, id, J.width, J.height, J.palette, lcr, lcg, lcb,
                    J.tape, J.partial + (size_t)tile * (J.n + 1) * 8, lds);
  }
}

// ---------------------------------------------------------------------------
// Deterministic finalize: sum tile rows in tile order (two stages, FP64),
// then the chain rule to the program parameters.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
    k_sum_tiles(const float* __restrict__ partial, int rows8, int n_tiles, int tiles_per_group,
                double* __restrict__ out) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows8) return;
  int g = blockIdx.y;
  int t0 = g * tiles_per_group, t1 = min(n_tiles, t0 + tiles_per_group);
  double acc = 0.0;
  for (int t = t0; t < t1; ++t) acc += (double)partial[(size_t)t * rows8 + e];
  out[(size_t)g * rows8 + e] = acc;
}

__global__ void __launch_bounds__(256)
    k_finalize(const double* __restrict__ groups, int n_groups, KProgram p, KOpts o,
               KGrad grad, float* __restrict__ gcol, float* __restrict__ pal_terms) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > p.n) return;
  double s[8];
  for (int v = 0; v < 8; ++v) s[v] = 0.0;
  const int rows8 = (p.n + 1) * 8;
  for (int g = 0; g < n_groups; ++g)
    for (int v = 0; v < 8; ++v) s[v] += groups[(size_t)g * rows8 + (size_t)i * 8 + v];
  // colour gradient rows (stroke colours, then the background at row n)
  gcol[3 * i + 0] = (float)s[5];
  gcol[3 * i + 1] = (float)s[6];
  gcol[3 * i + 2] = (float)s[7];
  if (i == p.n) return;
  grad.cx[i] = (float)s[0];
  grad.cy[i] = (float)s[1];
  // a drop's map and coverage are invariant under rotation about its centre:
  // the angle gradient is exactly zero there (the sum above is rounding
  // noise). Not so under the coupling, whose profile turns with the stroke.
  grad.angle[i] = (p.length[i] == 0.f && !o.coupling) ? 0.f : (float)s[2];
  grad.length[i] = p.length[i] < 0.f ? -(float)s[3] : (float)s[3];  // d|L|/dL, +1 at 0
  grad.half_width[i] = (float)s[4];
  // colour weights s_ik = softmax(z_i / tau_c)_k (one-hot argmax when tau_c = 0)
  const float* z = p.logits + (size_t)i * p.k;
  float* gz = grad.logits + (size_t)i * p.k;
  float* pt = pal_terms + (size_t)i * p.k * 3;  // s_ik dL/dc_i, summed over i later
  int best = 0;
  float zmax = z[0];
  for (int j = 1; j < p.k; ++j)
    if (z[j] > zmax) {
      zmax = z[j];
      best = j;
    }
  if (o.tau_c > 0.f) {
    // logits: dL/dz_ik = s_ik (g . P_k - g . c_i) / tau_c
    float inv_tc = 1.0f / o.tau_c, tot = 0.f;
    for (int j = 0; j < p.k; ++j) tot += expf((z[j] - zmax) * inv_tc);
    float inv_tot = 1.0f / tot;
    double gc = 0.0;
    for (int j = 0; j < p.k; ++j) {
      double sj = (double)(expf((z[j] - zmax) * inv_tc) * inv_tot);
      gc += sj * (s[5] * p.palette[3 * j] + s[6] * p.palette[3 * j + 1] + s[7] * p.palette[3 * j + 2]);
    }
    for (int j = 0; j < p.k; ++j) {
      double sj = (double)(expf((z[j] - zmax) * inv_tc) * inv_tot);
      double gp = s[5] * p.palette[3 * j] + s[6] * p.palette[3 * j + 1] + s[7] * p.palette[3 * j + 2];
      gz[j] = (float)(sj * (gp - gc) * (double)inv_tc);
      pt[3 * j + 0] = (float)(sj * s[5]);
      pt[3 * j + 1] = (float)(sj * s[6]);
      pt[3 * j + 2] = (float)(sj * s[7]);
    }
  } else {
    for (int j = 0; j < p.k; ++j) {
      gz[j] = 0.f;
      float sj = j == best ? 1.f : 0.f;
      pt[3 * j + 0] = sj * (float)s[5];
      pt[3 * j + 1] = sj * (float)s[6];
      pt[3 * j + 2] = sj * (float)s[7];
    }
  }
}

// Palette gradient dL/dP_k = sum_i s_ik dL/dc_i (+ background at k = 0):
// one block per (k, channel), strided partial sums then a fixed tree.
__global__ void __launch_bounds__(256)
    k_palette_grad(const float* __restrict__ pal_terms, int n, int kpal,
                   const float* __restrict__ gcol, float* __restrict__ gpal) {
  __shared__ double red[256];
  const int e = blockIdx.x;  // k * 3 + channel
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += (double)pal_terms[(size_t)i * kpal * 3 + e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) gpal[e] = (float)(red[0] + (e < 3 ? (double)gcol[3 * n + e] : 0.0));
}

// Fixed-order sum of the per-block loss partials; loss = SSE / (3P).
__global__ void k_loss_final(const float* __restrict__ part, int n_part, float inv_count,
                             float* __restrict__ loss) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int j = threadIdx.x; j < n_part; j += blockDim.x) acc += part[j];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(red[0] * (double)inv_count);
}

// Adam on the packed parameter vector [cx|cy|angle|length|half_width|logits|palette]
// with one learning rate per group; clamps r into [r_lo, r_hi] and L into
// [-l_max, l_max].
__global__ void __launch_bounds__(256)
    k_adam(float* __restrict__ prm, const float* __restrict__ grd, float* __restrict__ m,
           float* __restrict__ v, int n, int kpal, KAdam a, const int32_t* __restrict__ records,
           int capacity) {
  // A step whose side table overflowed has an incomplete adjoint: leave the
  // parameters and moments as they were, so the step can be repeated with a
  // larger table.
  if (records && records[0] > capacity) return;
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  int total = 5 * n + n * kpal + 3 * kpal;
  if (e >= total) return;
  float lr;
  int grp = e < 5 * n ? e / n : (e < 5 * n + n * kpal ? 5 : 6);
  switch (grp) {
    case 0:
    case 1: lr = a.lr_centre; break;
    case 2: lr = a.lr_angle; break;
    case 3: lr = a.lr_length; break;
    case 4: lr = a.lr_width; break;
    case 5: lr = a.lr_logits; break;
    default: lr = a.lr_palette; break;
  }
  float g = grd[e];
  float mm = fmaf(a.beta1, m[e], (1.f - a.beta1) * g);
  float vv = fmaf(a.beta2, v[e], (1.f - a.beta2) * g * g);
  m[e] = mm;
  v[e] = vv;
  float mh = mm / a.bc1, vh = vv / a.bc2;
  float p = prm[e] - lr * mh / (sqrtf(vh) + a.eps);
  if (grp == 4) p = fminf(fmaxf(p, a.r_lo), a.r_hi);
  if (grp == 3) p = fminf(fmaxf(p, -a.l_max), a.l_max);
  if (grp == 6) p = fminf(fmaxf(p, 0.f), 1.f);
  prm[e] = p;
}

}  // namespace tbr

namespace tbr {

// ---------------------------------------------------------------------------
// Fitting loop (Sec. 5.1 parameterisation; Table hyper regulariser and
// schedule; Sec. 8 area budget). Free parameters, packed like the program:
//   [th_ax N | th_ay N | th_dx N | th_dy N | th_r N | th_c N*K | th_P K*3]
// with anchor a = a_lo + (a_hi - a_lo) sigmoid(th_a), offset
// d = l_max tanh(th_d) (componentwise), half-width
// r = (r_lo_frac + (r_hi_frac - r_lo_frac) sigmoid(th_r)) r0_i with r0_i
// geometric over the program, logits z = th_c and palette P = sigmoid(th_P).
// The stroke runs from a to a + d: m = a + d / 2, l = |d|, phi = atan2(d).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float logistic(float x) { return 1.0f / (1.0f + expf(-x)); }

__device__ __forceinline__ float window_r0(const KWindow& w, int i, int n) {
  return n > 1 ? w.r0_first * expf(w.r0_log_ratio * (float)i / (float)(n - 1)) : w.r0_first;
}

// One thread per packed entry; the thread of entry i < N also writes the
// stroke's five geometric parameters.
__global__ void __launch_bounds__(256)
    k_window_map(const float* __restrict__ th, float* __restrict__ nat, int n, int kpal,
                 KWindow w) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = 5 * n + n * kpal + 3 * kpal;
  if (e >= total) return;
  if (e < n) {
    const float ax = w.a_lo + w.a_span * logistic(th[e]);
    const float ay = w.a_lo + w.a_span * logistic(th[n + e]);
    const float dx = w.l_max * tanhf(th[2 * n + e]);
    const float dy = w.l_max * tanhf(th[3 * n + e]);
    const float len = sqrtf(fmaf(dx, dx, dy * dy));
    nat[e] = fmaf(0.5f, dx, ax);
    nat[n + e] = fmaf(0.5f, dy, ay);
    nat[2 * n + e] = len > 0.f ? atan2f(dy, dx) : 0.f;
    nat[3 * n + e] = len;
    nat[4 * n + e] = (w.r_lo_frac + w.r_span_frac * logistic(th[4 * n + e])) * window_r0(w, e, n);
  } else if (e >= 5 * n && e < 5 * n + n * kpal) {
    nat[e] = th[e];
  } else if (e >= 5 * n + n * kpal) {
    nat[e] = logistic(th[e]);
  }
}

// lambda sum_i l_i + lambda_A sum_i A_l(r_i), added to *loss in a fixed
// order (one block).
__global__ void k_reg_loss(const float* __restrict__ nat, int n, KWindow w, float* __restrict__ loss) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double l = fabs((double)nat[3 * n + i]), r = nat[4 * n + i];
    acc += (double)w.lambda_length * l + (double)w.lambda_area * (2.0 * l * r + 3.14159265358979323846 * r * r);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)((double)*loss + red[0]);
}

__device__ __forceinline__ float adam_update(float p, float g, float& m, float& v, float lr,
                                             const KAdam& a) {
  m = fmaf(a.beta1, m, (1.f - a.beta1) * g);
  v = fmaf(a.beta2, v, (1.f - a.beta2) * g * g);
  const float mh = m / a.bc1, vh = v / a.bc2;
  return p - lr * mh / (sqrtf(vh) + a.eps);
}

// Chain rule of the windows (the data gradient g_nat plus the regularisers'
// gradient in the natural parameters), then Adam on the free parameters with
// the group steps lr_centre (anchor), lr_length (offset), lr_width
// (half-width), lr_logits (colour) and lr_palette (palette). Skipped when the
// step's side table overflowed (records > capacity), like the fit step.
__global__ void __launch_bounds__(256)
    k_window_adam(float* __restrict__ th, const float* __restrict__ g_nat,
                  float* __restrict__ m, float* __restrict__ v, int n, int kpal, KWindow w,
                  KAdam a, const int32_t* __restrict__ records, int capacity) {
  if (records && records[0] > capacity) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = 5 * n + n * kpal + 3 * kpal;
  if (e >= total) return;
  if (e < n) {
    const float sax = logistic(th[e]), say = logistic(th[n + e]);
    const float tdx = tanhf(th[2 * n + e]), tdy = tanhf(th[3 * n + e]);
    const float dx = w.l_max * tdx, dy = w.l_max * tdy;
    const float len = sqrtf(fmaf(dx, dx, dy * dy));
    const float sr = logistic(th[4 * n + e]);
    const float c0 = window_r0(w, e, n);
    const float r = (w.r_lo_frac + w.r_span_frac * sr) * c0;
    const float gmx = g_nat[e], gmy = g_nat[n + e], gphi = g_nat[2 * n + e];
    // data term + lambda l + lambda_A A_l(r): dA/dl = 2 r, dA/dr = P_l(r)
    const float gl = g_nat[3 * n + e] + w.lambda_length + w.lambda_area * 2.f * r;
    const float gr = g_nat[4 * n + e] + w.lambda_area * fmaf(kTwoPi, r, 2.f * len);
    float gdx = 0.5f * gmx, gdy = 0.5f * gmy;
    if (len > 0.f) {  // l = |d|, phi = atan2(d): no direction at a drop
      const float il = 1.f / len, il2 = il * il;
      gdx = fmaf(gl * dx, il, fmaf(-gphi * dy, il2, gdx));
      gdy = fmaf(gl * dy, il, fmaf(gphi * dx, il2, gdy));
    }
    const float g5[5] = {gmx * w.a_span * sax * (1.f - sax), gmy * w.a_span * say * (1.f - say),
                         gdx * w.l_max * (1.f - tdx * tdx), gdy * w.l_max * (1.f - tdy * tdy),
                         gr * w.r_span_frac * c0 * sr * (1.f - sr)};
    const float lr5[5] = {a.lr_centre, a.lr_centre, a.lr_length, a.lr_length, a.lr_width};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const size_t o = (size_t)q * n + e;
      float mm = m[o], vv = v[o];
      th[o] = adam_update(th[o], g5[q], mm, vv, lr5[q], a);
      m[o] = mm;
      v[o] = vv;
    }
  } else if (e >= 5 * n) {
    const bool pal = e >= 5 * n + n * kpal;
    float g = g_nat[e];
    if (pal) {
      const float s = logistic(th[e]);
      g *= s * (1.f - s);
    }
    float mm = m[e], vv = v[e];
    th[e] = adam_update(th[e], g, mm, vv, pal ? a.lr_palette : a.lr_logits, a);
    m[e] = mm;
    v[e] = vv;
  }
}

}  // namespace tbr

namespace tbr {

// ---------------------------------------------------------------------------
// Closed-form compensation of an inert-mark program (Sec. "Closed-form
// compensation baseline"). Stroke i's anchor (and, for the endpoint variant,
// its end) must be pre-imaged through every later stroke in that stroke's
// compensated geometry, so the strokes are finished one at a time, last
// first. The N(N-1)/2 point maps are reordered into N sequential steps:
// before step k the pending points of strokes 0..k have been pre-imaged
// through strokes N-1..k+1, so stroke k's are final; step k pushes the
// points of strokes 0..k-1 through stroke k's backward map, all in
// parallel, and the thread that finishes stroke k-1's points builds its
// compensated record for the next step (two LDS slots, alternating). One
// workgroup runs the steps, so a step's barrier is a workgroup barrier. A
// step inside a later footprint (sigma' <= r) is blocked (Lemma
// obstruction): the extended map clamps it with the floor (eps r)^2, or it
// is skipped.
// ---------------------------------------------------------------------------

// Compensated geometry and backward-map record of stroke k from its final
// points (anchor, and end for the endpoint variant); writes the outputs.
__device__ __forceinline__ void comp_record(const KProgram& p, float eps, int endpoint, int k,
                                            const double2* __restrict__ pts, float* ocx,
                                            float* ocy, float* oangle, float* olength,
                                            StrokeRec& out) {
  const int np = endpoint ? 2 : 1;
  const double2 a = pts[np * k];
  float ang = p.angle[k], len = p.length[k];
  float ce = cosf(ang), se = sinf(ang);
  double mx, my;
  if (endpoint) {
    const double2 b = pts[2 * k + 1];
    const float dx = (float)(b.x - a.x), dy = (float)(b.y - a.y);
    const float d = sqrtf(fmaf(dx, dx, dy * dy));
    mx = 0.5 * (a.x + b.x);
    my = 0.5 * (a.y + b.y);
    len = d;
    if (d > 0.f) {
      ce = dx / d;
      se = dy / d;
      ang = atan2f(dy, dx);
    }
  } else {
    mx = a.x + (double)(0.5f * len * ce);
    my = a.y + (double)(0.5f * len * se);
  }
  ocx[k] = (float)mx;
  ocy[k] = (float)my;
  oangle[k] = ang;
  olength[k] = len;
  StrokeRec g{};
  const float ell = fabsf(len), r = p.half_width[k];
  g.mx = mx;
  g.my = my;
  g.ce = ce;
  g.se = se;
  g.ell = ell;
  g.hl = 0.5f * ell;
  g.two_ell = ell + ell;
  g.r = r;
  g.ar = r * fmaf(kPi, r, ell + ell);
  g.per_r = fmaf(kTwoPi, r, ell + ell);
  g.floor_c = (eps * r) * (eps * r);
  out = g;
}

__global__ void __launch_bounds__(kCompThreadsK)
    k_compensate(KProgram p, float eps, int endpoint, int skip, double2* __restrict__ pts,
                 float* __restrict__ ocx, float* __restrict__ ocy, float* __restrict__ oangle,
                 float* __restrict__ olength, int32_t* __restrict__ blocked) {
  __shared__ StrokeRec rec[2];
  const int N = p.n, np = endpoint ? 2 : 1;
  for (int i = threadIdx.x; i < N; i += kCompThreadsK) {
    const float c = cosf(p.angle[i]), sn = sinf(p.angle[i]), hl = 0.5f * p.length[i];
    pts[np * i] = make_double2((double)p.cx[i] - (double)(hl * c), (double)p.cy[i] - (double)(hl * sn));
    if (endpoint)
      pts[2 * i + 1] = make_double2((double)p.cx[i] + (double)(hl * c), (double)p.cy[i] + (double)(hl * sn));
    blocked[i] = 0;
  }
  // the last stroke has no later stroke: its points are final as drawn
  if ((int)threadIdx.x == (N - 1) % kCompThreadsK)
    comp_record(p, eps, endpoint, N - 1, pts, ocx, ocy, oangle, olength, rec[(N - 1) & 1]);
  __syncthreads();
  for (int k = N - 1; k > 0; --k) {
    const StrokeRec g = rec[k & 1];
    const Leaf lf = uniform_leaf(g);
    for (int i = threadIdx.x; i < k; i += kCompThreadsK) {
      int nb = 0;
      for (int q = 0; q < np; ++q) {
        double2 v = pts[np * i + q];
        const Chart c = chart(v.x, v.y, g);
        const bool inside = c.sig <= g.r;
        nb += inside ? 1 : 0;
        if (!(inside && skip)) {
          advance(v.x, v.y, c, displace(c, g, true, lf), g);
          pts[np * i + q] = v;
        }
      }
      if (nb) blocked[i] += nb;
      // stroke k-1 has now met every later stroke: build its record
      if (i == k - 1) comp_record(p, eps, endpoint, i, pts, ocx, ocy, oangle, olength, rec[i & 1]);
    }
    __syncthreads();
  }
}

}  // namespace tbr

namespace tbr {
// The per-pixel kernels for each transport: the capsule map, its calibrated
// coupling, the inert-mark model and the sixteen drops.
#define TBR_INSTANTIATE_RENDER(T)                                                               \
  template __global__ void k_trace_soft<T>(const StrokeRec*, const float4*, int, int, int,      \
                                           const float*, float*, KTape, KSeed);                 \
  template __global__ void k_trace_hard<T>(const StrokeRec*, const float4*, int, int, int,      \
                                           const float*, float*, int32_t*, int32_t*);
#define TBR_INSTANTIATE_ADJOINT(T)                                                              \
  template __global__ void k_replay<T>(const StrokeRec*, const float4*, int, int, int,          \
                                       const float*, const float*, KTape, float*);              \
  template __global__ void k_fit_fused<T, kFusedWaves<T>>(FitJobsK, int*);
TBR_INSTANTIATE_RENDER(kCapsule)
TBR_INSTANTIATE_RENDER(kCoupled)
TBR_INSTANTIATE_RENDER(kInert)
TBR_INSTANTIATE_RENDER(kDrops)
TBR_INSTANTIATE_ADJOINT(kCapsule)
TBR_INSTANTIATE_ADJOINT(kCoupled)
TBR_INSTANTIATE_ADJOINT(kInert)
TBR_INSTANTIATE_ADJOINT(kDrops)
template __global__ void k_fit_fused<kCapsule, kFusedWavesLong>(FitJobsK, int*);
#undef TBR_INSTANTIATE_RENDER
#undef TBR_INSTANTIATE_ADJOINT
}  // namespace tbr
