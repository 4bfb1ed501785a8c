// tbr_device.hpp -- per-lane FP32 arithmetic of the capsule transport.
//
// One pixel per lane. Stroke constants arrive as a wave-uniform 80-byte
// record; everything else lives in VGPRs. All maps are the
// closed forms of Sec. 4 of the paper (TBR, arxiv 2609.08722):
//   distance sigma to the segment, Steiner area A_l(s) = 2 l s + pi s^2 and
//   perimeter P_l(s) = 2 l + 2 pi s (Eq. steiner), the centred arclength
//   fraction w (Prop. centred arclength), the backward root (Eq. back) with
//   the implemented floor C >= (eps r)^2 (Sec. 5.2), the forward root
//   (Eq. fwd), and the soft coverage of Eq. (relax) clamped at 1 - 1e-7.
//   The calibrated variant (Eq. coupling, Eq. profile) changes only the area
//   a leaf receives, and with it where the leaf's deposit ends (Leaf).
//
// Transcendentals: raw v_sqrt/v_rcp/v_exp (about 1 ulp) plus the
// polynomials of minimax_coeffs.h (Remez fits): 2 atan on [0, 1] for the
// half-angle cap angle, sin and cos on [0, pi/2] (about 1e-7 absolute in
// FP32). Every branch of the chart is written
// branch-free: on the flank of the capsule the cap angle is exactly 0, its
// sine 0 and cosine 1, so the cap formulas reduce to the flank ones.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "minimax_coeffs.h"

namespace tbr {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kHalfPi = 1.57079632679489661923f;
constexpr float kLog2e = 1.44269504088896340736f;
// alpha = e^z / (1 + e^z) <= 1 - 1e-7   <=>   e^z <= (1 - 1e-7) / 1e-7
constexpr float kEzMax = 9999999.0f;
// Coverage below sigmoid(-28) = 7e-13 is skipped for a whole wave: 1 - alpha
// then rounds to exactly 1.0f, so transmittance is unchanged bitwise and every
// dropped colour / gradient term is below 2^-40 of the terms kept.
constexpr float kFarZ = -28.f;
// Smallest normal FP32 number: the floor of a reciprocal's argument where the
// argument is 0 only together with the factor it multiplies.
constexpr float kMinNormal = 1.17549435e-38f;

// Per-stroke constants, prepared once per launch (80 bytes, 20 words).
// Wave-uniform values are precomputed here: the vector ALU would otherwise
// spend a full instruction per wave on each of them.
struct __align__(16) StrokeRec {
  double mx, my;    // centre m, in FP64 like the trajectory state
  float ce, se;     // direction e = (cos phi, sin phi)
  float hl, ell;    // half-length l/2 and length l = |L|
  float two_ell;    // 2 l
  float r, ar;      // half-width r and inserted area A_l(r)
  float per_r;      // Steiner perimeter P_l(r) = 2 l + 2 pi r
  float inv_wd;     // 1 / max(tau r, tau_min)
  float floor_c;    // (eps r)^2
  float far_sig;    // r + 28 wd (at least): beyond it the coverage is below
                    // sigmoid(-28) and psi's floor cannot bind
  float dwd_dr;     // d max(tau r, tau_min) / dr: tau or 0
  float cr, cg, cb; // colour c_i = softmax(z_i / tau_c) P (or P[argmax])
  int label;        // argmax_k z_ik (hard colour index)
};
static_assert(sizeof(StrokeRec) == 80, "stroke record must be 80 bytes");

// Wave votes over the active lanes: the ballot's lane mask is compared with
// exec by scalar instructions, with no vector instruction beyond the compare
// that produces the predicate.
__device__ __forceinline__ bool wave_all(bool p) {
  return __builtin_amdgcn_ballot_w64(p) == __builtin_amdgcn_read_exec();
}
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }
// p && q on every active lane: the two ballots are combined in scalar
// registers (a vector && would first turn the compare results into 0 / 1).
__device__ __forceinline__ bool wave_all2(bool p, bool q) {
  return (__builtin_amdgcn_ballot_w64(p) & __builtin_amdgcn_ballot_w64(q)) ==
         __builtin_amdgcn_read_exec();
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hw_exp(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }

// The cap angle of a point from its folded offset (E, H) from the cap's
// centre, by the half-angle identity th = 2 atan(t), t = tan(th / 2) =
// E / (sigma + H) (sh = sigma + H). For th in [0, pi/2] the argument lies in
// [0, 1], so unlike atan(E / H) it needs no fold into [0, 1] (no min / max,
// select or pi/2 - atan). The polynomial for 2 atan (Horner's rule in t^2)
// gives the angle within 3.6e-7 in FP32 (RMS 7e-8), against 3.8e-7 (RMS
// 1.8e-7) for the folded atan(min / max) form of one degree less.
constexpr int kTwoAtanTerms = sizeof(kTwoAtan) / sizeof(kTwoAtan[0]);
__device__ __forceinline__ float cap_angle(float E, float sh) {
  const float t = E * rcp(sh);
  const float u = t * t;
  float p = kTwoAtan[kTwoAtanTerms - 1];
#pragma unroll
  for (int j = kTwoAtanTerms - 2; j >= 0; --j) p = fmaf(p, u, kTwoAtan[j]);
  return t * p;
}

// Chart of a point w.r.t. one stroke: local coordinates, distance to the
// segment, cap angle and centred arclength fraction folded into the first
// quadrant (the reflections of Prop. centred arclength unfold it again).
// The point is held in FP64; its offset from the stroke centre is rounded to
// FP32 once, and everything after that is FP32.
struct Chart {
  float s, h;      // signed coordinates along e and along n = (-se, ce)
  float sgs, sgh;  // their signs, +1 at 0
  float S, H;      // |s|, |h|
  float E;         // overshoot past the segment end, max(S - l/2, 0)
  float sig;       // distance to the segment
  float th;        // cap angle measured from the normal; 0 on the flank
  float sn, cs;    // sin / cos of th (E / sig, H / sig)
  float inv_sig;   // 1 / sigma, floored on the segment
  float per;       // P_l(sigma)
  float inv_per;   // 1 / P_l(sigma), floored at the drop centre (where t = 0)
  float w;         // arclength fraction from the flank midpoint, [0, 1/4]
};

// The chart in two parts: the distance (all a far vote needs), then the
// angle, fraction and reciprocals. kFar: the point is known to lie off the
// segment (sigma > 0, as beyond a stroke's far margin), so no reciprocal
// needs a floor and cos th needs no select.
__device__ __forceinline__ void chart_dist(double x, double y, const StrokeRec& g, Chart& c) {
  float dx = (float)(x - g.mx), dy = (float)(y - g.my);
  // The inner products take + 0, so s and h are never -0 and each fold sign,
  // one bit insert, is sgn with sgn(0) = +1.
  c.s = fmaf(dx, g.ce, fmaf(dy, g.se, 0.f));
  c.h = fmaf(dy, g.ce, fmaf(-dx, g.se, 0.f));
  c.sgs = copysignf(1.f, c.s);
  c.sgh = copysignf(1.f, c.h);
  c.S = fabsf(c.s);
  c.H = fabsf(c.h);
  c.E = fmaxf(c.S - g.hl, 0.f);
  c.sig = hw_sqrt(fmaf(c.H, c.H, c.E * c.E));
}

// The cap angle alone, for a point off the segment (sigma > 0): all that a
// far step which stays on the cap needs of the chart's angle part.
__device__ __forceinline__ float far_theta(const Chart& c) { return cap_angle(c.E, c.sig + c.H); }

template <bool kFar = false>
__device__ __forceinline__ void chart_angle(const StrokeRec& g, Chart& c) {
  if constexpr (kFar) {
    c.th = far_theta(c);
    c.inv_sig = rcp(c.sig);
    c.sn = c.E * c.inv_sig;
    c.cs = c.H * c.inv_sig;
    c.per = fmaf(kTwoPi, c.sig, g.two_ell);
    c.inv_per = rcp(c.per);
  } else {
    // on the segment E = sigma = H = 0, so the floored reciprocals give
    // th = 0 and sin th = 0
    c.th = cap_angle(c.E, fmaxf(c.sig + c.H, kMinNormal));
    c.inv_sig = rcp(fmaxf(c.sig, kMinNormal));
    c.sn = c.E * c.inv_sig;
    c.cs = c.sig > 0.f ? c.H * c.inv_sig : 1.f;
    c.per = fmaf(kTwoPi, c.sig, g.two_ell);           // P_l(sigma)
    c.inv_per = rcp(fmaxf(c.per, kMinNormal));
  }
  const float t = fmaf(c.sig, c.th, fminf(c.S, g.hl));  // arclength from the flank midpoint
  c.w = t * c.inv_per;                                  // drop centre: t = 0, w = 0
}

__device__ __forceinline__ Chart chart(double x, double y, const StrokeRec& g) {
  Chart c;
  chart_dist(x, y, g, c);
  chart_angle(g, c);
  return c;
}

// Distance whose parallel set has area Q: the cancellation-free root
// s = Q / D of pi s^2 + 2 l s = Q, D = l + sqrt(l^2 + pi Q) (Eq. back /
// Eq. fwd). As pi s + l = sqrt(l^2 + pi Q), D also gives the divisor of a
// distance increment from sig to s: 2 l + pi (sig + s) = pi sig + D.
struct Root {
  float sig_o, d;
};
__device__ __forceinline__ Root area_root(float q, const StrokeRec& g) {
  Root o;
  o.d = g.ell + hw_sqrt(fmaf(g.ell, g.ell, kPi * q));
  o.sig_o = q * rcp(o.d);
  return o;
}

// sin(d) and cos(d) - 1 for d in [-pi/2, pi/2] (odd / even polynomials).
__device__ __forceinline__ void sincosm1(float d, float& s, float& cm1) {
  float u = d * d;
  float ps = kSin[5];
  ps = fmaf(ps, u, kSin[4]);
  ps = fmaf(ps, u, kSin[3]);
  ps = fmaf(ps, u, kSin[2]);
  ps = fmaf(ps, u, kSin[1]);
  ps = fmaf(ps, u, kSin[0]);
  s = d * ps;
  float pc = kCos[5];
  pc = fmaf(pc, u, kCos[4]);
  pc = fmaf(pc, u, kCos[3]);
  pc = fmaf(pc, u, kCos[2]);
  pc = fmaf(pc, u, kCos[1]);
  cm1 = u * pc;  // kCos[0] == 1
}

// sin(d) and cos(d) - 1 for |d| < 1/16 by their Taylor series through d^5
// and d^6: the first omitted terms are below |d|^7 / 5040 < 7.5e-13 and
// d^8 / 40320 < 6e-15, far below FP32 resolution. A stroke turns a point's
// cap angle by less than this almost always, so a wave whose lanes all do
// takes these shorter polynomials.
constexpr float kSmallTurn = 0.0625f;
__device__ __forceinline__ void sincosm1_small(float d, float& s, float& cm1) {
  float u = d * d;
  s = d * fmaf(u, fmaf(u, 1.f / 120.f, -1.f / 6.f), 1.f);
  cm1 = u * fmaf(u, fmaf(u, -1.f / 720.f, 1.f / 24.f), -0.5f);
}

// Below |d| = 2^-12, sin d = d and cos d - 1 = -d^2 / 2 to within d^3 / 6 <
// 2.4e-12 and d^4 / 24 < 1.5e-16: relative errors below 1e-8, under FP32
// rounding. A far stroke turns a point's cap angle by about 1e-5 rad, so
// almost every wave of a far step takes this first-order rotation.
constexpr float kTinyTurn = 2.44140625e-4f;  // 2^-12

// (R(d) - I) p for p = (a, b) in the folded frame, where R(d) turns the
// cap angle (measured from the normal towards the segment direction) by d:
// returns (a (cos d - 1) + b sin d, b (cos d - 1) - a sin d). kTiny: |d| <
// kTinyTurn for every lane (first order; see above).
template <bool kTiny>
__device__ __forceinline__ void turn_increment(float d, float a, float b, float& ra,
                                               float& rb) {
  if constexpr (kTiny) {
    const float hd = -0.5f * d;
    ra = d * fmaf(a, hd, b);
    rb = d * fmaf(b, hd, -a);
  } else {
    float sd, cm1;
    if (wave_all(fabsf(d) < kSmallTurn)) {
      sincosm1_small(d, sd, cm1);
    } else {
      sincosm1(d, sd, cm1);
    }
    ra = fmaf(a, cm1, b * sd);
    rb = fmaf(b, cm1, -(a * sd));
  }
}

// What the stroke inserts along the leaf of a charted point. Uniform
// insertion (Eq. phi): the area A_l(r) on every leaf, whose deposit ends at
// distance r. Calibrated coupling (Eq. coupling, Eq. profile): the leaf of
// centred fraction w receives G = A_l(r) g(w), g(w) = 1 + sum_k c_k
// cos(4 pi k w), and its deposit ends at the root rl of A_l(rl) = G; Eq.
// back and Eq. fwd then hold with r replaced by rl.
struct Leaf {
  float r;        // edge of the deposit on this leaf
  float ar;       // area inserted along it, A_l(r) or G
  float g;        // g(w) (coupled only)
  float dg;       // dg/dw (coupled only)
  float inv_per;  // 1 / P_l(rl) (coupled only)
};

__device__ __forceinline__ Leaf uniform_leaf(const StrokeRec& g) {
  Leaf lf;
  lf.r = g.r;
  lf.ar = g.ar;
  lf.g = 1.f;
  lf.dg = 0.f;
  lf.inv_per = 0.f;
  return lf;
}

// a = (a0, a1, a2, a3): g as the cubic a0 + a1 W + a2 W^2 + a3 W^3 in
// W = cos(4 pi w) (cos 2x = 2 cos^2 x - 1, cos 3x = 4 cos^3 x - 3 cos x:
// a0 = 1 - c2, a1 = c1 - 3 c3, a2 = 2 c2, a3 = 4 c3). w is folded into
// [0, 1/4], so 4 pi w - pi/2 lies in the polynomials' range. A profile
// that is not positive somewhere is invalid input; there g is taken as 0.
__device__ __forceinline__ Leaf coupled_leaf(float w, const StrokeRec& g, const float4 a) {
  Leaf lf;
  float s, cm1;
  sincosm1(fmaf(2.f * kTwoPi, w, -kHalfPi), s, cm1);
  const float W = -s;          // cos(4 pi w)
  const float s4 = 1.f + cm1;  // sin(4 pi w)
  const float gv = fmaf(fmaf(fmaf(a.w, W, a.z), W, a.y), W, a.x);
  const float dgw = fmaf(fmaf(3.f * a.w, W, 2.f * a.z), W, a.y);
  const bool pos = gv > 0.f;
  lf.g = pos ? gv : 0.f;
  lf.dg = pos ? -2.f * kTwoPi * s4 * dgw : 0.f;  // dW/dw = -4 pi sin(4 pi w)
  lf.ar = g.ar * lf.g;
  // rl = G / (l + sqrt(l^2 + pi G)), and P_l(rl) = 2 sqrt(l^2 + pi G)
  const float X = fmaf(g.ell, g.ell, kPi * lf.ar);
  const float rs = X > 0.f ? __builtin_amdgcn_rsqf(X) : 0.f;
  lf.r = lf.ar > 0.f ? lf.ar * rcp(g.ell + X * rs) : 0.f;
  lf.inv_per = 0.5f * rs;
  return lf;
}

// A lane whose coverage z = (edge - sigma) / wd is below kFarZ. Uniform
// insertion compares sigma with the stroke's precomputed r + 28 wd (one
// compare); a coupled leaf's edge varies along the stroke.
template <bool kC>
__device__ __forceinline__ bool is_far(float sig, const Leaf& lf, const StrokeRec& g) {
  if constexpr (kC) {
    return sig - lf.r > g.far_sig - g.r;
  } else {
    return sig > g.far_sig;
  }
}

// d (eps r)^2 / dr = 2 eps^2 r = 2 (eps r)^2 / r (used where the floor binds).
__device__ __forceinline__ float dfloor_dr(const StrokeRec& g) {
  return g.r > 0.f ? 2.f * g.floor_c * rcp(g.r) : 0.f;
}

// Backward numerator C = A(sigma') - A(rl), factored (Eq. back).
__device__ __forceinline__ float back_area(float sig, const Leaf& lf, float two_ell) {
  return (sig - lf.r) * fmaf(kPi, sig + lf.r, two_ell);
}

// Forward numerator B = A(sigma) + A(rl) (Eq. fwd).
__device__ __forceinline__ float fwd_area(float sig, const Leaf& lf, float two_ell) {
  return fmaf(sig, fmaf(kPi, sig, two_ell), lf.ar);
}

// One application of the insertion map or its inverse to a charted point,
// as a DISPLACEMENT in the folded local frame. The new point is the one on
// the level curve at distance sig_o with the same fraction w. Writing the
// folded position as F(t, s) = (t - s (th - sin th), s - s (1 - cos th)),
// th = max(t - l/2, 0) / s, t = w P_l(s), the displacement is assembled from
//   dsig = sig_o - sig = (A(sig_o) - A(sig)) / (2 l + pi (sig + sig_o)),
//     where A(sig_o) - A(sig) = -A(r) (psi), +A(r) (Phi) or the floor term,
//   dt   = 2 pi w dsig,
//   dth  = dsig l (pi - 2 th) / (P_l(sig) sig_o)   (cap to cap; the identity
//          2 pi w - th = l (pi - 2 th) / P_l(sig) removes the cancellation),
//   and the rotation of (sin th, cos th) by dth,
// so no term of the size of the distance itself is rounded: the FP64 state
// then advances by a small FP32 increment.
struct Move {
  float sig_o;           // distance of the new point
  float dS, dH;          // folded displacement
  float th_o, sn_o, cs_o;  // cap angle of the new point and its sin / cos
  float inv_per_o;       // 1 / P_l(sig_o) (kPer only)
  bool floored;          // psi only: the floor C >= (eps r)^2 bound
  // Increments new - old of the chart coordinates, each formed without
  // cancellation (the replay's adjoint is built on them; unused elsewhere):
  float dsig, dth, dsin, dcos;
  float tf, tf_o;        // flank part min(S, l/2) of the arclength, old and new point
  float dtf;             // tf_o - tf
  bool all_cap;          // regenerate only: every lane of the wave on the cap
};

// Flank part of the arclength of both points and its increment: dS itself
// when both lie on the flank, 0 when both lie on a cap.
__device__ __forceinline__ void flank_part(const Chart& c, const StrokeRec& g, Move& m) {
  const float S_o = c.S + m.dS;
  m.tf = fminf(c.S, g.hl);
  m.tf_o = fminf(S_o, g.hl);
  m.dtf = fmaxf(c.S, S_o) <= g.hl ? m.dS : m.tf_o - m.tf;
}

// kPer: also return 1 / P_l(sig_o). The root of Eq. (back) / Eq. (fwd)
// satisfies sqrt(l^2 + pi q) = l + pi sig_o, so P_l(sig_o) =
// 2 sqrt(l^2 + pi q): one reciprocal square root gives both.
// kFloor = false: psi of a point where the floor cannot bind (C > (eps r)^2
// known beforehand), without the floor's test and terms.
template <bool kPer = false, bool kFloor = true>
__device__ __forceinline__ Move displace(const Chart& c, const StrokeRec& g, bool backward,
                                         const Leaf& lf) {
  Move m;
  const float two_ell = g.two_ell;
  // psi: Eq. (back) with the implemented floor; Phi: Eq. (fwd)
  float cq = back_area(c.sig, lf, two_ell);
  m.floored = kFloor && backward && cq < g.floor_c;
  float q = backward ? (kFloor ? fmaxf(cq, g.floor_c) : cq) : fwd_area(c.sig, lf, two_ell);
  float num =
      backward ? (m.floored ? g.floor_c - c.sig * fmaf(kPi, c.sig, two_ell) : -lf.ar) : lf.ar;
  float d;
  if constexpr (kPer) {
    const float X = fmaf(g.ell, g.ell, kPi * q);
    const float rs = __builtin_amdgcn_rsqf(X);
    d = g.ell + X * rs;
    m.sig_o = q * rcp(d);
    m.inv_per_o = 0.5f * rs;
  } else {
    const Root rt = area_root(q, g);
    m.sig_o = rt.sig_o;
    d = rt.d;
    m.inv_per_o = 0.f;
  }
  float dsig = num * rcp(fmaf(kPi, c.sig, d));
  float dt = kTwoPi * c.w * dsig;
  float t_o = c.w * fmaf(kTwoPi, m.sig_o, two_ell);
  const float inv_sig_o = rcp(m.sig_o);
  float th_o = fminf(fmaxf(t_o - g.hl, 0.f) * inv_sig_o, kHalfPi);
  const bool cap_in = c.th > 0.f, cap_out = th_o > 0.f;
  // 1 / P_l(sig) is the chart's reciprocal (it also gives w)
  float dth_cc = dsig * g.ell * (kPi - 2.f * c.th) * (c.inv_per * inv_sig_o);
  float dth = (cap_in && cap_out) ? dth_cc : th_o - c.th;
  float sd, cdm1;
  if (wave_all(fabsf(dth) < kSmallTurn)) {
    sincosm1_small(dth, sd, cdm1);
  } else {
    sincosm1(dth, sd, cdm1);
  }
  float dsin = fmaf(c.sn, cdm1, c.cs * sd);
  float dcos = fmaf(c.cs, cdm1, -(c.sn * sd));
  m.sn_o = c.sn + dsin;
  m.cs_o = c.cs + dcos;
  m.th_o = (cap_in && cap_out) ? c.th + dth : th_o;
  float extra = (cap_in && cap_out) ? 0.f : dt - dsig * th_o - c.sig * dth;
  m.dS = fmaf(dsig, m.sn_o, fmaf(c.sig, dsin, extra));
  m.dH = fmaf(dsig, m.cs_o, c.sig * dcos);
  m.dsig = dsig;
  m.dth = dth;
  m.dsin = dsin;
  m.dcos = dcos;
  flank_part(c, g, m);
  return m;
}

// Phi of a charted point with 1 / P_l(sig_o), for the replay's common steps:
// displace<true>(c, g, false, lf) with a uniform branch for a wave whose
// lanes all lie on the cap. Phi inserts area, so t_o = w P_l(sig_o) > t and
// a point on a cap stays on it; the cap-to-cap case (that of almost every
// wave a stroke is far from) needs neither t_o nor the flank terms.
__device__ __forceinline__ Move regenerate(const Chart& c, const StrokeRec& g, const Leaf& lf) {
  Move m;
  const float two_ell = g.two_ell;
  const float q = fwd_area(c.sig, lf, two_ell);
  m.floored = false;
  const float X = fmaf(g.ell, g.ell, kPi * q);
  const float rs = __builtin_amdgcn_rsqf(X);
  const float d = g.ell + X * rs;
  m.sig_o = q * rcp(d);
  m.inv_per_o = 0.5f * rs;
  const float dsig = lf.ar * rcp(fmaf(kPi, c.sig, d));
  const float inv_sig_o = rcp(m.sig_o);
  const bool cap_in = c.th > 0.f;
  const float dth_cc = dsig * g.ell * (kPi - 2.f * c.th) * (c.inv_per * inv_sig_o);
  float dth, th_o, extra;
  const bool all_cap = wave_all(cap_in);
  if (all_cap) {
    dth = dth_cc;
    th_o = c.th + dth;
    extra = 0.f;
  } else {
    const float t_o = c.w * fmaf(kTwoPi, m.sig_o, two_ell);
    const float th_new = fminf(fmaxf(t_o - g.hl, 0.f) * inv_sig_o, kHalfPi);
    const bool cc = cap_in && th_new > 0.f;
    dth = cc ? dth_cc : th_new - c.th;
    th_o = cc ? c.th + dth : th_new;
    const float dt = kTwoPi * c.w * dsig;
    extra = cc ? 0.f : dt - dsig * th_new - c.sig * dth;
  }
  float sd, cdm1;
  if (wave_all(fabsf(dth) < kSmallTurn)) {
    sincosm1_small(dth, sd, cdm1);
  } else {
    sincosm1(dth, sd, cdm1);
  }
  const float dsin = fmaf(c.sn, cdm1, c.cs * sd);
  const float dcos = fmaf(c.cs, cdm1, -(c.sn * sd));
  m.sn_o = c.sn + dsin;
  m.cs_o = c.cs + dcos;
  m.th_o = th_o;
  m.dS = fmaf(dsig, m.sn_o, fmaf(c.sig, dsin, extra));
  m.dH = fmaf(dsig, m.cs_o, c.sig * dcos);
  m.dsig = dsig;
  m.dth = dth;
  m.dsin = dsin;
  m.dcos = dcos;
  m.all_cap = all_cap;
  if (all_cap) {  // both points on the cap: the flank part is l/2 throughout
    m.tf = g.hl;
    m.tf_o = g.hl;
    m.dtf = 0.f;
  } else {
    flank_part(c, g, m);
  }
  return m;
}

// The displacement of the renderer R_D (Sec. "Transfer across transport
// constructions"): K = 16 drop maps (Lu 2012) of radius s, K pi s^2 =
// A_l(r), at the centres of K equal pieces of the segment, laid from its -e
// end; the backward map undoes the last drop first. A drop at c takes the
// point at distance rho from c to distance rho' = sqrt(rho^2 - s^2) on the
// same ray, floored at pi (rho'^2) >= (eps s)^2. The drops work on the FP32
// offset from the stroke centre, rounded once, and accumulate their small
// displacements, which are then added to the FP64 state: rho' / rho - 1 =
// (rho'^2 - rho^2) / (rho^2 (1 + rho' / rho)) has no cancellation.
constexpr int kNumDrops = 16;
// Returns whether a drop's floor bound (the replay then takes x_i from the
// side table: no map inverts a floored drop).
__device__ __forceinline__ bool drops_backward(double& x, double& y, const StrokeRec& g) {
  const float s2 = g.ar * (1.f / (kNumDrops * kPi));
  // eps^2 = floor_c / r^2, so the floor on rho'^2 is floor_c s^2 / (pi r^2)
  const float fl = g.r > 0.f ? g.floor_c * rcp(g.r * g.r) * (s2 * (1.f / kPi)) : 0.f;
  const float ux = g.ell * g.ce, uy = g.ell * g.se;  // the segment, -e end to +e end
  const float d0x = (float)(x - g.mx), d0y = (float)(y - g.my);
  float Dx = 0.f, Dy = 0.f;
  bool any = false;
#pragma unroll
  for (int j = kNumDrops - 1; j >= 0; --j) {
    const float f = ((float)j + 0.5f) * (1.f / kNumDrops) - 0.5f;
    const float px = fmaf(-f, ux, d0x) + Dx, py = fmaf(-f, uy, d0y) + Dy;
    const float rho2 = fmaf(px, px, py * py);
    const float cq = rho2 - s2;
    const bool floored = cq < fl;
    any |= floored;
    const float num = floored ? fl - rho2 : -s2;  // rho'^2 - rho^2
    const float inv = rho2 > 0.f ? rcp(rho2) : 0.f;
    const float k = hw_sqrt((floored ? fl : cq) * inv);
    const float sc = num * inv * rcp(1.f + k);
    Dx = fmaf(px, sc, Dx);
    Dy = fmaf(py, sc, Dy);
  }
  x += (double)Dx;
  y += (double)Dy;
  return any;
}

// The adjoint of R_D's displacement in the replay, with the stroke's
// contributions through the drops (d/d(m_x, m_y, phi, l, r); coverage is
// the caller's). psi_D = b_0 o b_1 o ... o b_15 (b_j the backward map of drop
// j, undone last drop first), so lambda^x_i = J_15^T ... J_0^T lambda^x_{i-1}
// with J_j the Jacobian of b_j at its input: b_0's comes first.
//  * Regenerated lane (the state holds x_{i-1}): drop 0's forward map is
//    applied first, p = c + (q - c) sqrt(1 + s^2 / |q - c|^2), so the points
//    met in that order are exactly the inputs of b_0, b_1, ...; the state
//    ends at x_i.
//  * Loaded lane (the state holds x_i, taken where a floor bound): the input
//    of b_j is recomputed from x_i through b_15 .. b_{j+1}, floors included.
// b_j(p) = c + v k with v = p - c, rho^2 = |v|^2 and k = sqrt(1 - s^2/rho^2),
// or k = sqrt(fl / rho^2) where the floor binds; J = k I + (s^2/(k rho^4)) v v^T
// (floored: k (I - v v^T / rho^2)) is symmetric, and its change
// (J - I) lambda = (k - 1) lambda + coef (v . lambda) v, with
// k - 1 = -(s^2/rho^2) / (1 + k), is formed without cancellation. The drop's
// centre c_j = m + f_j l e receives -(J - I) lambda; s^2 = A_l(r) / (16 pi)
// receives v . lambda dk/d(s^2).
struct DropsAdj {
  float nmx, nmy, gphi, gell, gr;  // nmx, nmy: the centre's, negated (as VjpOut's)
};

__device__ __forceinline__ DropsAdj drops_replay(double& x, double& y, const StrokeRec& g,
                                                 bool loaded, float& lx, float& ly) {
  const float s2 = g.ar * (1.f / (kNumDrops * kPi));
  const float fl = g.r > 0.f ? g.floor_c * rcp(g.r * g.r) * (s2 * (1.f / kPi)) : 0.f;
  const float inv_s2 = s2 > 0.f ? rcp(s2) : 0.f;
  const float ux = g.ell * g.ce, uy = g.ell * g.se;
  const float d0x = (float)(x - g.mx), d0y = (float)(y - g.my);
  float Dx = 0.f, Dy = 0.f;  // regenerated displacement from x_{i-1}
  float Sx = 0.f, Sy = 0.f;  // sum of (J_j - I) lambda_j
  float Fx = 0.f, Fy = 0.f;  // sum of f_j (J_j - I) lambda_j
  float S2 = 0.f;            // adjoint of s^2
  for (int j = 0; j < kNumDrops; ++j) {
    const float f = ((float)j + 0.5f) * (1.f / kNumDrops) - 0.5f;
    float vx, vy, rho2, km1, coef, dk;  // (J - I) lambda = km1 lambda + coef (v.lambda) v; dk/d(s^2)
    if (loaded) {
      float Ex = 0.f, Ey = 0.f;
      for (int jj = kNumDrops - 1; jj > j; --jj) {
        const float fj = ((float)jj + 0.5f) * (1.f / kNumDrops) - 0.5f;
        const float px = fmaf(-fj, ux, d0x) + Ex, py = fmaf(-fj, uy, d0y) + Ey;
        const float r2 = fmaf(px, px, py * py);
        const float cq = r2 - s2;
        const bool fb = cq < fl;
        const float num = fb ? fl - r2 : -s2;
        const float inv = r2 > 0.f ? rcp(r2) : 0.f;
        const float k = hw_sqrt((fb ? fl : cq) * inv);
        const float sc = num * inv * rcp(1.f + k);
        Ex = fmaf(px, sc, Ex);
        Ey = fmaf(py, sc, Ey);
      }
      vx = fmaf(-f, ux, d0x) + Ex;
      vy = fmaf(-f, uy, d0y) + Ey;
      rho2 = fmaf(vx, vx, vy * vy);
      const float inv = rho2 > 0.f ? rcp(rho2) : 0.f;
      if (rho2 - s2 < fl) {  // k = sqrt(fl / rho^2), fl proportional to s^2
        const float k = hw_sqrt(fl * inv);
        km1 = k - 1.f;
        coef = -k * inv;
        dk = 0.5f * k * inv_s2;   // dk/d(s^2) = k / (2 s^2)
      } else {
        const float a = s2 * inv;
        const float k = hw_sqrt(1.f - a);
        const float inv_k = rcp(k);
        km1 = -a * rcp(1.f + k);
        coef = a * inv * inv_k;
        dk = -0.5f * inv * inv_k;  // dk/d(s^2) = -1 / (2 k rho^2)
      }
    } else {
      const float qx = fmaf(-f, ux, d0x) + Dx, qy = fmaf(-f, uy, d0y) + Dy;
      const float q2 = fmaf(qx, qx, qy * qy);
      const float aq = q2 > 0.f ? s2 * rcp(q2) : 0.f;  // s^2 / |q - c|^2
      const float m = hw_sqrt(1.f + aq);
      const float mm1 = aq * rcp(1.f + m);              // m - 1
      Dx = fmaf(qx, mm1, Dx);
      Dy = fmaf(qy, mm1, Dy);
      vx = qx * m;
      vy = qy * m;
      rho2 = q2 + s2;
      const float inv = rcp(rho2);
      const float a = s2 * inv;     // s^2 / rho^2
      const float k = rcp(m);       // sqrt(1 - s^2 / rho^2)
      km1 = -a * rcp(1.f + k);
      coef = a * inv * m;
      dk = -0.5f * inv * m;         // dk/d(s^2) = -1 / (2 k rho^2)
    }
    const float vl = fmaf(vx, lx, vy * ly);
    const float ddx = fmaf(km1, lx, coef * vl * vx);
    const float ddy = fmaf(km1, ly, coef * vl * vy);
    lx += ddx;
    ly += ddy;
    Sx += ddx;
    Sy += ddy;
    Fx = fmaf(f, ddx, Fx);
    Fy = fmaf(f, ddy, Fy);
    S2 = fmaf(vl, dk, S2);
  }
  if (!loaded) {
    x += (double)Dx;
    y += (double)Dy;
  }
  DropsAdj o;
  o.nmx = Sx;
  o.nmy = Sy;
  // c_j = m + f_j l e: dc_j/dphi = f_j l n, dc_j/dl = f_j e
  o.gphi = -g.ell * fmaf(-Fx, g.se, Fy * g.ce);
  // s^2 = A_l(r) / (16 pi): d/dl = 2 r / (16 pi), d/dr = P_l(r) / (16 pi)
  const float s2n = S2 * (1.f / (kNumDrops * kPi));
  o.gell = fmaf(s2n, 2.f * g.r, -fmaf(Fx, g.ce, Fy * g.se));
  o.gr = s2n * g.per_r;
  return o;
}

// Apply a displacement (a, b) along (e, n), unfolded, to the FP64 state.
__device__ __forceinline__ void step_by(double& x, double& y, float a, float b,
                                        const StrokeRec& g) {
  x += (double)fmaf(a, g.ce, -(b * g.se));
  y += (double)fmaf(a, g.se, b * g.ce);
}

// Apply a folded displacement to the FP64 state.
__device__ __forceinline__ void advance(double& x, double& y, const Chart& c, const Move& m,
                                        const StrokeRec& g) {
  step_by(x, y, c.sgs * m.dS, c.sgh * m.dH, g);
}

// psi of a point beyond the stroke's far margin (no floor), for the forward
// traces' far steps, advanced into the FP64 state. The chart needs the
// distance part; th is its cap angle (kAngle: the chart holds the angle
// part too, as the coupled traces chart in full before their vote).
//
// psi moves a point along its leaf towards the segment: a point on a cap
// stays on it when th + dth > 0 with the cap-to-cap increment
//   dth = dsig l (pi - 2 th) / (P_l(sig) sig_o)
// (dth <= 0, so this also rules out the flank, th = 0), and there the new
// point is the old one turned by dth about the cap's centre and scaled by
// sig_o / sig = 1 + k, k = dsig / sig. Both come from one reciprocal each:
//   k = -A / (sig (pi sig + D))  (Eq. back: dsig = -A / (pi sig + D) with
//       D = l + sqrt(l^2 + pi q), q = A_l(sig) - A, the area root's
//       denominator),
//   dth = k l (pi - 2 th) / (P_l(sig) (1 + k)),
// and with the folded offset p = (E, H) from the cap's centre the
// displacement is k (p + r) + r, r = (R(dth) - I) p: no 1 / sigma, no sine
// and cosine of th. Beyond the margin q = A_l(sig) - A has no cancellation
// (sig - r >= 28 wd), so it is formed unfactored. A wave whose lanes all
// lie on the flank takes the flank's own step (S scaled by P_l(sig_o) /
// P_l(sig), H moved by dsig), and any other wave with a lane that reaches
// the flank takes the general map.
template <bool kAngle>
__device__ __forceinline__ void psi_far_advance(double& x, double& y, const Chart& c, float th,
                                                const StrokeRec& g, const Leaf& lf) {
  if constexpr (kAngle) {
    // The chart's own sine, cosine and 1 / P_l(sig) serve the same step
    // (fewer live values where the full chart exists anyway):
    // dS = dsig (sin th + dsin) + sig dsin, dH likewise.
    const float q = back_area(c.sig, lf, g.two_ell);
    const Root rt = area_root(q, g);
    const float dsig = -lf.ar * rcp(fmaf(kPi, c.sig, rt.d));
    const float dth = dsig * g.ell * (kPi - 2.f * c.th) * (c.inv_per * rcp(rt.sig_o));
    if (wave_all(c.th + dth > 0.f)) {
      float sd, cdm1;
      if (wave_all(fabsf(dth) < kSmallTurn)) {
        sincosm1_small(dth, sd, cdm1);
      } else {
        sincosm1(dth, sd, cdm1);
      }
      const float dsin = fmaf(c.sn, cdm1, c.cs * sd);
      const float dcos = fmaf(c.cs, cdm1, -(c.sn * sd));
      step_by(x, y, c.sgs * fmaf(dsig, c.sn + dsin, c.sig * dsin),
              c.sgh * fmaf(dsig, c.cs + dcos, c.sig * dcos), g);
      return;
    }
    advance(x, y, c, displace<false, false>(c, g, true, lf), g);
    return;
  }
  const float q = fmaf(c.sig, fmaf(kPi, c.sig, g.two_ell), -lf.ar);
  const float D = g.ell + hw_sqrt(fmaf(g.ell, g.ell, kPi * q));
  const float k = -lf.ar * rcp(c.sig * fmaf(kPi, c.sig, D));
  const float per = fmaf(kTwoPi, c.sig, g.two_ell);
  const float dth = (k * g.ell) * fmaf(-2.f, th, kPi) * rcp(per * (1.f + k));
  if (__builtin_expect(wave_all(th + dth > 0.f), 1)) {
    float ra, rb;
    if (__builtin_expect(wave_all(fabsf(dth) < kTinyTurn), 1)) {
      turn_increment<true>(dth, c.E, c.H, ra, rb);
    } else {
      turn_increment<false>(dth, c.E, c.H, ra, rb);
    }
    const float dS = fmaf(k, c.E + ra, ra), dH = fmaf(k, c.H + rb, rb);
    step_by(x, y, c.sgs * dS, c.sgh * dH, g);
    return;
  }
  if (__builtin_expect(wave_all(c.E == 0.f), 1)) {
    // every lane on the flank, where sigma = H and t = S: psi moves the
    // point towards the segment by dsig and scales S by P_l(sig_o) /
    // P_l(sig) <= 1 (fixed w), so it stays on the flank
    const float dsig = k * c.sig;
    step_by(x, y, c.sgs * (c.S * ((kTwoPi * dsig) * rcp(per))), c.sgh * dsig, g);
    return;
  }
  Chart cf = c;
  chart_angle<true>(g, cf);
  advance(x, y, cf, displace<false, false>(cf, g, true, lf), g);
}

// Soft coverage alpha = sigmoid((edge - sigma) / wd) with alpha <= 1 - 1e-7
// (edge = the deposit's edge on the point's leaf, r when uniform; wd =
// max(tau r, tau_min) of the stroke), returned with q = 1 - alpha and
// 1 / q = 1 + e^z (exact identities of the logistic function, so no
// cancellation in 1 - alpha).
struct Cover {
  float z, alpha, q, inv_q;
  bool clamped;
};

__device__ __forceinline__ Cover cover(float sig, const StrokeRec& g, float edge) {
  Cover v;
  v.z = (edge - sig) * g.inv_wd;
  float ez = hw_exp(v.z);
  v.clamped = !(ez < kEzMax);
  ez = v.clamped ? kEzMax : ez;
  v.inv_q = 1.f + ez;
  v.q = rcp(v.inv_q);
  v.alpha = ez * v.q;
  return v;
}

// Transmittance T = Tm * 2^Te with Tm in [0.5, 1): no underflow however many
// deposits a trajectory crosses (the paper carries log T for the same reason).
__device__ __forceinline__ void renorm(float& tm, int& te) {
  te += __builtin_amdgcn_frexp_expf(tm);
  tm = __builtin_amdgcn_frexp_mantf(tm);
}
__device__ __forceinline__ float trans_value(float tm, int te) {
  return __builtin_amdgcn_ldexpf(tm, te);
}

// Vector-Jacobian product of one stroke step (Eq. adjstep, Eq. adjparam):
// given lx, ly = lambda^x_{i-1} (the adjoint of the map's output
// psi_i(x_i)) and mu = the adjoint of alpha_i, return lambda^x_i and the
// stroke's contributions d/d(m_x, m_y, phi, l, r).
//
// In the chart of Sec. 4 the map takes (sigma', w) to (rho, w) on the same
// leaf, and the output is the reconstruction at (rho, w). The adjoint of the
// output point is carried by two numbers: the adjoint of rho with w fixed
// (which gives Cb, the adjoint of the area C, through rho = A_l^{-1}(C)) and
// the adjoint t'b of its arclength t' = w P_l(rho); in the folded frame the
// output's adjoint is A_o (sin th', cos th') + t'b (cos th', -sin th').
//
// Far from a stroke the map is close to the identity, and three results are
// small differences of terms of the size of the distance: lambda^x_i -
// lambda^x_{i-1} (minus the centre's contribution), the half-length's
// adjoint, and the angle's. The construction is invariant under rotations
// about m, so d psi / d phi = J (psi(x) - m) - D psi J (x - m) with J the
// quarter turn: two lever arms. Each of the three is therefore written in
// the increments output - input of the chart coordinates (dsig, dth, dsin,
// dcos, dtf), which the map forms without cancellation. For the angle the
// quarter turn is the chart velocity (a, b) per unit angle of the folded
// first-quadrant point, times sgs sgh:
//   a = tf cos th,  b = (tf (th cos th - sin th) - sigma - 2 pi w tf cos th)
//                       / P_l(sigma),
// tf = min(S, l/2), so that, with P0 = P_l(rho), P1 = P_l(sigma'),
//   lambda . d psi / d phi = sgs sgh [Cb (P0 a_o - P1 a_i) + t'b P0 (b_o - b_i)
//                                     + (coverage and coupling terms)],
// and P0 a_o - P1 a_i and P0 (b_o - b_i) expand into the increments.
struct VjpIn {
  float sgs, sgh;        // signs of the signed local coordinates (kept by the map)
  float w;               // centred arclength fraction (common to both points)
  // input point x_i
  float sig;             // sigma' = distance of x_i
  float th, sn, cs;      // cap angle of x_i and its sin / cos (0, 0, 1 on the flank)
  float tf;              // flank part min(S, l/2) of x_i's arclength
  float inv_p1;          // 1 / P_l(sigma') (0 at a drop centre)
  // output point x_{i-1}
  float rho;             // distance of x_{i-1}
  float inv_p0;          // 1 / P_l(rho)
  float th_o, sn_o, cs_o;
  float tf_o;
  // increments x_{i-1} - x_i of the chart coordinates
  float dsig, dth, dsin, dcos, dtf;
  bool floored;          // the floor C >= (eps r)^2 bound at x_i
  // coverage at x_i
  float z, alpha, q;
  bool clamped;
};

struct VjpOut {
  float gx, gy;                          // lambda^x_i
  // stroke contributions; nmx, nmy are the centre's NEGATED (the point's
  // adjoint increment itself: the block sums flip their sign once per stroke)
  float nmx, nmy, gphi, gell, gr;
};

// The inert-mark model R_U (psi = id, Def. inert-mark): the point never
// moves, so a stroke's step depends on its parameters only through the
// coverage z = (r - sigma) / wd at the fixed point. Its contributions, given
// mu = the adjoint of alpha (gx, gy are 0: the point's adjoint is not needed).
__device__ __forceinline__ VjpOut vjp_cover_only(const Chart& c, const StrokeRec& g,
                                                 const Cover& v, float mu) {
  VjpOut o;
  const float zb = v.clamped ? 0.f : mu * v.alpha * v.q;
  const float zw = zb * g.inv_wd;
  o.gr = zw * fmaf(-v.z, g.dwd_dr, 1.f);
  // sigma = sqrt(H^2 + E^2), E = S - l/2 on the caps (sin th = 0 on the flank)
  const float hb = -zw * c.cs, eb = -zw * c.sn;
  const float ssb = c.sgs * eb, shb = c.sgh * hb;
  const float gx = fmaf(ssb, g.ce, -(shb * g.se));
  const float gy = fmaf(ssb, g.se, shb * g.ce);
  o.gx = 0.f;
  o.gy = 0.f;
  o.nmx = gx;
  o.nmy = gy;
  // turning the stroke by dphi changes sigma as turning the point by -dphi
  o.gphi = zw * (c.sgs * c.sgh) * (fminf(c.S, g.hl) * c.cs);
  o.gell = -0.5f * eb;
  return o;
}

// kCover = false drops the coverage terms (a far stroke, alpha = 0 to FP32).
// kCoupled: the leaf's area G = A_l(r) g(w) and edge rl depend on w, l and r
// (the Leaf of the input point): dG = g P_l(r) dr + 2 r g dl + A_l(r) g' dw
// and P_l(rl) drl + 2 rl dl = dG.
template <bool kCover, bool kCoupled = false>
__device__ __forceinline__ VjpOut vjp_step(const VjpIn& v, const StrokeRec& g, float lx,
                                           float ly, float mu, const Leaf& lf) {
  VjpOut o;
  const float two_ell = g.two_ell;
  // output point m + sgs S' e + sgh H' n
  const float ge = fmaf(lx, g.ce, ly * g.se);
  const float gn = fmaf(ly, g.ce, -(lx * g.se));
  const float sbp = v.sgs * ge, hbp = v.sgh * gn;
  const float tpb = fmaf(sbp, v.cs_o, -(hbp * v.sn_o));  // adjoint of t'
  const float ao = fmaf(sbp, v.sn_o, hbp * v.cs_o);
  const float tw = kTwoPi * v.w;
  // rho's adjoint with w fixed (through S', H' and t' = w P_l(rho)), then
  // C's: rho = A_l^{-1}(C), dC = P_l(rho) drho + 2 rho dl
  const float cb = fmaf(tpb, tw - v.th_o, ao) * v.inv_p0;
  const float p0 = fmaf(kTwoPi, v.rho, two_ell);
  const float p1 = fmaf(kTwoPi, v.sig, two_ell);
  const float t1 = kTwoPi * v.dsig;  // P0 - P1
  const float du = v.dsig * v.inv_p1;
  const float u = kTwoPi * du;       // (P0 - P1) / P1
  float zw = 0.f;
  if constexpr (kCover) {
    const float zb = v.clamped ? 0.f : mu * v.alpha * v.q;
    zw = zb * g.inv_wd;  // minus sigma''s adjoint from z = (edge - sigma') / wd
  }
  const float pr = g.per_r;
  float wbx = 0.f, ellx = 0.f, rl_c;
  // C = A_l(sigma') - A_l(r) (coupled: - G), or the floor (eps r)^2
  if constexpr (kCoupled) {
    o.gr = v.floored ? cb * dfloor_dr(g) : -(cb * pr * lf.g);
    wbx = v.floored ? 0.f : -cb * g.ar * lf.dg;
    rl_c = v.floored ? -v.rho : fmaf(-g.r, lf.g, -v.dsig);
    if constexpr (kCover) {
      // coverage z = (rl - sigma') / wd: rl follows G
      const float rlb = zw * lf.inv_per;
      o.gr = fmaf(rlb * pr, lf.g, fmaf(-zw * v.z, g.dwd_dr, o.gr));
      ellx = 2.f * rlb * fmaf(g.r, lf.g, -lf.r);
      wbx = fmaf(rlb * g.ar, lf.dg, wbx);
    }
  } else {
    o.gr = v.floored ? cb * dfloor_dr(g) : -(cb * pr);
    rl_c = v.floored ? -v.rho : -v.dsig - g.r;
    if constexpr (kCover) o.gr = fmaf(zw, fmaf(-v.z, g.dwd_dr, 1.f), o.gr);
  }
  // t's adjoint at the input, (t'b P0 + wbx) / P1, in excess of t'b
  const float dT = kCoupled ? fmaf(wbx, v.inv_p1, tpb * u) : tpb * u;
  const float kap = v.th - tw;
  // sigma''s adjoint at the input (C through P1, w = t / P1, t's cap term,
  // the coverage), in excess of A_o
  const float dsg = fmaf(kap, dT, -fmaf(v.dth, tpb, cb * (v.floored ? p0 : t1))) - zw;
  // lambda^x_i - lambda^x_{i-1} in the folded frame
  const float de = fmaf(dsg, v.sn, fmaf(dT, v.cs, -fmaf(ao, v.dsin, tpb * v.dcos)));
  const float dh = fmaf(dsg, v.cs, fmaf(-dT, v.sn, fmaf(-ao, v.dcos, tpb * v.dsin)));
  // l: through t' and w, the area root, C, and l/2 in the chart and the
  // reconstruction (adjoint dT - de)
  o.gell = fmaf(0.5f, dT - de, fmaf(-2.f * v.w, dT, fmaf(2.f * cb, rl_c, ellx)));
  // phi: Cb (P0 a_o - P1 a_i) + t'b P0 (b_o - b_i) + zw a_i - wbx b_i
  const float Y = v.floored ? p0 * v.tf_o * v.cs_o
                            : fmaf(t1 * v.tf_o, v.cs_o, p1 * fmaf(v.dtf, v.cs_o, v.tf * v.dcos));
  float br = fmaf(v.dth, v.cs_o, -v.dsin);
  br = fmaf(kap, v.dcos, br);
  br = fmaf(-u, fmaf(kap, v.cs, -v.sn), br);
  float X = fmaf(v.tf, br, -two_ell * du);
  X = fmaf(v.dtf, fmaf(v.th_o - tw, v.cs_o, -v.sn_o), X);
  float ang = fmaf(cb, Y, fmaf(tpb, X, zw * v.tf * v.cs));
  if constexpr (kCoupled) {
    ang = fmaf(-wbx * v.inv_p1, fmaf(v.tf, fmaf(kap, v.cs, -v.sn), -v.sig), ang);
  }
  o.gphi = (v.sgs * v.sgh) * ang;
  // unfold the adjoint increment
  const float ssd = v.sgs * de, shd = v.sgh * dh;
  const float dx = fmaf(ssd, g.ce, -(shd * g.se));
  const float dy = fmaf(ssd, g.se, shd * g.ce);
  o.gx = lx + dx;
  o.gy = ly + dy;
  o.nmx = dx;
  o.nmy = dy;
  return o;
}

// The replay's common step when every lane of the wave lies on the stroke's
// cap (E > 0) beyond its far margin, under uniform insertion: regenerates
// x_i = Phi_i(x_{i-1}) into the FP64 state, replaces lambda^x_{i-1} (lx, ly)
// by lambda^x_i and returns the stroke's contributions (the centre's
// negated, phi, l, r) in v.
//
// In polar coordinates about the cap's centre c = m + sgs (l/2) e the chart
// point a = x_{i-1} sits at (sig_a, th_a), and Phi moves it along its leaf
// (fixed fraction w) to b = x_i at (sig_b, th_b), sig_b = sig_a (1 + k),
// th_b = th_a + dth (Eq. fwd; the forward far step's formulas with the
// inserted area's sign flipped). With kap = 2 pi w - th = l (pi - 2 th) /
// P_l(sig) at either point, u = (P_b - P_a) / P_a and v = (P_b - P_a) / P_b,
// psi's vector-Jacobian product (Eq. adjstep) takes lambda_a, whose radial
// and tangential parts at a are ao and tpb, to lambda_b with
//   tangential part at b  tpb P_a / P_b = tpb - tpb v,
//   radial part at b      ao + ao u + tpb (dth (1 - v) + kap_a (u + v)),
// and the area's adjoint is cb = (ao + tpb kap_a) / P_a. Every difference
// between the two points is a product of increments, so nothing cancels.
// The stroke's contributions (Eq. adjparam):
//   centre  lambda_a - lambda_b (translation invariance; returned negated),
//   r       -cb P_l(r),
//   l       2 cb (dsig - r) + tpb v (2 w - 1/2) - (lambda_b - lambda_a) . e_c / 2
//           (the area root, the fraction, and the cap's centre moving by
//           e_c / 2 = sgs e / 2),
//   phi     rotation invariance about m, split at c: the lever c - m turning
//           with the stroke gives -sgs sgh (l/2) dh (dh the folded normal part
//           of lambda_b - lambda_a), and the turn about c gives sgs sgh
//           (sig_b tpb_b - sig_a tpb_a) = sgs sgh (l / pi) tpb v, because
//           sig_a P_b - sig_b P_a = -2 l dsig.
__device__ __forceinline__ void far_cap_step(double& x, double& y, float& lx, float& ly,
                                             const Chart& a, const StrokeRec& g, float (&v)[5]) {
  constexpr float kInvPi = 0.318309886183790671538f;
  const float th = far_theta(a);
  // Phi (Eq. fwd): A_l(sig_b) = A_l(sig_a) + A_l(r); with D = l + sqrt(l^2 +
  // pi q) the root's denominator, dsig = A / (pi sig_a + D), and
  // sqrt(l^2 + pi q) = P_l(sig_b) / 2
  const float q = fmaf(a.sig, fmaf(kPi, a.sig, g.two_ell), g.ar);
  const float X = fmaf(g.ell, g.ell, kPi * q);
  const float rs = __builtin_amdgcn_rsqf(X);  // 2 / P_l(sig_b)
  const float pd = fmaf(kPi, a.sig, fmaf(X, rs, g.ell));
  const float K = rcp(a.sig * pd);
  const float k = g.ar * K;  // dsig / sig_a
  const float dsig = k * a.sig;
  const float inv_sa = pd * K;
  const float Pa = fmaf(kTwoPi, a.sig, g.two_ell);
  const float R = rcp(Pa * (1.f + k));
  const float inv_Pa = (1.f + k) * R;
  const float Ath = g.ell * fmaf(-2.f, th, kPi);
  const float kap = Ath * inv_Pa;  // 2 pi w - th_a
  const float dth = Ath * k * R;   // th_b - th_a = dsig kap_a / sig_b
  float ra, rb;                    // (R(dth) - I) (E, H)
  if (__builtin_expect(wave_all(fabsf(dth) < kTinyTurn), 1)) {
    turn_increment<true>(dth, a.E, a.H, ra, rb);
  } else {
    turn_increment<false>(dth, a.E, a.H, ra, rb);
  }
  step_by(x, y, a.sgs * fmaf(k, a.E + ra, ra), a.sgh * fmaf(k, a.H + rb, rb), g);
  // unit vectors (sin th, cos th) at a and b, and their increments
  const float sn_a = a.E * inv_sa, cs_a = a.H * inv_sa;
  const float dsn = ra * inv_sa, dcs = rb * inv_sa;
  const float sn_b = sn_a + dsn, cs_b = cs_a + dcs;
  // lambda_a in the folded frame at a: radial ao, tangential tpb
  const float ge = fmaf(lx, g.ce, ly * g.se);
  const float gn = fmaf(ly, g.ce, -(lx * g.se));
  const float sbp = a.sgs * ge, hbp = a.sgh * gn;
  const float ao = fmaf(sbp, sn_a, hbp * cs_a);
  const float tpb = fmaf(sbp, cs_a, -(hbp * sn_a));
  const float cb = fmaf(tpb, kap, ao) * inv_Pa;
  const float vb = (kPi * dsig) * rs;        // (P_b - P_a) / P_b
  const float u = (kTwoPi * dsig) * inv_Pa;  // (P_b - P_a) / P_a
  const float dtan = -tpb * vb;
  const float drad = fmaf(tpb, fmaf(kap, u + vb, fmaf(-dth, vb, dth)), ao * u);
  // lambda_b - lambda_a in the folded frame, then unfolded
  const float de = fmaf(drad, sn_b, fmaf(dtan, cs_b, fmaf(ao, dsn, tpb * dcs)));
  const float dh = fmaf(drad, cs_b, fmaf(-dtan, sn_b, fmaf(ao, dcs, -(tpb * dsn))));
  const float ssd = a.sgs * de, shd = a.sgh * dh;
  const float dx = fmaf(ssd, g.ce, -(shd * g.se));
  const float dy = fmaf(ssd, g.se, shd * g.ce);
  lx += dx;
  ly += dy;
  v[0] = dx;
  v[1] = dy;
  v[2] = -(a.sgs * a.sgh) * fmaf(g.ell * kInvPi, dtan, g.hl * dh);
  // 2 w - 1/2 = (th_a + kap_a) / pi - 1/2
  v[3] = fmaf(-0.5f, de, fmaf(-dtan, fmaf(th + kap, kInvPi, -0.5f), 2.f * cb * (dsig - g.r)));
  v[4] = -(cb * g.per_r);
}

// Phi and psi's VJP for a wave whose lanes all lie on the stroke's flank
// (E = 0) beyond its far margin and stay there: about 70% of the far waves
// that are not all on the cap. On the flank sigma = H and the arclength
// from the flank midpoint is t = S, so Phi (Eq. fwd), keeping the fraction
// w = S / P_l(sigma), moves the point away from the segment by dsig and
// scales S by P_b / P_a: the folded displacement is (S u, dsig) with
// u = (P_b - P_a) / P_a. psi's Jacobian at b is triangular (S_a depends on
// S_b and sigma_b, sigma_a on sigma_b alone), and with v = (P_b - P_a) / P_b
// its VJP (Eq. adjstep) takes the folded lambda_a = (lS, lH) to lambda_b:
//   lS_b - lS = -v lS,
//   lH_b - lH = u lH + 2 pi S u (1 / P_b + 1 / P_a) lS.
// With cb = (lH + 2 pi w lS) / P_a, the adjoint of the inserted area, the
// stroke's contributions (Eq. adjparam) are
//   centre  lambda_a - lambda_b (translation invariance; returned negated),
//   r       -cb P_l(r),
//   l       2 cb (dsig - r) + 2 v w lS (the area root, and S_a = w P_l(sig_a)
//           with P_l growing by 2 per unit of l),
//   phi     rotation invariance about m: the change of the cross product of
//           the offset from m with the adjoint, (a - m) x lambda_a -
//           (b - m) x lambda_b, which folded is
//           -sgs sgh (S dlH + dS lH_b - H dlS - dsig lS_b).
// Every difference between the two points is again a product of
// increments. Returns false, with nothing changed, unless every lane stays on
// the flank (S + S u <= l/2; a lane on the cap has S > l/2 and fails too).
__device__ __forceinline__ bool far_flank_step(double& x, double& y, float& lx, float& ly,
                                               const Chart& a, const StrokeRec& g,
                                               float (&v)[5]) {
  constexpr float kInvPi = 0.318309886183790671538f;
  const float q = fmaf(a.sig, fmaf(kPi, a.sig, g.two_ell), g.ar);
  const float X = fmaf(g.ell, g.ell, kPi * q);
  const float rs = __builtin_amdgcn_rsqf(X);  // 2 / P_l(sig_b)
  // 2 l + pi (sig_a + sig_b) = pi sig_a + l + sqrt(l^2 + pi q)
  const float dsig = g.ar * rcp(fmaf(kPi, a.sig, fmaf(X, rs, g.ell)));
  const float inv_Pa = rcp(fmaf(kTwoPi, a.sig, g.two_ell));
  const float hdp = kPi * dsig;        // (P_b - P_a) / 2
  const float u = 2.f * hdp * inv_Pa;  // (P_b - P_a) / P_a
  const float dS = a.S * u;
  if (__builtin_expect(!wave_all(a.S + dS <= g.hl), 0)) return false;
  const float vb = hdp * rs;  // (P_b - P_a) / P_b
  step_by(x, y, a.sgs * dS, a.sgh * dsig, g);
  const float ge = fmaf(lx, g.ce, ly * g.se);
  const float gn = fmaf(ly, g.ce, -(lx * g.se));
  const float lS = a.sgs * ge, lH = a.sgh * gn;
  const float dlS = -vb * lS;
  const float dlH = fmaf(u, lH, (dS * fmaf(kPi, rs, kTwoPi * inv_Pa)) * lS);
  const float ssd = a.sgs * dlS, shd = a.sgh * dlH;
  const float dx = fmaf(ssd, g.ce, -(shd * g.se));
  const float dy = fmaf(ssd, g.se, shd * g.ce);
  lx += dx;
  ly += dy;
  const float w2 = (kTwoPi * a.S) * inv_Pa;  // 2 pi w
  const float cb = fmaf(w2, lS, lH) * inv_Pa;
  v[0] = dx;
  v[1] = dy;
  v[2] = -(a.sgs * a.sgh) *
         (fmaf(a.S, dlH, dS * (lH + dlH)) - fmaf(a.H, dlS, dsig * (lS + dlS)));
  v[3] = fmaf(2.f * cb, dsig - g.r, ((vb * kInvPi) * w2) * lS);
  v[4] = -(cb * g.per_r);
  return true;
}

}  // namespace tbr
