// tbr_oracle.cpp -- FP64 CPU oracle of the deposition-stroke renderer.
//
// TEST INFRASTRUCTURE ONLY. This file is a plain, slow, double-precision
// statement of what the renderer and its gradient compute, written from the
// paper's definitions so that the GPU kernels can be checked against it.
// Only the tests, the smoke check and the benchmark's CPU-baseline leg may
// load it. It shares no code, header, table or constant with the GPU library.
//
// What each part follows (TBR: Transport-Based Rendering with Deposition
// Strokes, arxiv 2609.08722):
//   * footprint, program, pixel chain and compositing: Sec. 3, Eq. (chain),
//     Eq. (render);
//   * distance, Steiner area/perimeter, centred arclength, insertion map and
//     its closed-form inverse: Sec. 4, Eq. (steiner), Eq. (phi),
//     Prop. (centred arclength), Eq. (back), Eq. (fwd);
//   * extension into the footprint and the implemented floor C >= (eps r)^2
//     with its record rule: Sec. 4 "The chain", Sec. 5.2 after the Lemma;
//   * the calibrated variant Phi_g (Sec. 4, "A variant closer to line-source
//     potential flow", Eq. coupling, Eq. profile): the area added along the
//     leaf of centred fraction v is A_l(r) g(v), g(v) = 1 + sum_k c_k
//     cos(4 pi k v), and the deposit is {u <= A_l(r) g(v)};
//   * the two other renderers the paper scores with: the inert-mark model
//     R_U (psi = id, Def. inert-mark) and R_D (Sec. "Transfer across
//     transport constructions"): capsule coverage, but the displacement of
//     stroke i is K = 16 drop maps (Lu 2012) of radius s, K pi s^2 = A_l(r),
//     laid along the segment;
//   * the closed-form compensation baseline (Sec. "Closed-form compensation
//     baseline", Table compensation, Lemma obstruction): each stroke of an
//     inert-mark program is moved to the pre-image of its anchor (or of
//     both segment ends) under every later, already compensated stroke;
//   * soft coverage: Sec. 5.1, Eq. (relax); alpha clamp 1 - 1e-7: Sec. 5.2;
//   * colour model c = softmax(z / tau_c) P: Sec. 5.1;
//   * gradient: plain reverse-mode chain rule over the state of Eq. (state),
//     with every local Jacobian obtained by forward-mode dual numbers pushed
//     through the implemented map (exact differentiation, as the paper does
//     for Table detj). The paper's hand-derived adjoint recurrence is NOT
//     used here; the GPU path implements that one, so the two are
//     independent derivations of the same gradient.
//
// Readings where the paper is silent (documented with the project design):
//   pixel centres ((j+.5)/W, (i+.5)/H), row-major; stroke = centre m, angle
//   phi (direction (cos phi, sin phi)), length L (|L| used, 0 = drop),
//   half-width r; sgn(0) = +1; the closed footprint includes sigma' = r;
//   hard colour = palette[argmax logits]; background = palette[0].

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const double kPi = 3.14159265358979323846264338327950288;
const double kAlphaMax = 1.0 - 1e-7;  // Sec. 5.2: alpha clamped at 1 - 1e-7

// ---------------------------------------------------------------------------
// Forward-mode dual numbers with a fixed set of 7 directions:
// 0,1 = the point (x, y); 2..6 = stroke (m_x, m_y, phi, L, r).
// ---------------------------------------------------------------------------
const int ND = 7;

struct Dual {
  double v;
  double d[ND];
  Dual() : v(0) { std::memset(d, 0, sizeof d); }
  Dual(double a) : v(a) { std::memset(d, 0, sizeof d); }  // NOLINT: implicit
};

inline double val(double a) { return a; }
inline double val(const Dual& a) { return a.v; }

inline Dual operator+(const Dual& a, const Dual& b) {
  Dual r(a.v + b.v);
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
inline Dual operator-(const Dual& a, const Dual& b) {
  Dual r(a.v - b.v);
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
inline Dual operator-(const Dual& a) {
  Dual r(-a.v);
  for (int k = 0; k < ND; ++k) r.d[k] = -a.d[k];
  return r;
}
inline Dual operator*(const Dual& a, const Dual& b) {
  Dual r(a.v * b.v);
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  for (int k = 0; k < ND; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
  return r;
}
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) { return a * Dual(b); }
inline Dual operator*(double a, const Dual& b) { return Dual(a) * b; }
inline Dual operator/(const Dual& a, double b) { return a / Dual(b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }

inline Dual chain(const Dual& a, double f, double df) {
  Dual r(f);
  for (int k = 0; k < ND; ++k) r.d[k] = df * a.d[k];
  return r;
}
inline double m_sqrt(double a) { return std::sqrt(a); }
inline Dual m_sqrt(const Dual& a) {
  double f = std::sqrt(a.v);
  return chain(a, f, 0.5 / f);
}
inline double m_sin(double a) { return std::sin(a); }
inline Dual m_sin(const Dual& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
inline double m_cos(double a) { return std::cos(a); }
inline Dual m_cos(const Dual& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
inline double m_exp(double a) { return std::exp(a); }
inline Dual m_exp(const Dual& a) {
  double f = std::exp(a.v);
  return chain(a, f, f);
}
inline double m_atan2(double y, double x) { return std::atan2(y, x); }
inline Dual m_atan2(const Dual& y, const Dual& x) {
  Dual r(std::atan2(y.v, x.v));
  double q = x.v * x.v + y.v * y.v;
  for (int k = 0; k < ND; ++k) r.d[k] = (x.v * y.d[k] - y.v * x.d[k]) / q;
  return r;
}

// ---------------------------------------------------------------------------
// One stroke g = (m, phi, L, r) in a scalar type T.
// ---------------------------------------------------------------------------
template <class T>
struct Stroke {
  T mx, my, phi, L, r;
  const double* coup = nullptr;  // c_1..c_3 of Eq. profile (constants), or none: g = 1
};

// Chart coordinates of a point with respect to a stroke (Sec. 4):
// sigma = distance to the segment, w = centred arclength fraction folded into
// one quadrant, and the two reflection signs that unfold it again.
template <class T>
struct Chart {
  int sgn_s, sgn_h;  // side of the perpendicular bisector / of the axis
  T ell, hl;         // segment length |L| and half-length
  T ce, se;          // direction e = (cos phi, sin phi)
  T sigma;           // distance to the segment
  T w;               // arclength fraction from the flank midpoint, in [0, 1/4]
};

// Steiner perimeter of the parallel set, Eq. (steiner): P = 2 l + 2 pi sigma.
template <class T>
T perimeter(const T& ell, const T& sigma) {
  return 2.0 * ell + 2.0 * kPi * sigma;
}

template <class T>
Chart<T> chart(const T& x, const T& y, const Stroke<T>& g) {
  Chart<T> c;
  c.ell = val(g.L) < 0 ? -g.L : g.L;  // d|L|/dL := +1 at L = 0
  c.hl = 0.5 * c.ell;
  c.ce = m_cos(g.phi);
  c.se = m_sin(g.phi);
  T dx = x - g.mx, dy = y - g.my;
  T s = dx * c.ce + dy * c.se;   // coordinate along the segment
  T h = -dx * c.se + dy * c.ce;  // coordinate across it
  c.sgn_s = val(s) < 0 ? -1 : 1;
  c.sgn_h = val(h) < 0 ? -1 : 1;
  T S = c.sgn_s < 0 ? -s : s;
  T H = c.sgn_h < 0 ? -h : h;
  bool on_cap = val(S) > val(c.hl);
  T E = on_cap ? S - c.hl : T(0.0);  // overshoot past the segment end
  c.sigma = m_sqrt(H * H + E * E);
  // Arclength from the flank midpoint along the stadium {dist = sigma}:
  // straight flank up to l/2, then the cap arc sigma * angle from the normal.
  T t = (on_cap ? c.hl : S) + c.sigma * m_atan2(E, H);
  T P = perimeter(c.ell, c.sigma);
  c.w = val(P) > 0 ? t / P : T(0.0);  // drop centre (measure zero): w := 0
  return c;
}

// The point of the parallel curve at distance rho whose centred arclength
// fraction is w, unfolded into the quadrant given by the chart's signs.
template <class T>
void reconstruct(const Chart<T>& c, const Stroke<T>& g, const T& rho, T& ox, T& oy) {
  T t = c.w * perimeter(c.ell, rho);
  T Sp, Hp;
  if (val(t) <= val(c.hl)) {  // on the flank (always so when rho = 0)
    Sp = t;
    Hp = rho;
  } else {  // on the cap: arc angle measured from the normal direction
    T th = (t - c.hl) / rho;
    Sp = c.hl + rho * m_sin(th);
    Hp = rho * m_cos(th);
  }
  T a = double(c.sgn_s) * Sp, b = double(c.sgn_h) * Hp;
  ox = g.mx + a * c.ce - b * c.se;
  oy = g.my + a * c.se + b * c.ce;
}

// Steiner area of the parallel set, Eq. (steiner): A = 2 l sigma + pi sigma^2.
template <class T>
T steiner_area(const T& ell, const T& sigma) {
  return (2.0 * ell + kPi * sigma) * sigma;
}

// Eq. (profile): g(v) = 1 + sum_{k=1..3} c_k cos(4 pi k v).
template <class T>
T profile(const T& v, const double* c) {
  T g = T(1.0);
  for (int k = 1; k <= 3; ++k) g = g + c[k - 1] * m_cos(4.0 * kPi * double(k) * v);
  return g;
}

// Area the stroke inserts along the leaf of the charted point: A_l(r), or
// A_l(r) g(v) under the calibrated coupling (Eq. coupling).
template <class T>
T leaf_area(const Chart<T>& c, const Stroke<T>& g) {
  T A = steiner_area(c.ell, g.r);
  return g.coup ? A * profile(c.w, g.coup) : A;
}

// Distance at which the deposit ends on the point's leaf: r, or the root of
// A_l(rho) = A_l(r) g(v) (the deposit {u <= A_l(r) g(v)} of Eq. coupling).
template <class T>
T leaf_edge(const Chart<T>& c, const Stroke<T>& g) {
  if (!g.coup) return g.r;
  T G = leaf_area(c, g);
  return G / (c.ell + m_sqrt(c.ell * c.ell + kPi * G));
}

// psi: backward material map of one stroke, Eq. (back), with the implemented
// floor C >= (eps r)^2 (eps = 0 gives the ideal clamp C -> 0). Returns
// whether the floor bound (the record rule C < (eps r)^2).
template <class T>
bool psi(const T& x, const T& y, const Stroke<T>& g, double eps, T& ox, T& oy,
         T* sigma_out = nullptr, T* edge_out = nullptr) {
  Chart<T> c = chart(x, y, g);
  if (sigma_out) *sigma_out = c.sigma;
  if (edge_out) *edge_out = leaf_edge(c, g);
  // C = A_l(sigma') - A_l(r) in factored form; under the coupling the
  // subtracted area is A_l(r) g(v), written as the plain difference.
  T C = g.coup ? steiner_area(c.ell, c.sigma) - leaf_area(c, g)
               : (c.sigma - g.r) * (2.0 * c.ell + kPi * (c.sigma + g.r));
  T fl = (eps * g.r) * (eps * g.r);
  bool rec = val(C) < val(fl);
  if (rec) C = fl;
  T rho = val(C) > 0 ? C / (c.ell + m_sqrt(c.ell * c.ell + kPi * C)) : T(0.0);
  reconstruct(c, g, rho, ox, oy);
  return rec;
}

// Phi: exterior forward map, Eq. (fwd): the parallel curve enclosing
// A_l(r) more area, same centred arclength fraction.
template <class T>
void phi_map(const T& x, const T& y, const Stroke<T>& g, T& ox, T& oy) {
  Chart<T> c = chart(x, y, g);
  T B = g.coup ? steiner_area(c.ell, c.sigma) + leaf_area(c, g)
               : 2.0 * c.ell * (c.sigma + g.r) + kPi * (c.sigma * c.sigma + g.r * g.r);
  T sp = B / (c.ell + m_sqrt(c.ell * c.ell + kPi * B));
  reconstruct(c, g, sp, ox, oy);
}

// R_D's displacement. The drops sit at the centres of K equal pieces of the
// segment and are laid in one sweep from its -e end to its +e end, so the
// forward map inserts drop 0 first and the backward map undoes drop K-1
// first. A drop of radius s at c moves a point at distance rho from c to
// distance sqrt(rho^2 + s^2) on the same ray (forward) or back to
// sqrt(rho^2 - s^2), floored at pi (rho^2 - s^2) >= (eps s)^2 (the capsule's
// implemented floor, for the drop's own radius). Returns whether a floor
// bound.
const int kDropsK = 16;

template <class T>
void drop_centre(const Stroke<T>& g, int j, T& cx, T& cy, T& s2) {
  T ell = val(g.L) < 0 ? -g.L : g.L;
  double f = (j + 0.5) / kDropsK - 0.5;  // along e, in units of l
  cx = g.mx + f * ell * m_cos(g.phi);
  cy = g.my + f * ell * m_sin(g.phi);
  s2 = steiner_area(ell, g.r) / (kDropsK * kPi);
}

template <class T>
bool psi_drops(const T& x, const T& y, const Stroke<T>& g, double eps, T& ox, T& oy) {
  T px = x, py = y;
  bool rec = false;
  for (int j = kDropsK - 1; j >= 0; --j) {
    T cx, cy, s2;
    drop_centre(g, j, cx, cy, s2);
    T dx = px - cx, dy = py - cy;
    T rho2 = dx * dx + dy * dy;
    T C = kPi * (rho2 - s2);
    T fl = eps * eps * s2;  // (eps s)^2, an area like C
    if (val(C) < val(fl)) {
      C = fl;
      rec = true;
    }
    if (val(rho2) > 0) {
      T k = m_sqrt(C / (kPi * rho2));
      px = cx + dx * k;
      py = cy + dy * k;
    }
  }
  ox = px;
  oy = py;
  return rec;
}

template <class T>
void phi_drops(const T& x, const T& y, const Stroke<T>& g, T& ox, T& oy) {
  T px = x, py = y;
  for (int j = 0; j < kDropsK; ++j) {
    T cx, cy, s2;
    drop_centre(g, j, cx, cy, s2);
    T dx = px - cx, dy = py - cy;
    T rho2 = dx * dx + dy * dy;
    if (val(rho2) > 0) {
      T k = m_sqrt((rho2 + s2) / rho2);
      px = cx + dx * k;
      py = cy + dy * k;
    }
  }
  ox = px;
  oy = py;
}

// Soft coverage, Eq. (relax), clamped at 1 - 1e-7: the signed distance from
// the deposit's edge on the point's leaf (r, or the coupled leaf_edge) over
// the width max(tau r, tau_min) of the stroke's half-width r.
template <class T>
T soft_alpha(const T& sigma, const T& edge, const T& r, double tau, double tau_min) {
  T wd = val(r) * tau > tau_min ? tau * r : T(tau_min);
  T z = (edge - sigma) / wd;
  // The logistic function, written so that the exponential never overflows
  // (far pixels reach z < -709): e^z / (1 + e^z) for z < 0.
  T a;
  if (val(z) >= 0) {
    a = 1.0 / (1.0 + m_exp(-z));
  } else {
    T ez = m_exp(z);
    a = ez / (1.0 + ez);
  }
  if (val(a) > kAlphaMax) a = T(kAlphaMax);
  return a;
}

// ---------------------------------------------------------------------------
// Program, options, colours.
// ---------------------------------------------------------------------------
struct Program {
  int32_t n, k;
  const double *cx, *cy, *angle, *length, *half_width, *logits, *palette;
};

struct Opts {
  int32_t width, height;
  double tau, tau_min, tau_c, eps;
  int32_t transport;       // 1 = capsule renderer R_A, 0 = inert-mark R_U, 2 = R_D (16 drops)
  const double* coupling;  // [N][3] c_1..c_3 per stroke (Eq. profile), or NULL: g = 1
};

Stroke<double> stroke_at(const Program& p, const Opts& o, int i) {
  Stroke<double> g{p.cx[i], p.cy[i], p.angle[i], p.length[i], p.half_width[i]};
  g.coup = o.coupling ? o.coupling + 3 * size_t(i) : nullptr;
  return g;
}

// The displacement the renderer applies after stroke g (psi_i of Eq. chain):
// the capsule map (or its calibrated coupling), the identity (R_U) or the
// sixteen drops (R_D). Returns whether a floor bound.
template <class T>
bool transport_step(const Opts& o, const T& x, const T& y, const Stroke<T>& g, T& ox, T& oy) {
  if (o.transport == 2) return psi_drops(x, y, g, o.eps, ox, oy);
  if (o.transport == 1) return psi(x, y, g, o.eps, ox, oy);
  ox = x;
  oy = y;
  return false;
}

int argmax_row(const double* z, int k) {
  int b = 0;
  for (int j = 1; j < k; ++j)
    if (z[j] > z[b]) b = j;  // ties to the lowest index
  return b;
}

// Colour of every stroke, c_i = softmax(z_i / tau_c) P; tau_c = 0 is the
// argmax (hard) limit. Also returns the weights s_i for the chain rule.
void stroke_colours(const Program& p, double tau_c, std::vector<double>& col,
                    std::vector<double>& wts) {
  col.assign(size_t(p.n) * 3, 0.0);
  wts.assign(size_t(p.n) * p.k, 0.0);
  for (int i = 0; i < p.n; ++i) {
    const double* z = p.logits + size_t(i) * p.k;
    double* s = &wts[size_t(i) * p.k];
    if (tau_c > 0) {
      double zmax = z[0];
      for (int j = 1; j < p.k; ++j) zmax = std::max(zmax, z[j]);
      double tot = 0;
      for (int j = 0; j < p.k; ++j) tot += (s[j] = std::exp((z[j] - zmax) / tau_c));
      for (int j = 0; j < p.k; ++j) s[j] /= tot;
    } else {
      s[argmax_row(z, p.k)] = 1.0;
    }
    for (int j = 0; j < p.k; ++j)
      for (int ch = 0; ch < 3; ++ch) col[size_t(i) * 3 + ch] += s[j] * p.palette[j * 3 + ch];
  }
}

void pixel_centre(const Opts& o, int64_t pix, double& x, double& y) {
  int64_t row = pix / o.width, colm = pix % o.width;
  x = (double(colm) + 0.5) / o.width;
  y = (double(row) + 0.5) / o.height;
}

int64_t pixel_of(int64_t j, const int64_t* pix) { return pix ? pix[j] : j; }

}  // namespace

// ---------------------------------------------------------------------------
// C entry points (ctypes).
// ---------------------------------------------------------------------------
extern "C" {

typedef struct {
  int32_t n, k;
  const double *cx, *cy, *angle, *length, *half_width, *logits, *palette;
} orc_program;

typedef struct {
  int32_t width, height;
  double tau, tau_min, tau_c, eps;
  int32_t transport;
  const double* coupling;
} orc_opts;

static Program to_prog(const orc_program* p) {
  return {p->n, p->k, p->cx, p->cy, p->angle, p->length, p->half_width, p->logits, p->palette};
}
static Opts to_opts(const orc_opts* o) {
  return {o->width, o->height, o->tau, o->tau_min, o->tau_c, o->eps, o->transport, o->coupling};
}

// psi for a batch of points; stroke = (m_x, m_y, phi, L, r).
// coup: c_1..c_3 of the calibrated coupling, or NULL (uniform insertion).
void orc_psi(const double* stroke, double eps, int64_t n, const double* pts, double* out,
             int32_t* rec, const double* coup) {
  Stroke<double> g{stroke[0], stroke[1], stroke[2], stroke[3], stroke[4]};
  g.coup = coup;
  for (int64_t j = 0; j < n; ++j) {
    bool b = psi(pts[2 * j], pts[2 * j + 1], g, eps, out[2 * j], out[2 * j + 1]);
    if (rec) rec[j] = b ? 1 : 0;
  }
}

void orc_phi(const double* stroke, int64_t n, const double* pts, double* out,
             const double* coup) {
  Stroke<double> g{stroke[0], stroke[1], stroke[2], stroke[3], stroke[4]};
  g.coup = coup;
  for (int64_t j = 0; j < n; ++j) phi_map(pts[2 * j], pts[2 * j + 1], g, out[2 * j], out[2 * j + 1]);
}

// R_D's backward / forward displacement of one stroke at a batch of points.
void orc_psi_drops(const double* stroke, double eps, int64_t n, const double* pts, double* out,
                   int32_t* rec) {
  Stroke<double> g{stroke[0], stroke[1], stroke[2], stroke[3], stroke[4]};
  for (int64_t j = 0; j < n; ++j) {
    bool b = psi_drops(pts[2 * j], pts[2 * j + 1], g, eps, out[2 * j], out[2 * j + 1]);
    if (rec) rec[j] = b ? 1 : 0;
  }
}

void orc_phi_drops(const double* stroke, int64_t n, const double* pts, double* out) {
  Stroke<double> g{stroke[0], stroke[1], stroke[2], stroke[3], stroke[4]};
  for (int64_t j = 0; j < n; ++j)
    phi_drops(pts[2 * j], pts[2 * j + 1], g, out[2 * j], out[2 * j + 1]);
}

// Distance to the segment, centred arclength fraction and the deposit's
// edge on the point's leaf (diagnostics; edge may be NULL).
void orc_chart(const double* stroke, int64_t n, const double* pts, double* sigma, double* w,
               double* edge, const double* coup) {
  Stroke<double> g{stroke[0], stroke[1], stroke[2], stroke[3], stroke[4]};
  g.coup = coup;
  for (int64_t j = 0; j < n; ++j) {
    Chart<double> c = chart(pts[2 * j], pts[2 * j + 1], g);
    sigma[j] = c.sigma;
    w[j] = c.w;
    if (edge) edge[j] = leaf_edge(c, g);
  }
}

// Exact Jacobians (dual numbers) of psi (which = 0), Phi (1), or R_D's
// backward (2) / forward (3) displacement:
// jac[j] is 2 x 7, row-major, columns (x, y, m_x, m_y, phi, L, r).
void orc_map_jacobian(int which, const double* stroke, double eps, int64_t n, const double* pts,
                      double* jac, const double* coup) {
  for (int64_t j = 0; j < n; ++j) {
    Dual x(pts[2 * j]), y(pts[2 * j + 1]);
    x.d[0] = 1;
    y.d[1] = 1;
    Stroke<Dual> g;
    g.mx = Dual(stroke[0]);
    g.mx.d[2] = 1;
    g.my = Dual(stroke[1]);
    g.my.d[3] = 1;
    g.phi = Dual(stroke[2]);
    g.phi.d[4] = 1;
    g.L = Dual(stroke[3]);
    g.L.d[5] = 1;
    g.r = Dual(stroke[4]);
    g.r.d[6] = 1;
    g.coup = coup;
    Dual ox, oy;
    if (which == 0)
      psi(x, y, g, eps, ox, oy);
    else if (which == 1)
      phi_map(x, y, g, ox, oy);
    else if (which == 2)
      psi_drops(x, y, g, eps, ox, oy);
    else
      phi_drops(x, y, g, ox, oy);
    for (int k = 0; k < ND; ++k) {
      jac[j * 14 + k] = ox.d[k];
      jac[j * 14 + 7 + k] = oy.d[k];
    }
  }
}

// Forward render at pixel centres (all pixels if pix == NULL, else the
// n_pix listed flat indices). Outputs may be NULL.
//   rgb_soft  [n_pix*3]  soft composite, Eq. (render) with Eq. (relax)
//   rgb_hard  [n_pix*3]  hard composite (first footprint hit going N -> 1)
//   label     [n_pix]    palette index of the hard colour (0 = background)
//   owner     [n_pix]    stroke index (0-based) owning the pixel, -1 if none
//   dmin      [n_pix]    min |sigma'_i - r_i| over the hard trace's visited steps
//   n_rec     [n_pix]    soft trace: number of steps where the floor binds
int orc_render(const orc_program* prog, const orc_opts* opts, int64_t n_pix, const int64_t* pix,
               double* rgb_soft, double* rgb_hard, int32_t* label, int32_t* owner, double* dmin,
               int32_t* n_rec) {
  Program p = to_prog(prog);
  Opts o = to_opts(opts);
  if (!pix) n_pix = int64_t(o.width) * o.height;
  std::vector<double> col, wts;
  stroke_colours(p, o.tau_c, col, wts);
  const double* bg = p.palette;  // c_0 = palette[0]

#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t j = 0; j < n_pix; ++j) {
    double x0, y0;
    pixel_centre(o, pixel_of(j, pix), x0, y0);
    if (rgb_soft || n_rec) {
      double x = x0, y = y0, C[3] = {0, 0, 0}, T = 1.0;
      int32_t nr = 0;
      for (int i = p.n - 1; i >= 0; --i) {
        Stroke<double> g = stroke_at(p, o, i);
        double ox, oy, sig, edge;
        bool rec = psi(x, y, g, o.eps, ox, oy, &sig, &edge);
        double a = soft_alpha(sig, edge, g.r, o.tau, o.tau_min);
        for (int ch = 0; ch < 3; ++ch) C[ch] += T * a * col[size_t(i) * 3 + ch];
        T *= (1.0 - a);
        if (o.transport == 2) rec = psi_drops(x, y, g, o.eps, ox, oy);
        nr += rec ? 1 : 0;
        if (o.transport) {
          x = ox;
          y = oy;
        }
      }
      if (rgb_soft)
        for (int ch = 0; ch < 3; ++ch) rgb_soft[j * 3 + ch] = C[ch] + T * bg[ch];
      if (n_rec) n_rec[j] = nr;
    }
    if (rgb_hard || label || owner || dmin) {
      double x = x0, y = y0, dm = INFINITY;
      int own = -1;
      for (int i = p.n - 1; i >= 0; --i) {
        Stroke<double> g = stroke_at(p, o, i);
        Chart<double> c = chart(x, y, g);
        const double edge = leaf_edge(c, g);
        dm = std::min(dm, std::fabs(c.sigma - edge));
        if (c.sigma <= edge) {  // closed footprint
          own = i;
          break;
        }
        double ox, oy;
        transport_step(o, x, y, g, ox, oy);
        x = ox;
        y = oy;
      }
      int lab = own >= 0 ? argmax_row(p.logits + size_t(own) * p.k, p.k) : 0;
      if (rgb_hard)
        for (int ch = 0; ch < 3; ++ch) rgb_hard[j * 3 + ch] = p.palette[lab * 3 + ch];
      if (label) label[j] = lab;
      if (owner) owner[j] = own;
      if (dmin) dmin[j] = dm;
    }
  }
  return 0;
}

// Gradient of sum_x grad_rgb(x) . R(x) for the soft render (i.e. the
// vector-Jacobian product with an upstream gradient grad_rgb [n_pix*3]).
// Outputs (all overwritten):
//   grad_geom    [5*N]  SoA: d/d m_x | m_y | phi | L | r
//   grad_colour  [N*3]  d/d c_i
//   grad_logits  [N*K]  through c_i = softmax(z_i/tau_c) P (0 if tau_c = 0)
//   grad_palette [K*3]  through every c_i and the background c_0 = P[0]
// Method: per pixel, store the FP64 trajectory x_N..x_0, T_N..T_0; then walk
// i = 1..N applying the transpose of each step's Jacobian to the state
// adjoint (x, C, T). Local Jacobians of psi_i and alpha_i come from dual
// numbers. Pixel contributions are summed in fixed 256-pixel blocks, and the
// blocks in order, so the result does not depend on the thread count.
int orc_backward(const orc_program* prog, const orc_opts* opts, int64_t n_pix, const int64_t* pix,
                 const double* grad_rgb, double* grad_geom, double* grad_colour,
                 double* grad_logits, double* grad_palette) {
  Program p = to_prog(prog);
  Opts o = to_opts(opts);
  if (!pix) n_pix = int64_t(o.width) * o.height;
  const int N = p.n;
  std::vector<double> col, wts;
  stroke_colours(p, o.tau_c, col, wts);
  const int64_t kBlock = 256;
  const int64_t nblk = (n_pix + kBlock - 1) / kBlock;
  const int W8 = 8;  // per stroke: 5 geometric + 3 colour
  std::vector<double> part(size_t(nblk) * (size_t(N) * W8 + 3), 0.0);

#pragma omp parallel
  {
    std::vector<double> xs(size_t(N + 1) * 2), Ts(N + 1);
#pragma omp for schedule(dynamic, 1)
    for (int64_t b = 0; b < nblk; ++b) {
      double* acc = &part[size_t(b) * (size_t(N) * W8 + 3)];
      for (int64_t j = b * kBlock; j < std::min(n_pix, (b + 1) * kBlock); ++j) {
        const double* gR = grad_rgb + j * 3;
        if (gR[0] == 0 && gR[1] == 0 && gR[2] == 0) continue;
        double x, y;
        pixel_centre(o, pixel_of(j, pix), x, y);
        // Forward: state index i holds x_i (input of psi_i) and T_i.
        double T = 1.0;
        xs[2 * N] = x;
        xs[2 * N + 1] = y;
        Ts[N] = 1.0;
        for (int i = N; i >= 1; --i) {
          Stroke<double> g = stroke_at(p, o, i - 1);
          double ox, oy, sig, edge;
          psi(x, y, g, o.eps, ox, oy, &sig, &edge);
          double a = soft_alpha(sig, edge, g.r, o.tau, o.tau_min);
          T *= (1.0 - a);
          if (o.transport == 2) psi_drops(x, y, g, o.eps, ox, oy);
          if (o.transport) {
            x = ox;
            y = oy;
          }
          xs[2 * (i - 1)] = x;
          xs[2 * (i - 1) + 1] = y;
          Ts[i - 1] = T;
        }
        // R = C_0 + T_0 c_0: seed the state adjoint.
        double lC[3] = {gR[0], gR[1], gR[2]};
        double lT = lC[0] * p.palette[0] + lC[1] * p.palette[1] + lC[2] * p.palette[2];
        double lx[2] = {0, 0};
        for (int ch = 0; ch < 3; ++ch) acc[size_t(N) * W8 + ch] += lC[ch] * Ts[0];
        // Reverse over steps i = 1..N (s_i -> s_{i-1}).
        for (int i = 1; i <= N; ++i) {
          const int si = i - 1;
          Stroke<double> gd = stroke_at(p, o, si);
          Dual X(xs[2 * i]), Y(xs[2 * i + 1]);
          X.d[0] = 1;
          Y.d[1] = 1;
          Stroke<Dual> g;
          g.mx = Dual(gd.mx);
          g.mx.d[2] = 1;
          g.my = Dual(gd.my);
          g.my.d[3] = 1;
          g.phi = Dual(gd.phi);
          g.phi.d[4] = 1;
          g.L = Dual(gd.L);
          g.L.d[5] = 1;
          g.r = Dual(gd.r);
          g.r.d[6] = 1;
          g.coup = gd.coup;
          Dual ox, oy, sig, edge;
          psi(X, Y, g, o.eps, ox, oy, &sig, &edge);
          Dual a = soft_alpha(sig, edge, g.r, o.tau, o.tau_min);
          if (o.transport == 2) psi_drops(X, Y, g, o.eps, ox, oy);
          if (!o.transport) {  // psi = id
            ox = X;
            oy = Y;
          }
          const double Ti = Ts[i];
          const double* ci = &col[size_t(si) * 3];
          // Local Jacobian of s_{i-1} = f(s_i, theta_i, c_i):
          //   C' = C + T a c,  T' = T (1 - a),  x' = psi(x).
          // Adjoint of alpha:
          double la = Ti * (lC[0] * ci[0] + lC[1] * ci[1] + lC[2] * ci[2]) - Ti * lT;
          // Parameter gradients (columns 2..6 of the duals).
          for (int q = 0; q < 5; ++q) {
            acc[size_t(si) * W8 + q] +=
                lx[0] * ox.d[2 + q] + lx[1] * oy.d[2 + q] + la * a.d[2 + q];
          }
          for (int ch = 0; ch < 3; ++ch) acc[size_t(si) * W8 + 5 + ch] += lC[ch] * Ti * a.v;
          // State adjoint s_{i-1} -> s_i.
          double nx = lx[0] * ox.d[0] + lx[1] * oy.d[0] + la * a.d[0];
          double ny = lx[0] * ox.d[1] + lx[1] * oy.d[1] + la * a.d[1];
          double nT = lT * (1.0 - a.v) + a.v * (lC[0] * ci[0] + lC[1] * ci[1] + lC[2] * ci[2]);
          lx[0] = nx;
          lx[1] = ny;
          lT = nT;
        }
      }
    }
  }
  // Fixed-order block sum.
  std::vector<double> tot(size_t(N) * W8 + 3, 0.0);
  for (int64_t b = 0; b < nblk; ++b)
    for (size_t q = 0; q < tot.size(); ++q) tot[q] += part[size_t(b) * tot.size() + q];
  for (int i = 0; i < N; ++i) {
    for (int q = 0; q < 5; ++q) grad_geom[size_t(q) * N + i] = tot[size_t(i) * W8 + q];
    for (int ch = 0; ch < 3; ++ch) grad_colour[size_t(i) * 3 + ch] = tot[size_t(i) * W8 + 5 + ch];
  }
  // Chain through c_i = sum_k s_ik P_k and s_i = softmax(z_i / tau_c).
  for (int q = 0; q < p.k * 3; ++q) grad_palette[q] = 0.0;
  for (int ch = 0; ch < 3; ++ch) grad_palette[ch] += tot[size_t(N) * W8 + ch];  // background
  for (int i = 0; i < N; ++i) {
    const double* g = &grad_colour[size_t(i) * 3];
    const double* s = &wts[size_t(i) * p.k];
    const double* c = &col[size_t(i) * 3];
    double gc = g[0] * c[0] + g[1] * c[1] + g[2] * c[2];
    for (int k = 0; k < p.k; ++k) {
      const double* Pk = p.palette + k * 3;
      double gp = g[0] * Pk[0] + g[1] * Pk[1] + g[2] * Pk[2];
      grad_logits[size_t(i) * p.k + k] = o.tau_c > 0 ? s[k] * (gp - gc) / o.tau_c : 0.0;
      for (int ch = 0; ch < 3; ++ch) grad_palette[k * 3 + ch] += s[k] * g[ch];
    }
  }
  return 0;
}

// Hard trace at arbitrary points of the final plane (not only pixel
// centres): owner [n] = 0-based index of the first footprint hit going
// N -> 1, or -1.
void orc_hard_points(const orc_program* prog, const orc_opts* opts, int64_t n, const double* pts,
                     int32_t* owner) {
  Program p = to_prog(prog);
  Opts o = to_opts(opts);
#pragma omp parallel for schedule(static, 4096)
  for (int64_t j = 0; j < n; ++j) {
    double x = pts[2 * j], y = pts[2 * j + 1];
    int own = -1;
    for (int i = p.n - 1; i >= 0; --i) {
      Stroke<double> g = stroke_at(p, o, i);
      Chart<double> c = chart(x, y, g);
      if (c.sigma <= leaf_edge(c, g)) {
        own = i;
        break;
      }
      double ox, oy;
      transport_step(o, x, y, g, ox, oy);
      x = ox;
      y = oy;
    }
    owner[j] = own;
  }
}

// Closed-form compensation of an inert-mark program (Sec. "Closed-form
// compensation baseline"), written as its definition: for i = N-1 .. 0,
// stroke i's anchor a_i = m_i - (L_i / 2) e_i (endpoint = 1: also its end
// m_i + (L_i / 2) e_i) is pre-imaged through the later strokes j = N-1 down
// to i+1, in their compensated geometry, by the backward maps psi_j with the
// floor (eps r_j)^2. A step is blocked when the point lies in K_j (sigma' <=
// r_j): no pre-image exists there (Lemma obstruction); it is then clamped by
// the extended psi_j, or left out (skip = 1). The anchor variant keeps the
// offset L e; the endpoint variant takes the segment between the two
// pre-images (its angle is kept if they coincide). Radii, logits and palette
// are unchanged. Outputs [N]: cx, cy, angle, length of the compensated
// program, the number of blocked steps of each stroke, and (may be NULL)
// dmin, the smallest |sigma' - r_j| its points met on the way, and smin, the
// smallest sigma' at a blocked step (a point on a later segment has no
// defined side or, at a drop, direction: its clamp is ill-conditioned).
// later (may be NULL): pre-image through these later strokes (cx, cy, angle,
// length [N]) instead of the ones this call compensates -- each stroke is
// then the compensation step alone, given the later geometry. amp (may be
// NULL): the largest Frobenius norm, over the steps of a stroke's chains, of
// the Jacobian from that step's point to the chain's end (dual numbers): how
// much an error made at any step can grow by the end.
void orc_compensate(const orc_program* prog, double eps, int32_t endpoint, int32_t skip,
                    double* cx, double* cy, double* angle, double* length, int32_t* blocked,
                    double* dmin, double* smin, const double* later_cx, const double* later_cy,
                    const double* later_angle, const double* later_length, double* amp) {
  Program p = to_prog(prog);
  const int N = p.n;
  const bool given = later_cx && later_cy && later_angle && later_length;
  for (int i = N - 1; i >= 0; --i) {
    const double ce = std::cos(p.angle[i]), se = std::sin(p.angle[i]), L = p.length[i];
    double pts[2][2] = {{p.cx[i] - 0.5 * L * ce, p.cy[i] - 0.5 * L * se},
                        {p.cx[i] + 0.5 * L * ce, p.cy[i] + 0.5 * L * se}};
    const int npts = endpoint ? 2 : 1;
    int nb = 0;
    double dm = INFINITY, sm = INFINITY;
    std::vector<double> jac[2];  // per point: the steps' 2x2 Jacobians, row-major
    for (int j = N - 1; j > i; --j) {
      Stroke<double> g = given ? Stroke<double>{later_cx[j], later_cy[j], later_angle[j],
                                                later_length[j], p.half_width[j]}
                               : Stroke<double>{cx[j], cy[j], angle[j], length[j], p.half_width[j]};
      for (int q = 0; q < npts; ++q) {
        Chart<double> c = chart(pts[q][0], pts[q][1], g);
        dm = std::min(dm, std::fabs(c.sigma - g.r));
        const bool inside = c.sigma <= g.r;
        if (inside) sm = std::min(sm, c.sigma);
        nb += inside ? 1 : 0;
        if (inside && skip) continue;
        if (amp) {
          Dual X(pts[q][0]), Y(pts[q][1]);
          X.d[0] = 1;
          Y.d[1] = 1;
          Stroke<Dual> gd{Dual(g.mx), Dual(g.my), Dual(g.phi), Dual(g.L), Dual(g.r)};
          Dual OX, OY;
          psi(X, Y, gd, eps, OX, OY);
          jac[q].insert(jac[q].end(), {OX.d[0], OX.d[1], OY.d[0], OY.d[1]});
        }
        double ox, oy;
        psi(pts[q][0], pts[q][1], g, eps, ox, oy);
        pts[q][0] = ox;
        pts[q][1] = oy;
      }
    }
    blocked[i] = nb;
    if (dmin) dmin[i] = dm;
    if (smin) smin[i] = sm;
    if (amp) {
      double a = 1.0;
      for (int q = 0; q < npts; ++q) {
        double S[4] = {1, 0, 0, 1};  // product of the Jacobians from a step to the end
        for (size_t t = jac[q].size(); t >= 4; t -= 4) {
          const double* J = &jac[q][t - 4];
          const double P[4] = {S[0] * J[0] + S[1] * J[2], S[0] * J[1] + S[1] * J[3],
                               S[2] * J[0] + S[3] * J[2], S[2] * J[1] + S[3] * J[3]};
          std::copy(P, P + 4, S);
          a = std::max(a, std::sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2] + S[3] * S[3]));
        }
      }
      amp[i] = a;
    }
    if (endpoint) {
      const double dx = pts[1][0] - pts[0][0], dy = pts[1][1] - pts[0][1];
      const double len = std::sqrt(dx * dx + dy * dy);
      cx[i] = 0.5 * (pts[0][0] + pts[1][0]);
      cy[i] = 0.5 * (pts[0][1] + pts[1][1]);
      angle[i] = len > 0 ? std::atan2(dy, dx) : p.angle[i];
      length[i] = len;
    } else {
      cx[i] = pts[0][0] + 0.5 * L * ce;
      cy[i] = pts[0][1] + 0.5 * L * se;
      angle[i] = p.angle[i];
      length[i] = L;
    }
  }
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n);
#else
  (void)n;
#endif
}

}  // extern "C"
