/*
 * oracle.cpp -- plain, slow, single-threaded FP64 reference of the particle
 * step of the special-relativistic curvilinear PIC method of Entity paper I
 * (arXiv 2511.17710).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py; never by the product path.  It shares no code
 * with the HIP library.  Built with -O2 -ffp-contract=off, no fast-math.
 *
 * Every routine is templated on the scalar so that forward-mode dual numbers
 * give exact derivatives of the same code (used by the adjoint reference).
 *
 * What it computes, per particle and step (Sec. 2.3, steps 3-8):
 *   interpolate E,B (first-order shape) at x^n            (step 3)
 *   tetrad + rotation into the global Cartesian basis      (step 4, eq. tetradtrans)
 *   relativistic Boris push of u^{n-1/2} -> u^{n+1/2}       (step 5, eq. equations-of-motion)
 *   move x^n -> x^{n+1} in Cartesian space, convert back   (steps 6-7, Sec. 2.4 maps)
 *   charge-conserving zig-zag deposit of conformal current (step 8, eq. chargecons-2,
 *                                                           Sec. 3.2 footnote)
 *
 * Readings where the paper is silent (each is listed in the design doc):
 *   - interpolation weights: cloud-in-cell on each component's own Yee lattice;
 *   - fields static during the call and centred at t^n (test-particle mode);
 *   - push coefficient k = q dt / (2 m rho0) with q, m in fiducial units (Sec. 2.1);
 *   - each zig-zag segment deposits the exact flux of the first-order shape
 *     along its straight path (midpoint weights + F_a F_b / 12), exact charge
 *     conservation in 3D as well as 2D;
 *   - out-of-plane 2D current: half of C*dx3 per zig-zag segment with that
 *     segment's exact area-weight integral, dx3 = dt*u_z/gamma (Cartesian) or
 *     the wrapped azimuthal step (axisymmetric);
 *   - axisymmetric move evaluated in an offset-relative form algebraically
 *     equal to backward(forward(x^n) + dX) (tests pin it against the literal
 *     composition of the Sec. 2.4 maps);
 *   - theta^{-1} for the quasi-spherical grid from the depressed cubic
 *     (the printed App. B formula does not invert theta(T)), Newton-polished;
 *   - a radial exit deposits the whole step (into ghost cells), then kills the
 *     particle; theta is clamped into [0, pi].
 */
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

namespace {

constexpr int NG = 2;  // ghost cells per side (Sec. 3.1, N_GHOST = 2)
constexpr double PI = 3.14159265358979323846;

// ---------------------------------------------------------------- dual numbers
template <int N>
struct Dual {
  double v;
  double g[N];
  Dual() : v(0.0) {
    for (int i = 0; i < N; ++i) g[i] = 0.0;
  }
  Dual(double x) : v(x) {  // NOLINT: implicit on purpose
    for (int i = 0; i < N; ++i) g[i] = 0.0;
  }
};

inline double val(double x) { return x; }
template <int N>
inline double val(const Dual<N> &x) { return x.v; }

template <int N>
Dual<N> operator+(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r(a.v + b.v);
  for (int i = 0; i < N; ++i) r.g[i] = a.g[i] + b.g[i];
  return r;
}
template <int N>
Dual<N> operator-(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r(a.v - b.v);
  for (int i = 0; i < N; ++i) r.g[i] = a.g[i] - b.g[i];
  return r;
}
template <int N>
Dual<N> operator-(const Dual<N> &a) {
  Dual<N> r(-a.v);
  for (int i = 0; i < N; ++i) r.g[i] = -a.g[i];
  return r;
}
template <int N>
Dual<N> operator*(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r(a.v * b.v);
  for (int i = 0; i < N; ++i) r.g[i] = a.g[i] * b.v + a.v * b.g[i];
  return r;
}
template <int N>
Dual<N> operator/(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r(a.v / b.v);
  for (int i = 0; i < N; ++i) r.g[i] = (a.g[i] - r.v * b.g[i]) / b.v;
  return r;
}
template <int N>
Dual<N> operator+(const Dual<N> &a, double b) { return a + Dual<N>(b); }
template <int N>
Dual<N> operator+(double a, const Dual<N> &b) { return Dual<N>(a) + b; }
template <int N>
Dual<N> operator-(const Dual<N> &a, double b) { return a - Dual<N>(b); }
template <int N>
Dual<N> operator-(double a, const Dual<N> &b) { return Dual<N>(a) - b; }
template <int N>
Dual<N> operator*(const Dual<N> &a, double b) {
  Dual<N> r(a.v * b);
  for (int i = 0; i < N; ++i) r.g[i] = a.g[i] * b;
  return r;
}
template <int N>
Dual<N> operator*(double a, const Dual<N> &b) { return b * a; }
template <int N>
Dual<N> operator/(const Dual<N> &a, double b) { return a / Dual<N>(b); }
template <int N>
Dual<N> operator/(double a, const Dual<N> &b) { return Dual<N>(a) / b; }

// elementary functions: value from libm, derivative from calculus
template <int N>
Dual<N> chain(const Dual<N> &a, double f, double df) {
  Dual<N> r(f);
  for (int i = 0; i < N; ++i) r.g[i] = df * a.g[i];
  return r;
}
inline double d_sqrt(double x) { return std::sqrt(x); }
template <int N>
Dual<N> d_sqrt(const Dual<N> &a) {
  double s = std::sqrt(a.v);
  return chain(a, s, 0.5 / s);
}
inline double d_sin(double x) { return std::sin(x); }
template <int N>
Dual<N> d_sin(const Dual<N> &a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
inline double d_cos(double x) { return std::cos(x); }
template <int N>
Dual<N> d_cos(const Dual<N> &a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
inline double d_exp(double x) { return std::exp(x); }
template <int N>
Dual<N> d_exp(const Dual<N> &a) {
  double e = std::exp(a.v);
  return chain(a, e, e);
}
inline double d_log(double x) { return std::log(x); }
template <int N>
Dual<N> d_log(const Dual<N> &a) { return chain(a, std::log(a.v), 1.0 / a.v); }
inline double d_log1p(double x) { return std::log1p(x); }
template <int N>
Dual<N> d_log1p(const Dual<N> &a) { return chain(a, std::log1p(a.v), 1.0 / (1.0 + a.v)); }
inline double d_expm1(double x) { return std::expm1(x); }
template <int N>
Dual<N> d_expm1(const Dual<N> &a) { return chain(a, std::expm1(a.v), std::exp(a.v)); }
inline double d_atan2(double y, double x) { return std::atan2(y, x); }
template <int N>
Dual<N> d_atan2(const Dual<N> &y, const Dual<N> &x) {
  Dual<N> r(std::atan2(y.v, x.v));
  double den = x.v * x.v + y.v * y.v;
  for (int i = 0; i < N; ++i) r.g[i] = (x.v * y.g[i] - y.v * x.g[i]) / den;
  return r;
}

// a copy of x with the same derivative but a prescribed value
template <class T>
T with_value(const T &x, double v) {
  return x - T(val(x)) + T(v);
}

// ---------------------------------------------------------------- grid / metric
struct Grid {
  int geom, dim;
  int n[3];
  double lo[3], hi[3];
  double r0, vt;
  int periodic[3];
  double rho0;
  double d[3];                // Cartesian cell sizes
  double dr, dth;             // spherical
  double Rmin, dR, dT;        // quasi-spherical
  int np[3];                  // padded extents
  int64_t npts;               // np0*np1*np2
};

bool make_grid(const orc_grid *in, Grid &G) {
  G.geom = in->geom;
  G.dim = in->dim;
  for (int d = 0; d < 3; ++d) {
    G.n[d] = in->n[d];
    G.lo[d] = in->lo[d];
    G.hi[d] = in->hi[d];
    G.periodic[d] = in->periodic[d];
  }
  G.r0 = in->r0;
  G.vt = in->vartheta;
  G.rho0 = in->rho0;
  if (G.geom < 0 || G.geom > 2) return false;
  if (G.geom == 0 && (G.dim < 2 || G.dim > 3)) return false;
  if (G.geom != 0 && G.dim != 2) return false;
  for (int d = 0; d < 3; ++d) {
    G.np[d] = (d < G.dim) ? G.n[d] + 2 * NG : 1;
    G.d[d] = (d < G.dim && G.geom == 0) ? (G.hi[d] - G.lo[d]) / G.n[d] : 1.0;
  }
  G.npts = (int64_t)G.np[0] * G.np[1] * G.np[2];
  // Sec. 2.4: spherical dr = (r_max - r_min)/N_r, dtheta = pi/N_theta
  G.dr = (G.hi[0] - G.lo[0]) / G.n[0];
  G.dth = PI / G.n[1];
  // Sec. 2.4: quasi-spherical R = log(r - r0), dR = [log(rmax-r0) - log(rmin-r0)]/N_R, dT = pi/N_T
  if (G.geom == 2) {
    G.Rmin = std::log(G.lo[0] - G.r0);
    G.dR = (std::log(G.hi[0] - G.r0) - G.Rmin) / G.n[0];
    G.dT = PI / G.n[1];
  } else {
    G.Rmin = G.dR = G.dT = 0.0;
  }
  return true;
}

// Sec. 2.4, quasi-spherical: theta(T) = T + 2*vt*T*(1 - 2T/pi)*(1 - T/pi)
template <class T>
T theta_of_T(const Grid &G, const T &Tc) {
  return Tc + 2.0 * G.vt * Tc * (1.0 - 2.0 * Tc / PI) * (1.0 - Tc / PI);
}
// Sec. 2.4: d theta / d T = 1 + 2 vt + 12 vt (T/pi)(T/pi - 1)
template <class T>
T dtheta_dT(const Grid &G, const T &Tc) {
  return 1.0 + 2.0 * G.vt + 12.0 * G.vt * (Tc / PI) * (Tc / PI - 1.0);
}
// radius at code coordinate x1 (Sec. 2.4 forward maps)
template <class T>
T r_of(const Grid &G, const T &x1) {
  if (G.geom == 1) return G.lo[0] + x1 * G.dr;
  return G.r0 + d_exp(G.Rmin + x1 * G.dR);
}
template <class T>
T theta_of(const Grid &G, const T &x2) {
  if (G.geom == 1) return x2 * G.dth;
  return theta_of_T(G, x2 * G.dT);
}
// sqrt(h_ii) at code coordinates (Sec. 2.4 metric list)
template <class T>
void sqrt_h(const Grid &G, const T &x1, const T &x2, T h[3]) {
  if (G.geom == 0) {
    for (int d = 0; d < 3; ++d) h[d] = T(d < G.dim ? G.d[d] : 1.0);
    return;
  }
  T r = r_of(G, x1);
  T th = theta_of(G, x2);
  if (G.geom == 1) {
    h[0] = T(G.dr);
    h[1] = r * G.dth;
  } else {
    T Tc = x2 * G.dT;
    h[0] = G.dR * d_exp(G.Rmin + x1 * G.dR);
    h[1] = G.dT * dtheta_dT(G, Tc) * r;
  }
  h[2] = r * d_sin(th);
}

// inverse of theta(T): with T = pi/2 + s the map is theta = pi/2 + (1-vt) s + (4 vt/pi^2) s^3,
// i.e. the depressed cubic s^3 + p s + q = 0 solved by Cardano (one real root for
// 0 < vt < 1), then polished by Newton on theta(T) - theta.
double T_of_theta(const Grid &G, double th) {
  if (G.geom != 2 || G.vt == 0.0) return th;
  double vt = G.vt;
  double p = (1.0 - vt) * PI * PI / (4.0 * vt);
  double q = (PI / 2.0 - th) * PI * PI / (4.0 * vt);
  double disc = q * q / 4.0 + p * p * p / 27.0;
  double sq = std::sqrt(disc);
  double s = std::cbrt(-q / 2.0 + sq) + std::cbrt(-q / 2.0 - sq);
  double Tc = PI / 2.0 + s;
  for (int it = 0; it < 3; ++it) {
    double f = theta_of_T(G, Tc) - th;
    double fp = dtheta_dT(G, Tc);
    Tc -= f / fp;
  }
  return Tc;
}

// field / current padded index
inline int64_t pidx(const Grid &G, int c, int i, int j, int k) {
  int kk = (G.dim == 3) ? k + NG : 0;
  return (int64_t)c * G.npts + (int64_t)(i + NG) +
         (int64_t)G.np[0] * ((int64_t)(j + NG) + (int64_t)G.np[1] * kk);
}

// Yee staggering (App. A): E1 (i+1/2,j,k), E2 (i,j+1/2,k), E3 (i,j,k+1/2),
// B1 (i,j+1/2,k+1/2), B2 (i+1/2,j,k+1/2), B3 (i+1/2,j+1/2,k)
const double STAG[6][3] = {{0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 0.5},
                           {0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}};

// ---------------------------------------------------------------- step pieces
// Step 3 (Sec. 2.3): F_p = integral of F S(x - x_p); first-order shape on each
// component's own staggered lattice.
template <class T, class F>
void interp(const Grid &G, const F *EB, const int cell[3], const T d[3], T out[6]) {
  for (int c = 0; c < 6; ++c) {
    int b[3] = {0, 0, 0};
    T f[3] = {T(0.0), T(0.0), T(0.0)};
    for (int dd = 0; dd < G.dim; ++dd) {
      T xi = d[dd] - STAG[c][dd];
      if (val(xi) >= 0.0) {
        b[dd] = cell[dd];
        f[dd] = xi;
      } else {
        b[dd] = cell[dd] - 1;
        f[dd] = xi + 1.0;
      }
    }
    T acc(0.0);
    for (int e = 0; e < (1 << G.dim); ++e) {
      T wgt(1.0);
      int o[3] = {0, 0, 0};
      for (int dd = 0; dd < G.dim; ++dd) {
        o[dd] = (e >> dd) & 1;
        wgt = wgt * (o[dd] ? f[dd] : T(1.0) - f[dd]);
      }
      acc = acc + wgt * EB[pidx(G, c, b[0] + o[0], b[1] + o[1], b[2] + o[2])];
    }
    out[c] = acc;
  }
}

// plain-double stencil of the same interpolation (used to scatter adjoints)
void interp_stencil(const Grid &G, int c, const int cell[3], const double d[3], int64_t idx[8],
                    double w[8]) {
  int b[3] = {0, 0, 0};
  double f[3] = {0, 0, 0};
  for (int dd = 0; dd < G.dim; ++dd) {
    double xi = d[dd] - STAG[c][dd];
    if (xi >= 0.0) {
      b[dd] = cell[dd];
      f[dd] = xi;
    } else {
      b[dd] = cell[dd] - 1;
      f[dd] = xi + 1.0;
    }
  }
  for (int e = 0; e < (1 << G.dim); ++e) {
    double wgt = 1.0;
    int o[3] = {0, 0, 0};
    for (int dd = 0; dd < G.dim; ++dd) {
      o[dd] = (e >> dd) & 1;
      wgt *= o[dd] ? f[dd] : 1.0 - f[dd];
    }
    idx[e] = pidx(G, c, b[0] + o[0], b[1] + o[1], b[2] + o[2]);
    w[e] = wgt;
  }
}

// Step 4: tetrad (eq. tetradtrans, A^i_hat = sqrt(h_ii) A^i) at x_p, then the
// rotation (r,theta,phi)_hat -> (x,y,z)_hat for axisymmetric grids.
template <class T>
void to_cart(const Grid &G, const int cell[3], const T d[3], const T &phi, const T F[6], T E[3],
             T B[3]) {
  if (G.geom == 0) {
    for (int dd = 0; dd < 3; ++dd) {
      double s = dd < G.dim ? G.d[dd] : 1.0;
      E[dd] = F[dd] * s;
      B[dd] = F[3 + dd] * s;
    }
    return;
  }
  T x1 = d[0] + (double)cell[0];
  T x2 = d[1] + (double)cell[1];
  T h[3];
  sqrt_h(G, x1, x2, h);
  T th = theta_of(G, x2);
  T st = d_sin(th), ct = d_cos(th), sp = d_sin(phi), cp = d_cos(phi);
  T Fr[2][3];
  for (int f = 0; f < 2; ++f)
    for (int dd = 0; dd < 3; ++dd) Fr[f][dd] = F[3 * f + dd] * h[dd];
  T *outs[2] = {E, B};
  for (int f = 0; f < 2; ++f) {
    const T &a = Fr[f][0];  // r-hat
    const T &b = Fr[f][1];  // theta-hat
    const T &c = Fr[f][2];  // phi-hat
    outs[f][0] = a * st * cp + b * ct * cp - c * sp;
    outs[f][1] = a * st * sp + b * ct * sp + c * cp;
    outs[f][2] = a * ct - b * st;
  }
}

// Step 5: relativistic Boris push (Boris 1970) of eq. equations-of-motion,
// half kick / rotation / half kick with k = q dt / (2 m rho0).
template <class T>
void boris(double k, const T E[3], const T B[3], T u[3]) {
  T um[3], t[3], s[3], up[3], upl[3];
  for (int a = 0; a < 3; ++a) um[a] = u[a] + k * E[a];
  T g = d_sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  for (int a = 0; a < 3; ++a) t[a] = k * B[a] / g;
  T tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  for (int a = 0; a < 3; ++a) s[a] = 2.0 * t[a] / (1.0 + tt);
  up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
  up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
  up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
  upl[0] = um[0] + (up[1] * s[2] - up[2] * s[1]);
  upl[1] = um[1] + (up[2] * s[0] - up[0] * s[2]);
  upl[2] = um[2] + (up[0] * s[1] - up[1] * s[0]);
  for (int a = 0; a < 3; ++a) u[a] = upl[a] + k * E[a];
}

template <class T>
struct MoveOut {
  int cell[3];
  T d[3];
  T phi;
  T dx3;
  int m[3];
  bool alive;
};

// Sec. 2.4 forward map (code -> global Cartesian), plain doubles
void code_to_cart(const Grid &G, const double x[3], double phi, double X[3]) {
  if (G.geom == 0) {
    for (int d = 0; d < 3; ++d) X[d] = (d < G.dim) ? G.lo[d] + x[d] * G.d[d] : 0.0;
    return;
  }
  double r = r_of(G, x[0]);
  double th = theta_of(G, x[1]);
  X[0] = r * std::sin(th) * std::cos(phi);
  X[1] = r * std::sin(th) * std::sin(phi);
  X[2] = r * std::cos(th);
}

// Sec. 2.4 backward map (global Cartesian -> code), literal form
void cart_to_code(const Grid &G, const double X[3], double x[3], double *phi) {
  if (G.geom == 0) {
    for (int d = 0; d < 3; ++d) x[d] = (d < G.dim) ? (X[d] - G.lo[d]) / G.d[d] : 0.0;
    *phi = 0.0;
    return;
  }
  double r = std::sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
  double th = PI / 2.0 - std::atan2(X[2], std::sqrt(X[0] * X[0] + X[1] * X[1]));
  double ph = PI - std::atan2(X[1], -X[0]);
  if (ph >= 2.0 * PI) ph -= 2.0 * PI;
  *phi = ph;
  if (G.geom == 1) {
    x[0] = (r - G.lo[0]) / G.dr;
    x[1] = th / G.dth;
  } else {
    x[0] = (std::log(r - G.r0) - G.Rmin) / G.dR;
    x[1] = T_of_theta(G, th) / G.dT;
  }
  x[2] = 0.0;
}

// Steps 6-7: x^n -> x^{n+1} with dX = dt u/gamma in global Cartesian space,
// then back to code coordinates.  Cartesian: offsets move by dX/Delta (the
// real position (i+delta) is never formed).  Axisymmetric: an offset-relative
// evaluation of backward(forward(x^n) + dX); canonicalisation to a cell
// index plus an offset in [0,1) (Sec. 3.1); boundaries.
template <class T>
void move(const Grid &G, double dt, const int cell[3], const T d[3], const T &phi, const T u[3],
          MoveOut<T> &o) {
  T g = d_sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  T DX[3];
  for (int a = 0; a < 3; ++a) DX[a] = dt * u[a] / g;
  T dx[3] = {T(0.0), T(0.0), T(0.0)};
  o.phi = phi;
  o.dx3 = T(0.0);
  if (G.geom == 0) {
    for (int dd = 0; dd < G.dim; ++dd) dx[dd] = DX[dd] / G.d[dd];
    if (G.dim == 2) o.dx3 = DX[2];
  } else {
    T x1 = d[0] + (double)cell[0];
    T x2 = d[1] + (double)cell[1];
    T ro = r_of(G, x1);
    T th = theta_of(G, x2);
    T st = d_sin(th), ct = d_cos(th), sp = d_sin(phi), cp = d_cos(phi);
    T xo = ro * st * cp, yo = ro * st * sp, zo = ro * ct;
    T rho_o = ro * st;
    T xn = xo + DX[0], yn = yo + DX[1], zn = zo + DX[2];
    T rho_n = d_sqrt(xn * xn + yn * yn);
    T dr, dth, dphi;
    if (val(rho_n) + val(rho_o) == 0.0) {
      // degenerate: both points on the axis; literal composition
      T rn = d_sqrt(xn * xn + yn * yn + zn * zn);
      dr = rn - ro;
      dth = (PI / 2.0 - d_atan2(zn, rho_n)) - th;
      dphi = T(0.0);
    } else {
      T sig = 2.0 * (xo * DX[0] + yo * DX[1] + zo * DX[2]) / (ro * ro) +
              (DX[0] * DX[0] + DX[1] * DX[1] + DX[2] * DX[2]) / (ro * ro);
      dr = ro * d_expm1(0.5 * d_log1p(sig));
      T drho = (2.0 * (xo * DX[0] + yo * DX[1]) + DX[0] * DX[0] + DX[1] * DX[1]) / (rho_n + rho_o);
      dth = d_atan2(drho * zo - DX[2] * rho_o, rho_o * rho_n + zo * zn);
      // azimuth step, numerator and denominator divided by rho_o so that a start
      // exactly on the axis takes the azimuth of the displacement itself
      dphi = d_atan2(cp * DX[1] - sp * DX[0], rho_o + cp * DX[0] + sp * DX[1]);
    }
    if (G.geom == 1) {
      dx[0] = dr / G.dr;
      dx[1] = dth / G.dth;
    } else {
      dx[0] = d_log1p(dr / (ro - G.r0)) / G.dR;
      // theta(T0 + s) - theta(T0) = theta'(T0) s + (6 vt/pi^2)(2 T0 - pi) s^2 + (4 vt/pi^2) s^3
      T T0 = x2 * G.dT;
      T a1 = dtheta_dT(G, T0);
      T a2 = (6.0 * G.vt / (PI * PI)) * (2.0 * T0 - PI);
      double a3 = 4.0 * G.vt / (PI * PI);
      T s = dth / a1;
      for (int it = 0; it < 4; ++it) {
        T f = a1 * s + a2 * s * s + a3 * s * s * s - dth;
        T fp = a1 + 2.0 * a2 * s + 3.0 * a3 * s * s;
        s = s - f / fp;
      }
      dx[1] = s / G.dT;
    }
    T pn = phi + dphi;
    if (val(pn) < 0.0) pn = pn + 2.0 * PI;
    if (val(pn) >= 2.0 * PI) pn = pn - 2.0 * PI;
    o.phi = pn;
    o.dx3 = dphi;
  }
  // canonicalise: cell index plus offset in [0,1)
  for (int dd = 0; dd < 3; ++dd) {
    o.cell[dd] = cell[dd];
    o.d[dd] = d[dd];
    o.m[dd] = 0;
  }
  for (int dd = 0; dd < G.dim; ++dd) {
    T y = d[dd] + dx[dd];
    double kf = std::floor(val(y));
    T dn = y - kf;
    int k = (int)kf;
    if (val(dn) >= 1.0) {  // y - floor(y) rounded up to 1
      k += 1;
      dn = with_value(y, 0.0);
    }
    o.cell[dd] = cell[dd] + k;
    o.d[dd] = dn;
  }
  o.alive = true;
  if (G.geom != 0) {
    // theta stays in [0, pi]: clamp rounding excursions
    if (o.cell[1] < 0) {
      o.cell[1] = 0;
      o.d[1] = T(0.0);
    } else if (o.cell[1] >= G.n[1]) {
      o.cell[1] = G.n[1] - 1;
      o.d[1] = T(std::nextafter(1.0, 0.0));
    }
    if (o.cell[0] < 0 || o.cell[0] >= G.n[0]) o.alive = false;  // radial exit
  }
  for (int dd = 0; dd < G.dim; ++dd) o.m[dd] = o.cell[dd] - cell[dd];
  if (G.geom == 0) {
    for (int dd = 0; dd < G.dim; ++dd) {
      int c = o.cell[dd] % G.n[dd];
      if (c < 0) c += G.n[dd];
      o.cell[dd] = c;  // periodic wrap after the (unwrapped) step m was taken
    }
  }
}

// Step 8: zig-zag scheme of Umeda et al. (2003) written on in-cell offsets (Sec. 3.2
// footnote): a = old offset, b = new offset measured from the old cell, relay point
// x_r = min(min(0,m)+1, max(max(0,m), (a+b)/2)); segment 1 lies in the old cell,
// segment 2 in the new one.  Each straight segment deposits the exact flux of the
// first-order (trilinear) shape through the Yee edges: midpoint weights plus the
// F_a F_b / 12 covariance term, which is what makes 3D (not only 2D) exactly
// charge conserving.  Conformal current (eq. chargecons-2), C = q w / dt, so that
// div J + (rho^{n+1} - rho^n)/dt = 0 at every node.
template <class T, class Dep>
void deposit(const Grid &G, double C, const int cell_old[3], const T d_old[3], const int m[3],
             const T d_new[3], const T &dx3, Dep &&dep) {
  T F[2][3], W[2][3];
  for (int dd = 0; dd < 3; ++dd) {
    F[0][dd] = F[1][dd] = W[0][dd] = W[1][dd] = T(0.0);
  }
  for (int dd = 0; dd < G.dim; ++dd) {
    const T &a = d_old[dd];
    T b = d_new[dd] + (double)m[dd];
    double lo = std::min(0, m[dd]) + 1.0;
    double hi = (double)std::max(0, m[dd]);
    T mid = (a + b) * 0.5;
    T mx = (val(mid) >= hi) ? mid : T(hi);
    T xr = (val(mx) <= lo) ? mx : T(lo);
    F[0][dd] = xr - a;
    F[1][dd] = b - xr;
    W[0][dd] = (a + xr) * 0.5;
    W[1][dd] = (xr + b) * 0.5 - (double)m[dd];
  }
  for (int s = 0; s < 2; ++s) {
    int I = cell_old[0] + (s ? m[0] : 0);
    int J = cell_old[1] + (s ? m[1] : 0);
    int K = cell_old[2] + (s ? m[2] : 0);
    const T *Fs = F[s];
    const T *Ws = W[s];
    if (G.dim == 2) {
      dep(0, I, J, 0, C * Fs[0] * (1.0 - Ws[1]));
      dep(0, I, J + 1, 0, C * Fs[0] * Ws[1]);
      dep(1, I, J, 0, C * Fs[1] * (1.0 - Ws[0]));
      dep(1, I + 1, J, 0, C * Fs[1] * Ws[0]);
      // out-of-plane: half the step per segment, exact area-weight integral
      T h = C * dx3 * 0.5;
      T cxy = Fs[0] * Fs[1] * (1.0 / 12.0);
      dep(2, I, J, 0, h * ((1.0 - Ws[0]) * (1.0 - Ws[1]) + cxy));
      dep(2, I + 1, J, 0, h * (Ws[0] * (1.0 - Ws[1]) - cxy));
      dep(2, I, J + 1, 0, h * ((1.0 - Ws[0]) * Ws[1] - cxy));
      dep(2, I + 1, J + 1, 0, h * (Ws[0] * Ws[1] + cxy));
    } else {
      // exact flux of the trilinear shape along the straight segment:
      // midpoint weights plus the covariance term F_a F_b / 12
      T cyz = Fs[1] * Fs[2] * (1.0 / 12.0);
      T cxz = Fs[0] * Fs[2] * (1.0 / 12.0);
      T cxy = Fs[0] * Fs[1] * (1.0 / 12.0);
      for (int e = 0; e < 4; ++e) {
        int e1 = e & 1, e2 = (e >> 1) & 1;
        double sg = (e1 == e2) ? 1.0 : -1.0;
        // J1 on x-edges (i+1/2, j, k): weights in y, z
        dep(0, I, J + e1, K + e2,
            C * Fs[0] * ((e1 ? Ws[1] : 1.0 - Ws[1]) * (e2 ? Ws[2] : 1.0 - Ws[2]) + sg * cyz));
        // J2 on y-edges (i, j+1/2, k): weights in x, z
        dep(1, I + e1, J, K + e2,
            C * Fs[1] * ((e1 ? Ws[0] : 1.0 - Ws[0]) * (e2 ? Ws[2] : 1.0 - Ws[2]) + sg * cxz));
        // J3 on z-edges (i, j, k+1/2): weights in x, y
        dep(2, I + e1, J + e2, K,
            C * Fs[2] * ((e1 ? Ws[0] : 1.0 - Ws[0]) * (e2 ? Ws[1] : 1.0 - Ws[1]) + sg * cxy));
      }
    }
  }
}

// current index with periodic wrap on write (Cartesian) or ghost cells (curvilinear)
int64_t jidx(const Grid &G, int c, int i, int j, int k) {
  int ii[3] = {i, j, k};
  for (int dd = 0; dd < G.dim; ++dd) {
    if (G.geom == 0 && G.periodic[dd]) {
      int v = ii[dd] % G.n[dd];
      if (v < 0) v += G.n[dd];
      ii[dd] = v;
    }
    if (ii[dd] < -NG || ii[dd] >= G.n[dd] + NG) std::abort();
  }
  return pidx(G, c, ii[0], ii[1], ii[2]);
}

// Pusher of a species (Sec. 2.2: a conventional pusher, Boris 1970 or Vay
// 2008, on the global Cartesian components; Sec. 5.2: optionally the hybrid
// that hands particles over to the guiding-centre approximation).
struct Pusher {
  int vay = 0;              // 0: Boris, 1: Vay
  int gca = 0;              // 1: guiding-centre hybrid
  double e_ovr = 0.9;       // GCA only while |E| < e_ovr |B|
  double larmor_max = 0.0;  // ... and the nominal gyroradius is below this length
};

// Guiding-centre regime test of the hybrid pusher (Sec. 5.2): the fields are
// drift-dominated (|E| < e_ovr |B|) and the nominal gyroradius
// rho_L = gamma beta m c^2 / (|q| B) = |u| m rho0 / (|q| |B|) = |u| dt / (2 |k| |B|)
// is below the critical one.
template <class T>
bool gca_regime(double k, double dt, const T E[3], const T B[3], const T u[3], const Pusher &P) {
  const double e2 = val(E[0]) * val(E[0]) + val(E[1]) * val(E[1]) + val(E[2]) * val(E[2]);
  const double b2 = val(B[0]) * val(B[0]) + val(B[1]) * val(B[1]) + val(B[2]) * val(B[2]);
  if (!(b2 > 0.0) || !(e2 < P.e_ovr * P.e_ovr * b2)) return false;
  const double uabs = std::sqrt(val(u[0]) * val(u[0]) + val(u[1]) * val(u[1]) + val(u[2]) * val(u[2]));
  const double rl = uabs * dt / (2.0 * std::fabs(k) * std::sqrt(b2));
  return rl < P.larmor_max;
}

// Guiding-centre update with zero magnetic moment (reading of Sec. 5.2 after
// Bacchini et al. 2020): the momentum perpendicular to B is dropped, the
// parallel four-velocity takes the full parallel kick 2 k (E.b), and the
// particle moves with its guiding centre, v = v_par b + E x B / B^2, whose
// Lorentz factor is gamma = kappa sqrt(1 + u_par^2), kappa = (1 - v_E^2)^(-1/2);
// u = u_par b + gamma v_E.
template <class T>
void gca_push(double k, const T E[3], const T B[3], T u[3]) {
  T b2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  T bn = d_sqrt(b2);
  T b[3] = {B[0] / bn, B[1] / bn, B[2] / bn};
  T vE[3] = {(E[1] * B[2] - E[2] * B[1]) / b2, (E[2] * B[0] - E[0] * B[2]) / b2,
             (E[0] * B[1] - E[1] * B[0]) / b2};
  T upar = u[0] * b[0] + u[1] * b[1] + u[2] * b[2] +
           2.0 * k * (E[0] * b[0] + E[1] * b[1] + E[2] * b[2]);
  T vE2 = vE[0] * vE[0] + vE[1] * vE[1] + vE[2] * vE[2];
  T g = d_sqrt((1.0 + upar * upar) / (1.0 - vE2));
  for (int a = 0; a < 3; ++a) u[a] = upar * b[a] + g * vE[a];
}

// Vay (2008) pusher: u^{n+1/2} = u^{n-1/2} + (q dt / m)(E + vbar x B) with
// vbar the mean of the velocities before and after, solved in closed form
// for the new Lorentz factor.  In code units (q dt / m) E = 2 k E and
// (q dt / m)(v / 2) x B = k v x B.
template <class T>
void vay(double k, const T E[3], const T B[3], T u[3]) {
  T g0 = d_sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  T v[3] = {u[0] / g0, u[1] / g0, u[2] / g0};
  T up[3] = {u[0] + 2.0 * k * E[0] + k * (v[1] * B[2] - v[2] * B[1]),
             u[1] + 2.0 * k * E[1] + k * (v[2] * B[0] - v[0] * B[2]),
             u[2] + 2.0 * k * E[2] + k * (v[0] * B[1] - v[1] * B[0])};
  T tau[3] = {k * B[0], k * B[1], k * B[2]};
  T ustar = up[0] * tau[0] + up[1] * tau[1] + up[2] * tau[2];
  T tau2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];
  T sigma = 1.0 + up[0] * up[0] + up[1] * up[1] + up[2] * up[2] - tau2;
  T gn = d_sqrt(0.5 * (sigma + d_sqrt(sigma * sigma + 4.0 * (tau2 + ustar * ustar))));
  T t[3] = {tau[0] / gn, tau[1] / gn, tau[2] / gn};
  T s = 1.0 / (1.0 + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  T ut = up[0] * t[0] + up[1] * t[1] + up[2] * t[2];
  T un[3] = {s * (up[0] + ut * t[0] + (up[1] * t[2] - up[2] * t[1])),
             s * (up[1] + ut * t[1] + (up[2] * t[0] - up[0] * t[2])),
             s * (up[2] + ut * t[2] + (up[0] * t[1] - up[1] * t[0]))};
  for (int a = 0; a < 3; ++a) u[a] = un[a];
}

// one particle, one step (steps 3-8); hook(F6) lets the caller perturb F_p
template <class T, class F, class Hook, class Dep>
bool push_particle(const Grid &G, const F *EB, double dt, double q, double mass, double w,
                   int cell[3], T d[3], T u[3], T &phi, Hook &&hook, Dep &&dep,
                   const Pusher &P = Pusher()) {
  T Fp[6], E[3], B[3];
  interp(G, EB, cell, d, Fp);
  hook(Fp);
  to_cart(G, cell, d, phi, Fp, E, B);
  double k = q * dt / (2.0 * mass * G.rho0);
  if (P.gca && gca_regime(k, dt, E, B, u, P))
    gca_push(k, E, B, u);
  else if (P.vay)
    vay(k, E, B, u);
  else
    boris(k, E, B, u);
  MoveOut<T> o;
  move(G, dt, cell, d, phi, u, o);
  int cell_unwrapped_old[3] = {cell[0], cell[1], cell[2]};
  deposit(G, q * w / dt, cell_unwrapped_old, d, o.m, o.d, o.dx3, dep);
  for (int dd = 0; dd < 3; ++dd) {
    cell[dd] = o.cell[dd];
    d[dd] = o.d[dd];
  }
  phi = o.phi;
  return o.alive;
}

// periodic ghost fill of a padded multi-component array (Cartesian)
template <class F>
void fill_periodic_ghosts(const Grid &G, F *A, int ncomp) {
  if (G.geom != 0) return;
  for (int c = 0; c < ncomp; ++c)
    for (int dd = 0; dd < G.dim; ++dd) {
      if (!G.periodic[dd]) continue;
      int lo3 = (G.dim == 3) ? -NG : 0, hi3 = (G.dim == 3) ? G.n[2] + NG : 1;
      for (int k = lo3; k < hi3; ++k)
        for (int j = -NG; j < G.n[1] + NG; ++j)
          for (int i = -NG; i < G.n[0] + NG; ++i) {
            int ii[3] = {i, j, k};
            int v = ii[dd];
            if (v >= 0 && v < G.n[dd]) continue;
            int s = v % G.n[dd];
            if (s < 0) s += G.n[dd];
            int src[3] = {i, j, k};
            src[dd] = s;
            A[pidx(G, c, i, j, k)] = A[pidx(G, c, src[0], src[1], src[2])];
          }
    }
}

// periodic fold of ghost contributions into their images (adjoint of the fill)
void fold_periodic_ghosts(const Grid &G, double *A, int ncomp) {
  if (G.geom != 0) return;
  for (int c = 0; c < ncomp; ++c)
    for (int dd = G.dim - 1; dd >= 0; --dd) {
      if (!G.periodic[dd]) continue;
      int lo3 = (G.dim == 3) ? -NG : 0, hi3 = (G.dim == 3) ? G.n[2] + NG : 1;
      for (int k = lo3; k < hi3; ++k)
        for (int j = -NG; j < G.n[1] + NG; ++j)
          for (int i = -NG; i < G.n[0] + NG; ++i) {
            int ii[3] = {i, j, k};
            int v = ii[dd];
            if (v >= 0 && v < G.n[dd]) continue;
            int s = v % G.n[dd];
            if (s < 0) s += G.n[dd];
            int dst[3] = {i, j, k};
            dst[dd] = s;
            A[pidx(G, c, dst[0], dst[1], dst[2])] += A[pidx(G, c, i, j, k)];
            A[pidx(G, c, i, j, k)] = 0.0;
          }
    }
}

struct PlainSpecies {
  std::vector<int32_t> cell;  // n*3
  std::vector<double> offs, u, w, phi;
  std::vector<int32_t> alive;
};

PlainSpecies copy_in(const Grid &G, const orc_species &s) {
  PlainSpecies p;
  int64_t n = s.n;
  p.cell.assign(s.cell, s.cell + 3 * n);
  p.offs.assign(s.offs, s.offs + 3 * n);
  p.u.assign(s.u, s.u + 3 * n);
  p.w.assign(s.w, s.w + n);
  if (G.geom != 0 && s.phi)
    p.phi.assign(s.phi, s.phi + n);
  else
    p.phi.assign(n, 0.0);
  p.alive.assign(s.alive, s.alive + n);
  return p;
}

// Sort key: cells ordered brick by brick (4x4x4 bricks in 3D, 8x8 in 2D), x
// fastest between and inside bricks, so that a run of consecutive particles
// covers a compact block of cells; dead particles last.
int32_t sort_key(const Grid &G, const int32_t *c, int32_t alive) {
  if (!alive) return INT32_MAX;
  const int B[3] = {G.dim == 3 ? 4 : 8, G.dim == 3 ? 4 : 8, G.dim == 3 ? 4 : 1};
  int nb[3], bi[3], li[3];
  for (int d = 0; d < 3; ++d) {
    nb[d] = (G.n[d] + B[d] - 1) / B[d];
    bi[d] = c[d] / B[d];
    li[d] = c[d] % B[d];
  }
  const int64_t brick = bi[0] + (int64_t)nb[0] * (bi[1] + (int64_t)nb[1] * bi[2]);
  const int64_t local = li[0] + (int64_t)B[0] * (li[1] + (int64_t)B[1] * li[2]);
  return (int32_t)(brick * (B[0] * B[1] * B[2]) + local);
}

// ---------------------------------------------------------------- field solver
// The field update around the particle step (Sec. 2.3 steps 2, 9-11), on the
// Yee lattice of App. A with the metric of Sec. 2.4: Faraday's and Ampere's
// laws in the discretized forms of App. A (covariant components
// F_i = h_ii F^i differenced over unit code-coordinate cells, divided by
// sqrt(h) = sqrt(h11 h22 h33) at the updated component's point), the axis
// rules of Sec. 2.6 on (quasi-)spherical grids, and the digital filter of
// Sec. 2.5.  `coupling` is the factor in front of the conformal current in
// Ampere's law (4 pi in the paper's units).

// sqrt(h_ii)^2 and sqrt(h) at code coordinates (x3 plays no role)
double h_comp(const Grid &G, int a, double x1, double x2) {
  double h[3];
  sqrt_h(G, x1, x2, h);
  return h[a] * h[a];
}
double sqrt_det_h(const Grid &G, double x1, double x2) {
  double h[3];
  sqrt_h(G, x1, x2, h);
  return h[0] * h[1] * h[2];
}

// node ranges updated by the solver, per component stagger: periodic
// Cartesian [0, N); (quasi-)spherical along x1 and x2: nodes [0, N] for an
// integer stagger, cells [0, N) for a half stagger (ghosts are the caller's)
void node_range(const Grid &G, int dim, double stag, int &lo, int &hi) {
  lo = 0;
  if (dim >= G.dim) {
    hi = 1;
    return;
  }
  if (G.geom == 0)
    hi = G.n[dim];
  else
    hi = (stag == 0.0) ? G.n[dim] + 1 : G.n[dim];
}

// covariant component m of field block f (0: E, 1: B) at array element (i,j,k)
double cov(const Grid &G, const double *EB, int f, int m, int i, int j, int k) {
  const int c = 3 * f + m;
  const double x1 = i + STAG[c][0], x2 = j + STAG[c][1];
  return h_comp(G, m, x1, x2) * EB[pidx(G, c, i, j, k)];
}

bool on_axis(const Grid &G, int j) { return G.geom != 0 && (j == 0 || j == G.n[1]); }

// B^i -= f * (curl E)^i / sqrt(h) (App. A, eq. discretized-faraday); f = dt/2
// for each of the two half steps of the loop
void faraday(const Grid &G, double *EB, double f) {
  std::vector<double> out(EB + 3 * G.npts, EB + 6 * G.npts);
  const bool d3 = G.dim == 3;
  for (int c = 3; c < 6; ++c) {
    int lo[3], hi[3];
    for (int dd = 0; dd < 3; ++dd) node_range(G, dd, STAG[c][dd], lo[dd], hi[dd]);
    for (int k = lo[2]; k < hi[2]; ++k)
      for (int j = lo[1]; j < hi[1]; ++j)
        for (int i = lo[0]; i < hi[0]; ++i) {
          if (c == 4 && on_axis(G, j)) continue;  // B2 on the axis stays 0 (Sec. 2.6)
          double curl = 0.0;
          if (c == 3) {  // B1 at (i, j+1/2, k+1/2)
            curl = cov(G, EB, 0, 2, i, j + 1, k) - cov(G, EB, 0, 2, i, j, k);
            if (d3) curl -= cov(G, EB, 0, 1, i, j, k + 1) - cov(G, EB, 0, 1, i, j, k);
          } else if (c == 4) {  // B2 at (i+1/2, j, k+1/2)
            curl = -(cov(G, EB, 0, 2, i + 1, j, k) - cov(G, EB, 0, 2, i, j, k));
            if (d3) curl += cov(G, EB, 0, 0, i, j, k + 1) - cov(G, EB, 0, 0, i, j, k);
          } else {  // B3 at (i+1/2, j+1/2, k)
            curl = (cov(G, EB, 0, 1, i + 1, j, k) - cov(G, EB, 0, 1, i, j, k)) -
                   (cov(G, EB, 0, 0, i, j + 1, k) - cov(G, EB, 0, 0, i, j, k));
          }
          const double sh = sqrt_det_h(G, i + STAG[c][0], j + STAG[c][1]);
          out[pidx(G, c - 3, i, j, k)] = EB[pidx(G, c, i, j, k)] - f * curl / sh;
        }
  }
  for (int c = 3; c < 6; ++c) {
    int lo[3], hi[3];
    for (int dd = 0; dd < 3; ++dd) node_range(G, dd, STAG[c][dd], lo[dd], hi[dd]);
    for (int k = lo[2]; k < hi[2]; ++k)
      for (int j = lo[1]; j < hi[1]; ++j)
        for (int i = lo[0]; i < hi[0]; ++i) {
          if (c == 4 && on_axis(G, j)) {
            EB[pidx(G, c, i, j, k)] = 0.0;
            continue;
          }
          EB[pidx(G, c, i, j, k)] = out[pidx(G, c - 3, i, j, k)];
        }
  }
  fill_periodic_ghosts(G, EB + 3 * G.npts, 3);
}

// Sec. 2.6: A(x1) = integral over x2 in [0, 1/2] of sqrt(h), in the paper's
// closed forms: spherical r^2 dr (1 - cos(dtheta/2)); quasi-spherical
// (r0 + e^R)^2 e^R dR (1 - cos(theta(dT/2)))
double polar_area(const Grid &G, double x1) {
  if (G.geom == 1) {
    const double r = G.lo[0] + x1 * G.dr;
    return r * r * G.dr * (1.0 - std::cos(0.5 * G.dth));
  }
  const double eR = std::exp(G.Rmin + x1 * G.dR);
  const double r = G.r0 + eR;
  const double tt = 0.5 * G.dT + G.vt * G.dT * (1.0 - G.dT / PI) * (1.0 - G.dT / (2.0 * PI));
  return r * r * eR * G.dR * (1.0 - std::cos(tt));
}

// E^i += dt (curl B)^i / sqrt(h) - coupling dt J^i / sqrt(h) (App. A,
// eq. discretized-ampere); on the axis nodes E3 = 0 and E1 takes the
// integrated form (Sec. 2.6)
void ampere(const Grid &G, double *EB, const double *J, double dt, double coupling) {
  std::vector<double> out(EB, EB + 3 * G.npts);
  const bool d3 = G.dim == 3;
  const double *Bv = EB;  // covariant B through cov(.., f = 1, ..)
  for (int c = 0; c < 3; ++c) {
    int lo[3], hi[3];
    for (int dd = 0; dd < 3; ++dd) node_range(G, dd, STAG[c][dd], lo[dd], hi[dd]);
    for (int k = lo[2]; k < hi[2]; ++k)
      for (int j = lo[1]; j < hi[1]; ++j)
        for (int i = lo[0]; i < hi[0]; ++i) {
          const double Jc = J[pidx(G, c, i, j, k)];
          double v;
          if (c == 2 && on_axis(G, j)) {
            v = 0.0;
          } else if (c == 0 && on_axis(G, j)) {
            // integrated over the half cell next to the axis: A dE1/dt =
            // +-B_3 at the half node inside - (coupling / 2) J1
            const double A = polar_area(G, i + 0.5);
            const double b3 = (j == 0) ? cov(G, Bv, 1, 2, i, 0, k) : -cov(G, Bv, 1, 2, i, j - 1, k);
            v = EB[pidx(G, c, i, j, k)] + dt * (b3 - 0.5 * coupling * Jc) / A;
          } else {
            double curl;
            if (c == 0) {  // E1 at (i+1/2, j, k)
              curl = cov(G, Bv, 1, 2, i, j, k) - cov(G, Bv, 1, 2, i, j - 1, k);
              if (d3) curl -= cov(G, Bv, 1, 1, i, j, k) - cov(G, Bv, 1, 1, i, j, k - 1);
            } else if (c == 1) {  // E2 at (i, j+1/2, k)
              curl = -(cov(G, Bv, 1, 2, i, j, k) - cov(G, Bv, 1, 2, i - 1, j, k));
              if (d3) curl += cov(G, Bv, 1, 0, i, j, k) - cov(G, Bv, 1, 0, i, j, k - 1);
            } else {  // E3 at (i, j, k+1/2)
              curl = (cov(G, Bv, 1, 1, i, j, k) - cov(G, Bv, 1, 1, i - 1, j, k)) -
                     (cov(G, Bv, 1, 0, i, j, k) - cov(G, Bv, 1, 0, i, j - 1, k));
            }
            const double sh = sqrt_det_h(G, i + STAG[c][0], j + STAG[c][1]);
            v = EB[pidx(G, c, i, j, k)] + dt * (curl - coupling * Jc) / sh;
          }
          out[pidx(G, c, i, j, k)] = v;
        }
  }
  for (int c = 0; c < 3; ++c) {
    int lo[3], hi[3];
    for (int dd = 0; dd < 3; ++dd) node_range(G, dd, STAG[c][dd], lo[dd], hi[dd]);
    for (int k = lo[2]; k < hi[2]; ++k)
      for (int j = lo[1]; j < hi[1]; ++j)
        for (int i = lo[0]; i < hi[0]; ++i) EB[pidx(G, c, i, j, k)] = out[pidx(G, c, i, j, k)];
  }
  fill_periodic_ghosts(G, EB, 3);
}

// One pass of the digital filter of Sec. 2.5 on the conformal current: each
// component on its own lattice, weights (1/2)^(D + |di| + |dj| + |dk|) over
// the 3^D neighbourhood.  Periodic Cartesian grids wrap; (quasi-)spherical
// grids mirror across the axes (Sec. 2.6: J1(j = -1) = J1(j = +1),
// J2(j = -1/2) = -J2(j = +1/2), J3 = 0 on the axis, and likewise at
// theta = pi) and read the stored ghost values across the radial edges
// (filtered: the updated node ranges of the solver; ghosts unchanged).
double j_at(const Grid &G, const double *J, int c, int i, int j, int k) {
  if (G.geom == 0) {
    int ii[3] = {i, j, k};
    for (int dd = 0; dd < G.dim; ++dd) {
      ii[dd] %= G.n[dd];
      if (ii[dd] < 0) ii[dd] += G.n[dd];
    }
    return J[pidx(G, c, ii[0], ii[1], ii[2])];
  }
  const int n2 = G.n[1];
  if (c == 2 && (j == 0 || j == n2)) return 0.0;
  if (c == 1) {  // half-integer points j + 1/2
    if (j < 0) return -J[pidx(G, c, i, -1 - j, k)];
    if (j >= n2) return -J[pidx(G, c, i, 2 * n2 - 1 - j, k)];
  } else {  // integer nodes
    if (j < 0) return J[pidx(G, c, i, -j, k)];
    if (j > n2) return J[pidx(G, c, i, 2 * n2 - j, k)];
  }
  return J[pidx(G, c, i, j, k)];
}

void filter_pass(const Grid &G, double *J) {
  std::vector<double> out(J, J + 3 * G.npts);
  const int D = G.dim;
  for (int c = 0; c < 3; ++c) {
    int lo[3], hi[3];
    for (int dd = 0; dd < 3; ++dd) node_range(G, dd, STAG[c][dd], lo[dd], hi[dd]);
    for (int k = lo[2]; k < hi[2]; ++k)
      for (int j = lo[1]; j < hi[1]; ++j)
        for (int i = lo[0]; i < hi[0]; ++i) {
          double acc = 0.0;
          const int kr = (D == 3) ? 1 : 0;
          for (int dk = -kr; dk <= kr; ++dk)
            for (int dj = -1; dj <= 1; ++dj)
              for (int di = -1; di <= 1; ++di) {
                const int e = D + std::abs(di) + std::abs(dj) + std::abs(dk);
                acc += std::ldexp(1.0, -e) * j_at(G, J, c, i + di, j + dj, k + dk);
              }
          out[pidx(G, c, i, j, k)] = (c == 2 && on_axis(G, j)) ? 0.0 : acc;
        }
  }
  std::copy(out.begin(), out.end(), J);
}

}  // namespace

// ============================================================== extern "C"
extern "C" {

int32_t orc_version(void) { return 1; }

int64_t orc_field_points(const orc_grid *g) {
  Grid G;
  if (!make_grid(g, G)) return -1;
  return G.npts;
}

// Sec. 2.4: dx_min = min over cell centres of (sum_i 1/h_ii)^(-1/2); dt = CFL dx_min
double orc_dt_from_cfl(const orc_grid *g, double cfl) {
  Grid G;
  if (!make_grid(g, G)) return -1.0;
  double best = INFINITY;
  int n2 = G.dim >= 2 ? G.n[1] : 1;
  int n3 = G.dim >= 3 ? G.n[2] : 1;
  for (int k = 0; k < n3; ++k)
    for (int j = 0; j < n2; ++j)
      for (int i = 0; i < G.n[0]; ++i) {
        double h[3];
        sqrt_h(G, i + 0.5, j + 0.5, h);
        int nd = (G.geom == 0) ? G.dim : 2;
        double s = 0.0;
        for (int d = 0; d < nd; ++d) s += 1.0 / (h[d] * h[d]);
        best = std::min(best, 1.0 / std::sqrt(s));
        if (G.geom == 0) return cfl * best;  // uniform
      }
  return cfl * best;
}

void orc_sqrt_h(const orc_grid *g, const double *x, double *h) {
  Grid G;
  make_grid(g, G);
  sqrt_h(G, x[0], x[1], h);
}

double orc_theta_of_T(const orc_grid *g, double T) {
  Grid G;
  make_grid(g, G);
  return theta_of_T(G, T);
}

double orc_T_of_theta(const orc_grid *g, double theta) {
  Grid G;
  make_grid(g, G);
  return T_of_theta(G, theta);
}

void orc_code_to_cart(const orc_grid *g, const double *x, double phi, double *X) {
  Grid G;
  make_grid(g, G);
  code_to_cart(G, x, phi, X);
}

void orc_cart_to_code(const orc_grid *g, const double *X, double *x, double *phi) {
  Grid G;
  make_grid(g, G);
  cart_to_code(G, X, x, phi);
}

// eq. tetradtrans: F^i = F^i_hat / sqrt(h_ii) at the component's own Yee point;
// axis rule of Sec. 2.6: E3 = B2 = 0 on the nodes j = 0 and j = N2.
// includes_ghosts = 0: `in` holds only the active region [6][n3][n2][n1]
// and periodic ghosts are copied; 1: `in` is the padded array.
int orc_fields_from_tetrad(const orc_grid *g, const double *in, int32_t includes_ghosts,
                           double *out) {
  Grid G;
  if (!make_grid(g, G)) return 1;
  std::fill(out, out + 6 * G.npts, 0.0);
  int lo3 = (G.dim == 3) ? -NG : 0, hi3 = (G.dim == 3) ? G.n[2] + NG : 1;
  for (int c = 0; c < 6; ++c)
    for (int k = lo3; k < hi3; ++k)
      for (int j = -NG; j < G.n[1] + NG; ++j)
        for (int i = -NG; i < G.n[0] + NG; ++i) {
          bool active = i >= 0 && i < G.n[0] && j >= 0 && j < G.n[1] &&
                        (G.dim < 3 || (k >= 0 && k < G.n[2]));
          double v;
          if (includes_ghosts) {
            v = in[pidx(G, c, i, j, k)];
          } else {
            if (!active) continue;
            int64_t a = (int64_t)c * G.n[0] * G.n[1] * (G.dim == 3 ? G.n[2] : 1) + i +
                        (int64_t)G.n[0] * (j + (int64_t)G.n[1] * (G.dim == 3 ? k : 0));
            v = in[a];
          }
          int d = c % 3;
          double x[3] = {i + STAG[c][0], j + STAG[c][1], k + STAG[c][2]};
          double h[3];
          sqrt_h(G, x[0], x[1], h);
          double res;
          bool axis_zero = (G.geom != 0) && (c == 2 || c == 4) && (j == 0 || j == G.n[1]);
          if (axis_zero)
            res = 0.0;
          else
            res = v / h[d];
          out[pidx(G, c, i, j, k)] = res;
        }
  if (!includes_ghosts) fill_periodic_ghosts(G, out, 6);
  return 0;
}

void orc_interp(const orc_grid *g, const double *EB, int64_t n, const int32_t *cell,
                const double *offs, double *out6) {
  Grid G;
  make_grid(g, G);
  for (int64_t p = 0; p < n; ++p) {
    int c[3] = {cell[3 * p], cell[3 * p + 1], cell[3 * p + 2]};
    interp(G, EB, c, offs + 3 * p, out6 + 6 * p);
  }
}

void orc_to_cart(const orc_grid *g, int64_t n, const int32_t *cell, const double *offs,
                 const double *phi, const double *F6, double *E3, double *B3) {
  Grid G;
  make_grid(g, G);
  for (int64_t p = 0; p < n; ++p) {
    int c[3] = {cell[3 * p], cell[3 * p + 1], cell[3 * p + 2]};
    double ph = phi ? phi[p] : 0.0;
    to_cart(G, c, offs + 3 * p, ph, F6 + 6 * p, E3 + 3 * p, B3 + 3 * p);
  }
}

void orc_boris(int64_t n, double k, const double *E3, const double *B3, double *u3) {
  for (int64_t p = 0; p < n; ++p) boris(k, E3 + 3 * p, B3 + 3 * p, u3 + 3 * p);
}

void orc_move(const orc_grid *g, double dt, int64_t n, int32_t *cell, double *offs, double *phi,
              const double *u3, int32_t *alive, int32_t *m3, double *dx3) {
  Grid G;
  make_grid(g, G);
  for (int64_t p = 0; p < n; ++p) {
    int c[3] = {cell[3 * p], cell[3 * p + 1], cell[3 * p + 2]};
    double ph = phi ? phi[p] : 0.0;
    MoveOut<double> o;
    move(G, dt, c, offs + 3 * p, ph, u3 + 3 * p, o);
    for (int dd = 0; dd < 3; ++dd) {
      cell[3 * p + dd] = o.cell[dd];
      offs[3 * p + dd] = o.d[dd];
      if (m3) m3[3 * p + dd] = o.m[dd];
    }
    if (phi) phi[p] = o.phi;
    if (alive) alive[p] = o.alive ? 1 : 0;
    if (dx3) dx3[p] = o.dx3;
  }
}

// literal composition x_new = backward(forward(x, phi) + dt u/gamma), absolute code coords
void orc_move_literal(const orc_grid *g, double dt, int64_t n, const int32_t *cell,
                      const double *offs, const double *phi, const double *u3, double *xnew,
                      double *phinew) {
  Grid G;
  make_grid(g, G);
  for (int64_t p = 0; p < n; ++p) {
    double x[3], X[3];
    for (int d = 0; d < 3; ++d) x[d] = cell[3 * p + d] + offs[3 * p + d];
    const double *u = u3 + 3 * p;
    double gm = std::sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    code_to_cart(G, x, phi ? phi[p] : 0.0, X);
    for (int d = 0; d < 3; ++d) X[d] += dt * u[d] / gm;
    double ph = 0.0;
    cart_to_code(G, X, xnew + 3 * p, &ph);
    if (phinew) phinew[p] = ph;
  }
}

void orc_vay(int64_t n, double k, const double *E3, const double *B3, double *u3) {
  for (int64_t p = 0; p < n; ++p) vay(k, E3 + 3 * p, B3 + 3 * p, u3 + 3 * p);
}

void orc_gca(int64_t n, double k, const double *E3, const double *B3, double *u3) {
  for (int64_t p = 0; p < n; ++p) gca_push(k, E3 + 3 * p, B3 + 3 * p, u3 + 3 * p);
}

// field solver pieces on the padded arrays (see the field solver section)
int orc_faraday(const orc_grid *g, double *EB, double f) {
  Grid G;
  if (!make_grid(g, G)) return 1;
  faraday(G, EB, f);
  return 0;
}
int orc_ampere(const orc_grid *g, double *EB, const double *J, double dt, double coupling) {
  Grid G;
  if (!make_grid(g, G)) return 1;
  ampere(G, EB, J, dt, coupling);
  return 0;
}
int orc_filter(const orc_grid *g, double *J, int32_t passes) {
  Grid G;
  if (!make_grid(g, G)) return 1;
  for (int p = 0; p < passes; ++p) filter_pass(G, J);
  return 0;
}
double orc_polar_area(const orc_grid *g, double x1) {
  Grid G;
  if (!make_grid(g, G) || G.geom == 0) return 0.0;
  return polar_area(G, x1);
}

void orc_sort_perm(int64_t n, const int32_t *keys, int32_t *perm) {
  std::vector<int32_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int32_t a, int32_t b) { return keys[a] < keys[b]; });
  std::copy(idx.begin(), idx.end(), perm);
}

int orc_sort_keys(const orc_grid *g, int64_t n, const int32_t *cell, const int32_t *alive,
                  int32_t *keys) {
  Grid G;
  if (!make_grid(g, G)) return 1;
  for (int64_t p = 0; p < n; ++p) keys[p] = sort_key(G, cell + 3 * p, alive[p]);
  return 0;
}

// K steps of the particle step for every species (fields static).  Before step s
// (global index step0+s) the particles are stably sorted by cell (brick order,
// see sort_key) when
// sort_every > 0 and (step0+s) % sort_every == 0; dead particles go last.
// J is zeroed at the start of each step; after the call it holds the current of
// the last step.  prev positions are recorded on the last step.
int orc_run(const orc_grid *g, double dt, int32_t nsteps, int32_t sort_every, int64_t step0,
            const double *EB, int32_t nspecies, const double *q, const double *m,
            orc_species *sp, double *J) {
  return orc_run_pushers(g, dt, nsteps, sort_every, step0, EB, nspecies, q, m, nullptr, nullptr,
                         nullptr, sp, J);
}

// orc_run with a pusher per species: pusher[s] = 0 Boris, 1 Vay, +2 for the
// guiding-centre hybrid with thresholds e_ovr[s], larmor_max[s] (NULL arrays:
// Boris for every species).
int orc_run_pushers(const orc_grid *g, double dt, int32_t nsteps, int32_t sort_every,
                    int64_t step0, const double *EB, int32_t nspecies, const double *q,
                    const double *m, const int32_t *pusher, const double *e_ovr,
                    const double *larmor_max, orc_species *sp, double *J) {
  Grid G;
  if (!make_grid(g, G)) return 1;
  if (G.geom == 0)
    for (int dd = 0; dd < G.dim; ++dd)
      if (!G.periodic[dd]) return 2;
  std::vector<double> EBg(EB, EB + 6 * G.npts);
  fill_periodic_ghosts(G, EBg.data(), 6);
  std::fill(J, J + 3 * G.npts, 0.0);
  for (int32_t st = 0; st < nsteps; ++st) {
    int64_t gstep = step0 + st;
    bool last = st == nsteps - 1;
    std::fill(J, J + 3 * G.npts, 0.0);
    for (int s = 0; s < nspecies; ++s) {
      orc_species &S = sp[s];
      int64_t n = S.n;
      if (sort_every > 0 && gstep % sort_every == 0) {
        std::vector<int32_t> keys(n), perm(n);
        for (int64_t p = 0; p < n; ++p) keys[p] = sort_key(G, S.cell + 3 * p, S.alive[p]);
        orc_sort_perm(n, keys.data(), perm.data());
        PlainSpecies old = copy_in(G, S);
        for (int64_t p = 0; p < n; ++p) {
          int64_t src = perm[p];
          for (int d = 0; d < 3; ++d) {
            S.cell[3 * p + d] = old.cell[3 * src + d];
            S.offs[3 * p + d] = old.offs[3 * src + d];
            S.u[3 * p + d] = old.u[3 * src + d];
          }
          S.w[p] = old.w[src];
          if (G.geom != 0 && S.phi) S.phi[p] = old.phi[src];
          S.alive[p] = old.alive[src];
        }
        if (S.perm) std::copy(perm.begin(), perm.end(), S.perm);
      }
      for (int64_t p = 0; p < n; ++p) {
        if (last && S.cell_prev) {
          for (int d = 0; d < 3; ++d) {
            S.cell_prev[3 * p + d] = S.cell[3 * p + d];
            S.offs_prev[3 * p + d] = S.offs[3 * p + d];
          }
        }
        if (!S.alive[p]) continue;
        int cell[3] = {S.cell[3 * p], S.cell[3 * p + 1], S.cell[3 * p + 2]};
        double *d = S.offs + 3 * p;
        double *u = S.u + 3 * p;
        double ph = (G.geom != 0 && S.phi) ? S.phi[p] : 0.0;
        Pusher P;
        if (pusher) {
          P.vay = pusher[s] & 1;
          P.gca = (pusher[s] >> 1) & 1;
          P.e_ovr = e_ovr ? e_ovr[s] : 0.9;
          P.larmor_max = larmor_max ? larmor_max[s] : 0.0;
        }
        bool alive = push_particle(
            G, EBg.data(), dt, q[s], m[s], S.w[p], cell, d, u, ph, [](double *) {},
            [&](int c, int i, int j, int k, double v) { J[jidx(G, c, i, j, k)] += v; }, P);
        for (int dd = 0; dd < 3; ++dd) S.cell[3 * p + dd] = cell[dd];
        if (G.geom != 0 && S.phi) S.phi[p] = ph;
        S.alive[p] = alive ? 1 : 0;
      }
    }
  }
  return 0;
}

// Reverse-mode derivative of L = sum(lamJ * J_final) + sum(lam_u . u_final)
// + sum(lam_d . delta_final) over K steps (no sorting inside), with respect to
// the contravariant fields (periodic ghosts folded into their images), the
// initial four-velocities and the initial offsets.  Each particle-step is
// differentiated by 13-direction forward-mode duals (offsets, u, phi, and the
// six interpolated field values), and the resulting local Jacobian is applied
// transposed; the field adjoint is scattered with the interpolation weights.
int orc_adjoint(const orc_grid *g, double dt, int32_t K, const double *EB, int32_t nspecies,
                const double *q, const double *m, const orc_species *sp, const double *lamJ,
                const double *const *lam_u, const double *const *lam_d, double *dEB,
                double **du0, double **dd0, double *loss) {
  Grid G;
  if (!make_grid(g, G)) return 1;
  if (G.geom == 0)
    for (int dd = 0; dd < G.dim; ++dd)
      if (!G.periodic[dd]) return 2;
  constexpr int ND = 13;
  using D13 = Dual<ND>;
  std::vector<double> EBg(EB, EB + 6 * G.npts);
  fill_periodic_ghosts(G, EBg.data(), 6);
  std::fill(dEB, dEB + 6 * G.npts, 0.0);
  double L = 0.0;
  for (int s = 0; s < nspecies; ++s) {
    const orc_species &S = sp[s];
    int64_t n = S.n;
    // forward, storing the state before every step
    std::vector<PlainSpecies> hist;
    hist.reserve(K + 1);
    hist.push_back(copy_in(G, S));
    for (int st = 0; st < K; ++st) {
      PlainSpecies nx = hist.back();
      for (int64_t p = 0; p < n; ++p) {
        if (!nx.alive[p]) continue;
        int cell[3] = {nx.cell[3 * p], nx.cell[3 * p + 1], nx.cell[3 * p + 2]};
        double ph = nx.phi[p];
        bool lastst = st == K - 1;
        bool alive = push_particle(G, EBg.data(), dt, q[s], m[s], nx.w[p], cell,
                                   nx.offs.data() + 3 * p, nx.u.data() + 3 * p, ph,
                                   [](double *) {}, [&](int c, int i, int j, int k, double v) {
                                     if (lastst) L += lamJ[jidx(G, c, i, j, k)] * v;
                                   });
        for (int dd = 0; dd < 3; ++dd) nx.cell[3 * p + dd] = cell[dd];
        nx.phi[p] = ph;
        nx.alive[p] = alive ? 1 : 0;
      }
      hist.push_back(std::move(nx));
    }
    const PlainSpecies &fin = hist.back();
    std::vector<double> lu(3 * n, 0.0), ld(3 * n, 0.0), lphi(n, 0.0);
    for (int64_t p = 0; p < n; ++p)
      for (int a = 0; a < 3; ++a) {
        if (lam_u && lam_u[s]) {
          lu[3 * p + a] = lam_u[s][3 * p + a];
          L += lam_u[s][3 * p + a] * fin.u[3 * p + a];
        }
        if (lam_d && lam_d[s] && a < G.dim) {
          ld[3 * p + a] = lam_d[s][3 * p + a];
          L += lam_d[s][3 * p + a] * fin.offs[3 * p + a];
        }
      }
    for (int st = K - 1; st >= 0; --st) {
      const PlainSpecies &cur = hist[st];
      bool lastst = st == K - 1;
      for (int64_t p = 0; p < n; ++p) {
        if (!cur.alive[p]) continue;  // frozen: identity map
        int cell[3] = {cur.cell[3 * p], cur.cell[3 * p + 1], cur.cell[3 * p + 2]};
        D13 d[3], u[3], ph(cur.phi[p]);
        for (int a = 0; a < 3; ++a) {
          d[a] = D13(cur.offs[3 * p + a]);
          if (a < G.dim) d[a].g[a] = 1.0;
          u[a] = D13(cur.u[3 * p + a]);
          u[a].g[3 + a] = 1.0;
        }
        if (G.geom != 0) ph.g[6] = 1.0;
        double acc[ND] = {0};
        push_particle(
            G, EBg.data(), dt, q[s], m[s], cur.w[p], cell, d, u, ph,
            [](D13 *F) {
              for (int c = 0; c < 6; ++c) F[c].g[7 + c] += 1.0;
            },
            [&](int c, int i, int j, int k, const D13 &v) {
              if (!lastst) return;
              double l = lamJ[jidx(G, c, i, j, k)];
              for (int t = 0; t < ND; ++t) acc[t] += l * v.g[t];
            });
        for (int a = 0; a < 3; ++a) {
          for (int t = 0; t < ND; ++t) {
            if (a < G.dim) acc[t] += ld[3 * p + a] * d[a].g[t];
            acc[t] += lu[3 * p + a] * u[a].g[t];
          }
        }
        if (G.geom != 0)
          for (int t = 0; t < ND; ++t) acc[t] += lphi[p] * ph.g[t];
        for (int a = 0; a < 3; ++a) {
          ld[3 * p + a] = a < G.dim ? acc[a] : 0.0;
          lu[3 * p + a] = acc[3 + a];
        }
        lphi[p] = G.geom != 0 ? acc[6] : 0.0;
        int c0[3] = {cur.cell[3 * p], cur.cell[3 * p + 1], cur.cell[3 * p + 2]};
        for (int c = 0; c < 6; ++c) {
          int64_t idx[8];
          double w[8];
          interp_stencil(G, c, c0, cur.offs.data() + 3 * p, idx, w);
          for (int e = 0; e < (1 << G.dim); ++e) dEB[idx[e]] += w[e] * acc[7 + c];
        }
      }
    }
    for (int64_t p = 0; p < n; ++p)
      for (int a = 0; a < 3; ++a) {
        if (du0 && du0[s]) du0[s][3 * p + a] = lu[3 * p + a];
        if (dd0 && dd0[s]) dd0[s][3 * p + a] = ld[3 * p + a];
      }
  }
  fold_periodic_ghosts(G, dEB, 6);
  if (loss) *loss = L;
  return 0;
}

// Forward-mode directional derivative of the same L along (vEB, vu0, vd0)
// (vEB is a perturbation of the active fields; periodic ghosts follow it).
int orc_jvp(const orc_grid *g, double dt, int32_t K, const double *EB, const double *vEB,
            int32_t nspecies, const double *q, const double *m, const orc_species *sp,
            const double *const *vu0, const double *const *vd0, const double *lamJ,
            const double *const *lam_u, const double *const *lam_d, double *loss,
            double *dloss) {
  Grid G;
  if (!make_grid(g, G)) return 1;
  if (G.geom == 0)
    for (int dd = 0; dd < G.dim; ++dd)
      if (!G.periodic[dd]) return 2;
  using D1 = Dual<1>;
  std::vector<D1> F(6 * G.npts);
  for (int64_t i = 0; i < 6 * G.npts; ++i) {
    F[i] = D1(EB[i]);
    F[i].g[0] = vEB ? vEB[i] : 0.0;
  }
  fill_periodic_ghosts(G, F.data(), 6);
  D1 L(0.0);
  for (int s = 0; s < nspecies; ++s) {
    const orc_species &S = sp[s];
    for (int64_t p = 0; p < S.n; ++p) {
      if (!S.alive[p]) {
        for (int a = 0; a < 3; ++a) {
          if (lam_u && lam_u[s]) L = L + lam_u[s][3 * p + a] * S.u[3 * p + a];
          if (lam_d && lam_d[s] && a < G.dim) L = L + lam_d[s][3 * p + a] * S.offs[3 * p + a];
        }
        continue;
      }
      int cell[3] = {S.cell[3 * p], S.cell[3 * p + 1], S.cell[3 * p + 2]};
      D1 d[3], u[3], ph((G.geom != 0 && S.phi) ? S.phi[p] : 0.0);
      for (int a = 0; a < 3; ++a) {
        d[a] = D1(S.offs[3 * p + a]);
        if (vd0 && vd0[s] && a < G.dim) d[a].g[0] = vd0[s][3 * p + a];
        u[a] = D1(S.u[3 * p + a]);
        if (vu0 && vu0[s]) u[a].g[0] = vu0[s][3 * p + a];
      }
      bool alive = true;
      for (int st = 0; st < K && alive; ++st) {
        bool lastst = st == K - 1;
        alive = push_particle(G, F.data(), dt, q[s], m[s], S.w[p], cell, d, u, ph,
                              [](D1 *) {}, [&](int c, int i, int j, int k, const D1 &v) {
                                if (lastst) L = L + lamJ[jidx(G, c, i, j, k)] * v;
                              });
      }
      for (int a = 0; a < 3; ++a) {
        if (lam_u && lam_u[s]) L = L + lam_u[s][3 * p + a] * u[a];
        if (lam_d && lam_d[s] && a < G.dim) L = L + lam_d[s][3 * p + a] * d[a];
      }
    }
  }
  if (loss) *loss = L.v;
  if (dloss) *dloss = L.g[0];
  return 0;
}

}  // extern "C"
