// step_device.h -- per-particle device arithmetic of the particle step.
//
// One thread owns one particle.  Positions are (cell index, in-cell offset)
// pairs (Sec. 3.1), so the real position (i + delta) is formed only where a
// metric coefficient needs it (curvilinear grids).  Each routine names the
// passage of arXiv 2511.17710 it implements.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace picstep {

constexpr double kPI = 3.14159265358979323846;

// ---------------------------------------------------------------- precision helpers
__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_r(double x) { return 1.0 / x; }
__device__ __forceinline__ float floor_r(float x) { return floorf(x); }
__device__ __forceinline__ double floor_r(double x) { return floor(x); }
__device__ __forceinline__ void sincos_r(float x, float *s, float *c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_r(double x, double *s, double *c) { sincos(x, s, c); }
__device__ __forceinline__ float exp_r(float x) { return expf(x); }
__device__ __forceinline__ double exp_r(double x) { return exp(x); }
__device__ __forceinline__ float log1p_r(float x) { return log1pf(x); }
__device__ __forceinline__ double log1p_r(double x) { return log1p(x); }
__device__ __forceinline__ float expm1_r(float x) { return expm1f(x); }
__device__ __forceinline__ double expm1_r(double x) { return expm1(x); }
__device__ __forceinline__ float atan2_r(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double atan2_r(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }

// ---------------------------------------------------------------- cell packing
__device__ __forceinline__ void cell_decode(const GridConst &g, int32_t c, int i[3]) {
  i[0] = (c & g.mask1) - 1;
  i[1] = (c >> g.shift2) & g.mask2;
  i[2] = (c >> g.shift3) & g.mask3;
}
__device__ __forceinline__ int32_t cell_encode(const GridConst &g, const int i[3]) {
  return (int32_t)((i[0] + 1) | (i[1] << g.shift2) | (i[2] << g.shift3));
}

// key of a cell: cells brick by brick (brick index, then the cell inside the
// brick, x fastest in both), or deadkey = 1 << (keybits - 1) when dead; brick
// sides are powers of two
__device__ __forceinline__ uint32_t brick_key(const GridConst &g, int32_t c, uint32_t deadkey) {
  if (c & DEAD_BIT) return deadkey;
  const uint32_t ii[3] = {(uint32_t)((c & g.mask1) - 1), (uint32_t)((c >> g.shift2) & g.mask2),
                          (uint32_t)((c >> g.shift3) & g.mask3)};
  const int s0 = g.brick_shift[0], s1 = g.brick_shift[1], s2 = g.brick_shift[2];
  const uint32_t brick = (ii[0] >> s0) + (uint32_t)g.nbrick[0] * ((ii[1] >> s1) +
                         (uint32_t)g.nbrick[1] * (ii[2] >> s2));
  const uint32_t local = (ii[0] & ((1u << s0) - 1)) | ((ii[1] & ((1u << s1) - 1)) << s0) |
                         ((ii[2] & ((1u << s2) - 1)) << (s0 + s1));
  return (brick << (s0 + s1 + s2)) | local;
}

// block -> (species, local index): blocks never straddle species
__device__ __forceinline__ bool locate(const SpeciesTable &sp, int &s, int64_t &local) {
  const int64_t b = blockIdx.x;
  s = 0;
#pragma unroll
  for (int t = 1; t < MAXSP; ++t)
    if (t < sp.nspec && b >= sp.blk0[t]) s = t;
  local = (b - sp.blk0[s]) * BLOCK + threadIdx.x;
  return local < sp.n[s];
}

// padded element index (the host guarantees 6 * npts < 2^31)
__device__ __forceinline__ int pad_index(const GridConst &g, int i, int j, int k, int dim) {
  const int kk = (dim == 3) ? (k + NG) : 0;
  return (i + NG) + g.np[0] * ((j + NG) + g.np[1] * kk);
}

// ---------------------------------------------------------------- step 3: interpolation
// First-order shape on each component's own Yee lattice (Sec. 2.3 step 3,
// App. A staggering).  Per dimension two weight sets exist: unstaggered
// (base i, weight delta) and half-staggered (xi = delta - 1/2; base i or
// i - 1 with weight xi or xi + 1).
template <class Real>
struct Stencil1 {
  int b0, bh;     // bases (unpadded)
  Real f0, fh;    // weights of the upper point
};

template <class Real>
__device__ __forceinline__ Stencil1<Real> stencil1(int i, Real d) {
  Stencil1<Real> s;
  s.b0 = i;
  s.f0 = d;
  Real xi = d - (Real)0.5;
  if (xi < (Real)0) {
    s.bh = i - 1;
    s.fh = xi + (Real)1;
  } else {
    s.bh = i;
    s.fh = xi;
  }
  return s;
}

// stagger flags (x, y, z) of E1, E2, E3, B1, B2, B3
__device__ constexpr int kStag[6][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                                        {0, 1, 1}, {1, 0, 1}, {1, 1, 0}};

// first-order interpolation from the lattice values around A[base] (row
// stride s1, plane stride s2): global memory or an LDS tile
template <int DIM, class Real>
__device__ __forceinline__ Real gather_at(const Real *__restrict__ A, int base, int s1, int s2,
                                          Real fx, Real fy, Real fz) {
  const Real gx = (Real)1 - fx, gy = (Real)1 - fy;
  Real v = gy * (gx * A[base] + fx * A[base + 1]) + fy * (gx * A[base + s1] + fx * A[base + s1 + 1]);
  if (DIM == 3) {
    Real v1 = gy * (gx * A[base + s2] + fx * A[base + s2 + 1]) +
              fy * (gx * A[base + s2 + s1] + fx * A[base + s2 + s1 + 1]);
    v = ((Real)1 - fz) * v + fz * v1;
  }
  return v;
}

template <int DIM, class Real>
__device__ __forceinline__ Real gather_one(const Real *__restrict__ A, const GridConst &g, int bx,
                                           int by, int bz, Real fx, Real fy, Real fz) {
  return gather_at<DIM, Real>(A, pad_index(g, bx, by, bz, DIM), g.np[0], g.np[0] * g.np[1], fx,
                              fy, fz);
}

template <int DIM, class Real>
__device__ __forceinline__ void interp6(const Real *__restrict__ EB, const GridConst &g,
                                        const Stencil1<Real> st[3], Real F[6]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const int sx = kStag[c][0], sy = kStag[c][1], sz = kStag[c][2];
    const int bx = sx ? st[0].bh : st[0].b0;
    const int by = sy ? st[1].bh : st[1].b0;
    const int bz = (DIM == 3) ? (sz ? st[2].bh : st[2].b0) : 0;
    const Real fx = sx ? st[0].fh : st[0].f0;
    const Real fy = sy ? st[1].fh : st[1].f0;
    const Real fz = (DIM == 3) ? (sz ? st[2].fh : st[2].f0) : (Real)0;
    F[c] = gather_one<DIM, Real>(EB + c * (int)g.npts, g, bx, by, bz, fx, fy, fz);
  }
}

// A block's copy of the six field components over a box of cells (LDS):
// component c, tile cell (x, y, z) at F[c*T + x + sy*y + sz*z]; o is the box
// origin in (unwrapped) cell coordinates.
template <class Real>
struct FieldTile {
  const Real *F;
  int T, sy, sz;
  int o[3], ts[3];
};

// every point of the interpolation stencil of cell ib (i-1 ... i+1) inside the tile
template <int DIM, class Real>
__device__ __forceinline__ bool fields_in_tile(const FieldTile<Real> &t, const int ib[3]) {
  bool in = true;
#pragma unroll
  for (int a = 0; a < DIM; ++a) in = in && (ib[a] - 1 >= t.o[a]) && (ib[a] + 1 < t.o[a] + t.ts[a]);
  return in;
}

// interp6 from the tile; dsh = unwrapped minus stored cell coordinates
template <int DIM, class Real>
__device__ __forceinline__ void interp6_tile(const FieldTile<Real> &t, const int dsh[3],
                                             const Stencil1<Real> st[3], Real F[6]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const int sx = kStag[c][0], sy = kStag[c][1], sz = kStag[c][2];
    const int bx = (sx ? st[0].bh : st[0].b0) + dsh[0] - t.o[0];
    const int by = (sy ? st[1].bh : st[1].b0) + dsh[1] - t.o[1];
    const int bz = (DIM == 3) ? (sz ? st[2].bh : st[2].b0) + dsh[2] - t.o[2] : 0;
    const Real fx = sx ? st[0].fh : st[0].f0;
    const Real fy = sy ? st[1].fh : st[1].f0;
    const Real fz = (DIM == 3) ? (sz ? st[2].fh : st[2].f0) : (Real)0;
    F[c] = gather_at<DIM, Real>(t.F + c * t.T, bx + t.sy * by + t.sz * bz, t.sy, t.sz, fx, fy, fz);
  }
}

// ---------------------------------------------------------------- step 5: Boris
// Relativistic Boris push (Boris 1970) of eq. curvspace-equations-of-motion,
// k = q dt / (2 m rho0): half electric kick, magnetic rotation, half kick.
// The intermediates, for the reverse sweep.
template <class Real>
struct BorisRec {
  Real um[3], igm, t[3], tt, sf, s[3], up[3];
};

template <class Real>
__device__ __forceinline__ void boris_rec(Real k, const Real E[3], const Real B[3], Real u[3],
                                          BorisRec<Real> &R) {
  Real um0 = u[0] + k * E[0], um1 = u[1] + k * E[1], um2 = u[2] + k * E[2];
  Real ig = rsqrt_r((Real)1 + um0 * um0 + um1 * um1 + um2 * um2);
  Real t0 = k * B[0] * ig, t1 = k * B[1] * ig, t2 = k * B[2] * ig;
  Real tt = t0 * t0 + t1 * t1 + t2 * t2;
  Real sf = (Real)2 * rcp_r((Real)1 + tt);
  Real s0 = t0 * sf, s1 = t1 * sf, s2 = t2 * sf;
  Real up0 = um0 + (um1 * t2 - um2 * t1);
  Real up1 = um1 + (um2 * t0 - um0 * t2);
  Real up2 = um2 + (um0 * t1 - um1 * t0);
  u[0] = um0 + (up1 * s2 - up2 * s1) + k * E[0];
  u[1] = um1 + (up2 * s0 - up0 * s2) + k * E[1];
  u[2] = um2 + (up0 * s1 - up1 * s0) + k * E[2];
  R.um[0] = um0; R.um[1] = um1; R.um[2] = um2;
  R.igm = ig;
  R.t[0] = t0; R.t[1] = t1; R.t[2] = t2;
  R.tt = tt;
  R.sf = sf;
  R.s[0] = s0; R.s[1] = s1; R.s[2] = s2;
  R.up[0] = up0; R.up[1] = up1; R.up[2] = up2;
}

template <class Real>
__device__ __forceinline__ void boris(Real k, const Real E[3], const Real B[3], Real u[3]) {
  BorisRec<Real> R;
  boris_rec(k, E, B, u, R);
}

// Vay (2008) pusher: u_new = u + (q dt/m)(E + vbar x B), vbar the mean of the
// velocities before and after the step, with the new Lorentz factor from the
// closed-form root of that implicit relation; (q dt/m) E = 2kE and
// (q dt/m)(v/2) x B = k v x B in code units.  It keeps the relativistic
// E x B drift exactly, which Boris's rotation does not.
template <class Real>
__device__ __forceinline__ void vay(Real k, const Real E[3], const Real B[3], Real u[3]) {
  const Real ig0 = rsqrt_r((Real)1 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const Real v0 = u[0] * ig0, v1 = u[1] * ig0, v2 = u[2] * ig0;
  const Real w0 = u[0] + (Real)2 * k * E[0] + k * (v1 * B[2] - v2 * B[1]);
  const Real w1 = u[1] + (Real)2 * k * E[1] + k * (v2 * B[0] - v0 * B[2]);
  const Real w2 = u[2] + (Real)2 * k * E[2] + k * (v0 * B[1] - v1 * B[0]);
  const Real t0 = k * B[0], t1 = k * B[1], t2 = k * B[2];
  const Real us = w0 * t0 + w1 * t1 + w2 * t2;
  const Real tau2 = t0 * t0 + t1 * t1 + t2 * t2;
  const Real sig = (Real)1 + w0 * w0 + w1 * w1 + w2 * w2 - tau2;
  const Real gn = sqrt_r((Real)0.5 * (sig + sqrt_r(sig * sig + (Real)4 * (tau2 + us * us))));
  const Real ign = (Real)1 / gn;
  const Real a0 = t0 * ign, a1 = t1 * ign, a2 = t2 * ign;
  const Real sf = (Real)1 / ((Real)1 + a0 * a0 + a1 * a1 + a2 * a2);
  const Real wa = w0 * a0 + w1 * a1 + w2 * a2;
  u[0] = sf * (w0 + wa * a0 + (w1 * a2 - w2 * a1));
  u[1] = sf * (w1 + wa * a1 + (w2 * a0 - w0 * a2));
  u[2] = sf * (w2 + wa * a2 + (w0 * a1 - w1 * a0));
}

// Hybrid pusher (Sec. 5.2): a particle whose fields are drift dominated
// (|E| < e_ovr |B|) and whose nominal gyroradius |u| m rho0 / (|q| |B|) =
// |u| dt / (2 |k| |B|) is below the critical length follows its guiding
// centre: the momentum perpendicular to B is dropped, the parallel
// four-velocity takes the kick 2k E.b, and u = u_par b + gamma v_E with
// v_E = E x B / B^2 and gamma = sqrt((1 + u_par^2) / (1 - v_E^2)).  The
// regime test is taken in FP64.
template <class Real>
__device__ __forceinline__ bool gca_regime(double k, double dt, double e_ovr, double larmor_max,
                                           const Real E[3], const Real B[3], const Real u[3]) {
  const double e2 = (double)E[0] * E[0] + (double)E[1] * E[1] + (double)E[2] * E[2];
  const double b2 = (double)B[0] * B[0] + (double)B[1] * B[1] + (double)B[2] * B[2];
  if (!(b2 > 0.0) || !(e2 < e_ovr * e_ovr * b2)) return false;
  const double ua = sqrt((double)u[0] * u[0] + (double)u[1] * u[1] + (double)u[2] * u[2]);
  return ua * dt / (2.0 * fabs(k) * sqrt(b2)) < larmor_max;
}

template <class Real>
__device__ __forceinline__ void gca_push(Real k, const Real E[3], const Real B[3], Real u[3]) {
  const Real b2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  const Real ib = rsqrt_r(b2), ib2 = (Real)1 / b2;
  const Real bx = B[0] * ib, by = B[1] * ib, bz = B[2] * ib;
  const Real e0 = (E[1] * B[2] - E[2] * B[1]) * ib2;
  const Real e1 = (E[2] * B[0] - E[0] * B[2]) * ib2;
  const Real e2 = (E[0] * B[1] - E[1] * B[0]) * ib2;
  const Real up = u[0] * bx + u[1] * by + u[2] * bz + (Real)2 * k * (E[0] * bx + E[1] * by + E[2] * bz);
  const Real ve2 = e0 * e0 + e1 * e1 + e2 * e2;
  const Real gm = sqrt_r(((Real)1 + up * up) / ((Real)1 - ve2));
  u[0] = up * bx + gm * e0;
  u[1] = up * by + gm * e1;
  u[2] = up * bz + gm * e2;
}

// The species' pusher (SpeciesTable::pusher: 0 Boris, 1 Vay, +2 the
// guiding-centre hybrid).
template <class Real>
__device__ __forceinline__ void push_momentum(const SpeciesTable &sp, int s, Real k, double dt,
                                              const Real E[3], const Real B[3], Real u[3]) {
  const int pk = sp.pusher[s];
  if ((pk & 2) && gca_regime<Real>(sp.k[s], dt, sp.gca_e_ovr[s], sp.gca_larmor[s], E, B, u)) {
    gca_push(k, E, B, u);
  } else if (pk & 1) {
    vay(k, E, B, u);
  } else {
    boris(k, E, B, u);
  }
}

// Reverse of the Boris push ("reverse Boris rotation"): dL/du_new -> dL/du,
// dL/dE, dL/dB (global Cartesian), from the recorded intermediates.
template <class Real>
__device__ __forceinline__ void boris_rev(Real k, const BorisRec<Real> &R, const Real unb[3],
                                          Real ub[3], Real Eb[3], Real Bb[3]) {
  const Real *um = R.um, *t = R.t, *s3 = R.s, *up = R.up;
  Real umb[3], upb[3], sb[3], tb[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Eb[a] = k * unb[a];  // u+ = u+' + k E
    umb[a] = unb[a];     // u+' = um + up x s
  }
  // up x s: upb += s x unb, sb = unb x up
  upb[0] = s3[1] * unb[2] - s3[2] * unb[1];
  upb[1] = s3[2] * unb[0] - s3[0] * unb[2];
  upb[2] = s3[0] * unb[1] - s3[1] * unb[0];
  sb[0] = unb[1] * up[2] - unb[2] * up[1];
  sb[1] = unb[2] * up[0] - unb[0] * up[2];
  sb[2] = unb[0] * up[1] - unb[1] * up[0];
  // up = um + um x t: umb += upb + t x upb, tb = upb x um
#pragma unroll
  for (int a = 0; a < 3; ++a) umb[a] += upb[a];
  umb[0] += t[1] * upb[2] - t[2] * upb[1];
  umb[1] += t[2] * upb[0] - t[0] * upb[2];
  umb[2] += t[0] * upb[1] - t[1] * upb[0];
  tb[0] = upb[1] * um[2] - upb[2] * um[1];
  tb[1] = upb[2] * um[0] - upb[0] * um[2];
  tb[2] = upb[0] * um[1] - upb[1] * um[0];
  // s = t sf, sf = 2 / (1 + t.t)
  const Real ts = t[0] * sb[0] + t[1] * sb[1] + t[2] * sb[2];
  const Real c4 = (Real)4 / (((Real)1 + R.tt) * ((Real)1 + R.tt));
#pragma unroll
  for (int a = 0; a < 3; ++a) tb[a] += R.sf * sb[a] - c4 * t[a] * ts;
  // t = k B / gm
  Real gmb = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Bb[a] = k * R.igm * tb[a];
    gmb -= t[a] * tb[a] * R.igm;
  }
  // gm = sqrt(1 + um.um); um = u + k E
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    umb[a] += gmb * um[a] * R.igm;
    Eb[a] += k * umb[a];
    ub[a] = umb[a];
  }
}

// Cartesian in-cell displacement dt u_a / (gamma Delta_a) (steps 6-7); the
// FP32 build multiplies by the reciprocal spacing, the FP64 build divides
// (it matches the reference's rounding).  The forward and the adjoint
// recompute share this routine, so both take the same step.
__device__ __forceinline__ float cart_disp(const GridConst &g, int a, float dt, float u, float gi) {
  return dt * u * gi * g.inv_dxf[a];
}

// A double constant in the storage precision: its host-rounded FP32 copy in
// FP32 contexts (equal to a conversion on the device, both round to
// nearest, but read from scalar registers), the double itself in FP64 ones.
template <class Real>
__device__ __forceinline__ Real konst(double d, float f);
template <>
__device__ __forceinline__ float konst<float>(double, float f) { return f; }
template <>
__device__ __forceinline__ double konst<double>(double d, float) { return d; }
__device__ __forceinline__ double cart_disp(const GridConst &g, int a, double dt, double u,
                                            double gi) {
  return dt * u * gi / g.dx[a];
}

// ---------------------------------------------------------------- positions
// Offset codec and canonicalisation (cell index + offset in [0,1), Sec. 3.1).
// FP32 build: the offset is q * 2^-32; the weights use it rounded to float,
// while the move and the zig-zag segments work on its exact value in FP64, so
// a displacement is never rounded to the float resolution of the offset.
template <class Real>
struct Pos;

template <>
struct Pos<float> {
  using S = uint32_t;
  static __device__ __forceinline__ float weight(S q) { return (float)q * 0x1p-32f; }
  static __device__ __forceinline__ double exact(S q) { return (double)q * 0x1p-32; }
  // new offset and cell step for a displacement dx (|dx| < 1)
  static __device__ __forceinline__ int move(S q, double dx, S &qn) {
    const double y = exact(q) + dx;
    double fl = floor(y);
    // |dx| < 1 under the CFL bound checked by the host; the clamp only keeps
    // every deposit index inside the ghost layer should that ever fail
    fl = fmin(fmax(fl, -1.0), 1.0);
    double r = rint((y - fl) * 0x1p32);
    r = fmin(fmax(r, 0.0), 0x1p32);
    if (r >= 0x1p32) {  // rounded onto the upper face: next cell, offset 0
      r = 0.0;
      fl += 1.0;
    }
    qn = (S)r;
    return (int)fl;
  }
};

template <>
struct Pos<double> {
  using S = double;
  static __device__ __forceinline__ double weight(S d) { return d; }
  static __device__ __forceinline__ double exact(S d) { return d; }
  static __device__ __forceinline__ int move(S d, double dx, S &dn) {
    const double y = d + dx;
    double fl = floor(y);
    fl = fmin(fmax(fl, -1.0), 1.0);
    double r = y - fl;
    if (r >= 1.0) {  // y - floor(y) rounded up to 1
      fl += 1.0;
      r = 0.0;
    }
    dn = r;
    return (int)fl;
  }
};

template <class Real>
__device__ __forceinline__ OffT<Real> largest_offset();
template <>
__device__ __forceinline__ uint32_t largest_offset<float>() { return 0xffffffffu; }
template <>
__device__ __forceinline__ double largest_offset<double>() { return 0x1.fffffffffffffp-1; }

// ---------------------------------------------------------------- step 8: zig-zag
// Umeda et al. (2003) zig-zag on in-cell offsets (Sec. 3.2 footnote): per
// dimension a = old offset, b = new offset + m measured from the old cell,
// relay x_r = min(min(0,m)+1, max(max(0,m),(a+b)/2)); segment 1 in the old
// cell, segment 2 in the new one.  Each segment deposits the exact flux of
// the first-order shape along its straight path (midpoint weights plus the
// F_a F_b / 12 cross term), so div J + d(rho)/dt = 0 holds exactly (eq.
// curvspace-chargecons-2).
template <class Real>
struct ZigZag {
  Real F[2][3];
  Real W[2][3];
};

// the whole in-cell step a -> b as segment 0 (used when m = 0 in every dimension)
template <int DIM, class Real>
__device__ __forceinline__ void straight(const double a[3], const double b[3], ZigZag<Real> &z) {
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    z.F[0][d] = (Real)(b[d] - a[d]);
    z.W[0][d] = (Real)((a[d] + b[d]) * 0.5);
  }
}

// a, b: exact old offset and new offset + m (both measured from the old cell)
template <int DIM, class Real>
__device__ __forceinline__ void zigzag(const double a[3], const int m[3], const double b[3],
                                       ZigZag<Real> &z) {
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double lo = (double)(min(0, m[d]) + 1);
    const double hi = (double)max(0, m[d]);
    const double mid = (a[d] + b[d]) * 0.5;
    const double xr = fmin(lo, fmax(hi, mid));
    z.F[0][d] = (Real)(xr - a[d]);
    z.F[1][d] = (Real)(b[d] - xr);
    z.W[0][d] = (Real)((a[d] + xr) * 0.5);
    z.W[1][d] = (Real)((xr + b[d]) * 0.5 - (double)m[d]);
  }
}

__device__ __forceinline__ void atomic_add_r(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_r(double *p, double v) { unsafeAtomicAdd(p, v); }

// LDS accumulator of a block's current tile.  FP32 builds accumulate in
// 64-bit fixed point: every contribution is computed in float from a
// coefficient pre-scaled by a power of two (so the float rounding is the
// unscaled one), rounded to an integer and added with an integer LDS atomic.
// The integer sum is exact and independent of the order of the adds, and on
// gfx950 integer LDS atomics run several times faster than float ones.  FP64
// builds accumulate in double.
template <class Real>
struct TileAcc { using type = Real; };
template <>
struct TileAcc<float> { using type = long long; };

// round-to-nearest of a float v with |v| < 2^51: adding 1.5 * 2^52 in double
// puts round(v) in the low mantissa bits of a number whose exponent is fixed
__device__ __forceinline__ long long fixed_round(float v) {
  const double d = (double)v + 0x1.8p52;
  return __double_as_longlong(d) - 0x4338000000000000LL;
}
// coefficient of a contribution to a tile: scaled by 2^esc for the
// fixed-point accumulator of FP32 builds (exact power-of-two scaling)
__device__ __forceinline__ float tile_coef(float C, int esc) { return ldexpf(C, esc); }
__device__ __forceinline__ double tile_coef(double C, int) { return C; }

__device__ __forceinline__ void atomic_add_r(long long *p, float v) {
  atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)fixed_round(v));
}

// Where a deposit lands: the global current (padded layout) or a block's LDS
// tile; element (I, J, K) of component c sits at
// c*cs + (I - o0) + sy*(J - o1) + sz*(K - o2).
template <class Acc>
struct DepTarget {
  Acc *J;
  int cs, sy, sz;
  int o[3];
};

// Scatter of the two zig-zag segments (indices may reach the ghost layer of
// the global array; periodic ghosts are folded after the step).
// nseg = 1: a step that stays in its cell is one straight segment (the two
// collinear halves of the zig-zag carry, summed, exactly its flux).
template <int DIM, class Real, class Acc, class Z>
__device__ __forceinline__ void deposit(const DepTarget<Acc> &t, Real C, const int i0[3],
                                        const int m[3], const ZigZag<Z> &z, Real dx3,
                                        int nseg = 2) {
  const int cs = t.cs, sy = t.sy, sz = t.sz;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (s >= nseg) break;
    const int I = i0[0] + (s ? m[0] : 0) - t.o[0];
    const int Jc = i0[1] + (s ? m[1] : 0) - t.o[1];
    const int K = (DIM == 3) ? i0[2] + (s ? m[2] : 0) - t.o[2] : 0;
    const int base = I + sy * Jc + sz * K;
    const Real Fx = (Real)z.F[s][0], Fy = (Real)z.F[s][1];
    const Real Wx = (Real)z.W[s][0], Wy = (Real)z.W[s][1];
    if (DIM == 2) {
      const Real cx = C * Fx, cy = C * Fy;
      atomic_add_r(t.J + base, cx * ((Real)1 - Wy));
      atomic_add_r(t.J + base + sy, cx * Wy);
      atomic_add_r(t.J + cs + base, cy * ((Real)1 - Wx));
      atomic_add_r(t.J + cs + base + 1, cy * Wx);
      const Real h = C * dx3 * (nseg == 1 ? (Real)1 : (Real)0.5);  // dx3 shared by the segments
      const Real cxy = Fx * Fy * (Real)(1.0 / 12.0);
      Acc *J3 = t.J + 2 * cs + base;
      atomic_add_r(J3, h * (((Real)1 - Wx) * ((Real)1 - Wy) + cxy));
      atomic_add_r(J3 + 1, h * (Wx * ((Real)1 - Wy) - cxy));
      atomic_add_r(J3 + sy, h * (((Real)1 - Wx) * Wy - cxy));
      atomic_add_r(J3 + sy + 1, h * (Wx * Wy + cxy));
    } else {
      const Real Fz = (Real)z.F[s][2], Wz = (Real)z.W[s][2];
      const Real cx = C * Fx, cy = C * Fy, cz = C * Fz;
      const Real cyz = Fy * Fz * (Real)(1.0 / 12.0);
      const Real cxz = Fx * Fz * (Real)(1.0 / 12.0);
      const Real cxy = Fx * Fy * (Real)(1.0 / 12.0);
      const Real gx = (Real)1 - Wx, gy = (Real)1 - Wy, gz = (Real)1 - Wz;
      Acc *J1 = t.J + base;
      atomic_add_r(J1, cx * (gy * gz + cyz));
      atomic_add_r(J1 + sy, cx * (Wy * gz - cyz));
      atomic_add_r(J1 + sz, cx * (gy * Wz - cyz));
      atomic_add_r(J1 + sz + sy, cx * (Wy * Wz + cyz));
      Acc *J2 = t.J + cs + base;
      atomic_add_r(J2, cy * (gx * gz + cxz));
      atomic_add_r(J2 + 1, cy * (Wx * gz - cxz));
      atomic_add_r(J2 + sz, cy * (gx * Wz - cxz));
      atomic_add_r(J2 + sz + 1, cy * (Wx * Wz + cxz));
      Acc *J3 = t.J + 2 * cs + base;
      atomic_add_r(J3, cz * (gx * gy + cxy));
      atomic_add_r(J3 + 1, cz * (Wx * gy - cxy));
      atomic_add_r(J3 + sy, cz * (gx * Wy - cxy));
      atomic_add_r(J3 + sy + 1, cz * (Wx * Wy + cxy));
    }
  }
}

// The same scatter into the fixed-point tile of FP32 builds, in FP64 from the
// exact segment data: each contribution c*s is rounded to an integer by one
// fused multiply-add onto 1.5*2^52 (|c*s| < 2^51), so it costs two FP64
// operations and an integer add; C carries the tile's 2^esc scale.
__device__ __forceinline__ void fixed_add(long long *p, double c, double s) {
  const long long v = __double_as_longlong(fma(c, s, 0x1.8p52)) - 0x4338000000000000LL;
  atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}

template <int DIM>
__device__ __forceinline__ void deposit_fixed(const DepTarget<long long> &t, double C,
                                              const int i0[3], const int m[3],
                                              const ZigZag<double> &z, double dx3, int nseg) {
  const int cs = t.cs, sy = t.sy, sz = t.sz;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (s >= nseg) break;
    const int I = i0[0] + (s ? m[0] : 0) - t.o[0];
    const int Jc = i0[1] + (s ? m[1] : 0) - t.o[1];
    const int K = (DIM == 3) ? i0[2] + (s ? m[2] : 0) - t.o[2] : 0;
    const int base = I + sy * Jc + sz * K;
    const double Fx = z.F[s][0], Fy = z.F[s][1];
    const double Wx = z.W[s][0], Wy = z.W[s][1];
    const double gx = 1.0 - Wx, gy = 1.0 - Wy;
    if (DIM == 2) {
      const double cx = C * Fx, cy = C * Fy;
      fixed_add(t.J + base, cx, gy);
      fixed_add(t.J + base + sy, cx, Wy);
      fixed_add(t.J + cs + base, cy, gx);
      fixed_add(t.J + cs + base + 1, cy, Wx);
      const double h = C * dx3 * (nseg == 1 ? 1.0 : 0.5);  // dx3 shared by the segments
      const double cxy = Fx * Fy * (1.0 / 12.0);
      long long *J3 = t.J + 2 * cs + base;
      fixed_add(J3, h, fma(gx, gy, cxy));
      fixed_add(J3 + 1, h, fma(Wx, gy, -cxy));
      fixed_add(J3 + sy, h, fma(gx, Wy, -cxy));
      fixed_add(J3 + sy + 1, h, fma(Wx, Wy, cxy));
    } else {
      const double Fz = z.F[s][2], Wz = z.W[s][2], gz = 1.0 - Wz;
      const double cx = C * Fx, cy = C * Fy, cz = C * Fz;
      const double cyz = Fy * Fz * (1.0 / 12.0);
      const double cxz = Fx * Fz * (1.0 / 12.0);
      const double cxy = Fx * Fy * (1.0 / 12.0);
      long long *J1 = t.J + base;
      fixed_add(J1, cx, fma(gy, gz, cyz));
      fixed_add(J1 + sy, cx, fma(Wy, gz, -cyz));
      fixed_add(J1 + sz, cx, fma(gy, Wz, -cyz));
      fixed_add(J1 + sz + sy, cx, fma(Wy, Wz, cyz));
      long long *J2 = t.J + cs + base;
      fixed_add(J2, cy, fma(gx, gz, cxz));
      fixed_add(J2 + 1, cy, fma(Wx, gz, -cxz));
      fixed_add(J2 + sz, cy, fma(gx, Wz, -cxz));
      fixed_add(J2 + sz + 1, cy, fma(Wx, Wz, cxz));
      long long *J3 = t.J + 2 * cs + base;
      fixed_add(J3, cz, fma(gx, gy, cxy));
      fixed_add(J3 + 1, cz, fma(Wx, gy, -cxy));
      fixed_add(J3 + sy, cz, fma(gx, Wy, -cxy));
      fixed_add(J3 + sy + 1, cz, fma(Wx, Wy, cxy));
    }
  }
}

// ---------------------------------------------------------------- axisymmetric metric + move
// Metric of Sec. 2.4 at code coordinates, evaluated in precision CT.
template <class CT>
struct AxiMetric {
  CT r, th, h1, h2, h3, st, ct;
};

template <int GEOM, class CT>
__device__ __forceinline__ AxiMetric<CT> axi_metric(const GridConst &g, CT x1, CT x2) {
  AxiMetric<CT> M;
  if (GEOM == 1) {
    M.r = (CT)g.rmin + x1 * (CT)g.dr;
    M.th = x2 * (CT)g.dth;
    M.h1 = (CT)g.dr;
    M.h2 = M.r * (CT)g.dth;
  } else {
    const CT eR = exp_r((CT)g.Rmin + x1 * (CT)g.dR);
    M.r = (CT)g.r0 + eR;
    const CT T = x2 * (CT)g.dT;
    const CT tp = T * (CT)(1.0 / kPI);
    const CT vt = (CT)g.vt;
    M.th = T + (CT)2 * vt * T * ((CT)1 - (CT)2 * tp) * ((CT)1 - tp);
    const CT thT = (CT)1 + (CT)2 * vt + (CT)12 * vt * tp * (tp - (CT)1);
    M.h1 = (CT)g.dR * eR;
    M.h2 = (CT)g.dT * thT * M.r;
  }
  sincos_r(M.th, &M.st, &M.ct);
  M.h3 = M.r * M.st;
  return M;
}

// Offset-relative evaluation of backward(forward(x^n) + dX) (Sec. 2.3 steps
// 6-7 with the Sec. 2.4 maps), in the local frame rotated to the particle's
// azimuth: returns code displacements and the azimuth step.
template <int GEOM, class CT>
__device__ __forceinline__ void axi_move(const GridConst &g, const AxiMetric<CT> &M, CT x2,
                                         CT sp, CT cp, CT DX, CT DY, CT DZ, CT &dx1, CT &dx2,
                                         CT &dphi) {
  const CT Dr = DX * cp + DY * sp;   // cylindrical radial
  const CT Dp = DY * cp - DX * sp;   // azimuthal
  const CT rho_o = M.r * M.st, z_o = M.r * M.ct;
  const CT D2 = DX * DX + DY * DY + DZ * DZ;
  const CT ir2 = (CT)1 / (M.r * M.r);
  const CT sig = ((CT)2 * (rho_o * Dr + z_o * DZ) + D2) * ir2;
  const CT hl = (CT)0.5 * log1p_r(sig);  // log(r_new / r_old)
  const CT rx = rho_o + Dr;
  const CT rho_n = sqrt_r(rx * rx + Dp * Dp);
  const CT z_n = z_o + DZ;
  CT dth;
  if (rho_n + rho_o > (CT)0) {
    const CT drho = ((CT)2 * rho_o * Dr + Dr * Dr + Dp * Dp) / (rho_n + rho_o);
    dth = atan2_r(drho * z_o - DZ * rho_o, rho_o * rho_n + z_o * z_n);
  } else {
    dth = ((CT)(kPI / 2) - atan2_r(z_n, rho_n)) - M.th;
  }
  dphi = atan2_r(Dp, rx);
  if (GEOM == 1) {
    dx1 = M.r * expm1_r(hl) * (CT)(1.0 / g.dr);
    dx2 = dth * (CT)(1.0 / g.dth);
  } else {
    if (g.r0 == 0.0)
      dx1 = hl * (CT)(1.0 / g.dR);
    else
      dx1 = log1p_r(M.r * expm1_r(hl) / (M.r - (CT)g.r0)) * (CT)(1.0 / g.dR);
    // theta(T0 + s) - theta(T0) = a1 s + a2 s^2 + a3 s^3 = dth, Newton from dth/a1
    const CT T0 = x2 * (CT)g.dT;
    const CT tp = T0 * (CT)(1.0 / kPI);
    const CT vt = (CT)g.vt;
    const CT a1 = (CT)1 + (CT)2 * vt + (CT)12 * vt * tp * (tp - (CT)1);
    const CT a2 = (CT)(6.0 / (kPI * kPI)) * vt * ((CT)2 * T0 - (CT)kPI);
    const CT a3 = (CT)(4.0 / (kPI * kPI)) * vt;
    CT s = dth / a1;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const CT f = ((a3 * s + a2) * s + a1) * s - dth;
      const CT fp = ((CT)3 * a3 * s + (CT)2 * a2) * s + a1;
      s = s - f / fp;
    }
    dx2 = s * (CT)(1.0 / g.dT);
  }
}


// Tetrad and rotation (Sec. 2.3 step 4): F^i_hat = sqrt(h_ii) F^i at x_p
// (eq. curvspace-tetradtrans), then (r, theta, phi)_hat -> (x, y, z)_hat at
// the particle's theta and azimuth.
template <class CT, class Real>
__device__ __forceinline__ void axi_to_cart(const AxiMetric<CT> &M, CT sp, CT cp, const Real F[6],
                                            Real E[3], Real B[3]) {
  const CT h[3] = {M.h1, M.h2, M.h3};
  CT Fh[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) Fh[c] = (CT)F[c] * h[c % 3];
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    const CT a = Fh[3 * f], b = Fh[3 * f + 1], cc = Fh[3 * f + 2];
    const CT ax = a * M.st + b * M.ct;  // cylindrical radial component
    Real *out = f ? B : E;
    out[0] = (Real)(ax * cp - cc * sp);
    out[1] = (Real)(ax * sp + cc * cp);
    out[2] = (Real)(a * M.ct - b * M.st);
  }
}

// Axisymmetric particle (Sec. 2.3 steps 4-7): tetrad and rotation, Boris in
// the global basis, offset-relative move.  Metric and move run in CT (FP64
// near the axis and r_min when Real is float).
// PUSHERS: the species may use another pusher than Boris (push_momentum).
template <int GEOM, class CT, class Real, class D, bool PUSHERS = false>
__device__ __forceinline__ void axi_particle(const GridConst &g, const SpeciesTable &sp, int s,
                                             double dt, int i1, int i2, D d1, D d2, Real phi,
                                             const Real F[6], Real u[3], CT &dx1, CT &dx2,
                                             CT &dphi) {
  const Real k = konst<Real>(sp.k[s], sp.kf[s]);
  const CT x1 = (CT)i1 + (CT)d1;
  const CT x2 = (CT)i2 + (CT)d2;
  const AxiMetric<CT> M = axi_metric<GEOM, CT>(g, x1, x2);
  CT sp_, cp;
  sincos_r((CT)phi, &sp_, &cp);
  Real E[3], B[3];
  axi_to_cart<CT, Real>(M, sp_, cp, F, E, B);
  if (PUSHERS)
    push_momentum<Real>(sp, s, k, dt, E, B, u);
  else
    boris(k, E, B, u);
  const CT uu0 = (CT)u[0], uu1 = (CT)u[1], uu2 = (CT)u[2];
  const CT gi = rsqrt_r((CT)1 + uu0 * uu0 + uu1 * uu1 + uu2 * uu2);
  const CT dtg = (CT)dt * gi;
  axi_move<GEOM, CT>(g, M, x2, sp_, cp, dtg * uu0, dtg * uu1, dtg * uu2, dx1, dx2, dphi);
}

template <class Real, class CT>
__device__ __forceinline__ Real next_phi(Real phi, CT dphi) {
  CT pn = (CT)phi + dphi;
  const CT twopi = (CT)(2.0 * kPI);
  if (pn < (CT)0) pn += twopi;
  if (pn >= twopi) pn -= twopi;
  Real pr = (Real)pn;
  if (pr >= (Real)(2.0 * kPI)) pr = (Real)0;
  return pr;
}

// ---------------------------------------------------------------- reverse (adjoint) pieces
// Adjoint of the metric quantities with respect to the code position.
template <class CT>
struct AxiMetricBar {
  CT r, th, h1, h2, h3, st, ct;
};

// (r, theta, sqrt h_ii, sin, cos) at (x1, x2) -> (dL/dx1, dL/dx2); the
// Sec. 2.4 metric differentiated by hand
template <int GEOM, class CT>
__device__ __forceinline__ void axi_metric_rev(const GridConst &g, const AxiMetric<CT> &M, CT x2,
                                               AxiMetricBar<CT> b, CT &x1b, CT &x2b) {
  // h3 = r sin(theta); st, ct = sin, cos of theta
  b.r += b.h3 * M.st;
  b.st += b.h3 * M.r;
  b.th += b.st * M.ct - b.ct * M.st;
  if (GEOM == 1) {
    // r = rmin + x1 dr, theta = x2 dth, h1 = dr, h2 = r dth
    b.r += b.h2 * (CT)g.dth;
    x1b += b.r * (CT)g.dr;
    x2b += b.th * (CT)g.dth;
  } else {
    // r = r0 + e^R, R = Rmin + x1 dR; h1 = dR e^R; h2 = dT theta_T(T) r; T = x2 dT
    const CT eR = M.r - (CT)g.r0;
    const CT T = x2 * (CT)g.dT;
    const CT tp = T * (CT)(1.0 / kPI);
    const CT vt = (CT)g.vt;
    const CT thT = (CT)1 + (CT)2 * vt + (CT)12 * vt * tp * (tp - (CT)1);
    const CT thTT = (CT)12 * vt * ((CT)2 * tp - (CT)1) * (CT)(1.0 / kPI);
    b.r += b.h2 * (CT)g.dT * thT;
    const CT thTb = b.h2 * (CT)g.dT * M.r;
    const CT eRb = b.r + b.h1 * (CT)g.dR;
    x1b += eRb * eR * (CT)g.dR;
    x2b += (b.th * thT + thTb * thTT) * (CT)g.dT;
  }
}

// Reverse of axi_move: given dL/d(dx1, dx2, dphi), accumulate dL/d of its
// inputs: the position (through the metric: into Mb and x2b), the azimuth
// (through sin, cos: spb, cpb) and the Cartesian displacement (DXb).  The
// intermediates are recomputed; the qsph Newton solve is differentiated as
// its converged root (implicit function theorem).
template <int GEOM, class CT>
__device__ __forceinline__ void axi_move_rev(const GridConst &g, const AxiMetric<CT> &M, CT x2,
                                             CT sp, CT cp, CT DX, CT DY, CT DZ, CT dx1b, CT dx2b,
                                             CT dphib, AxiMetricBar<CT> &Mb, CT &x2b, CT &spb,
                                             CT &cpb, CT DXb[3]) {
  const CT Dr = DX * cp + DY * sp;
  const CT Dp = DY * cp - DX * sp;
  const CT rho_o = M.r * M.st, z_o = M.r * M.ct;
  const CT D2 = DX * DX + DY * DY + DZ * DZ;
  const CT ir2 = (CT)1 / (M.r * M.r);
  const CT P = (CT)2 * (rho_o * Dr + z_o * DZ) + D2;
  const CT sig = P * ir2;
  const CT hl = (CT)0.5 * log1p_r(sig);
  const CT rx = rho_o + Dr;
  const CT rho_n = sqrt_r(rx * rx + Dp * Dp);
  const CT z_n = z_o + DZ;
  // adjoints of the intermediates
  CT hlb = 0, dthb = 0;
  CT rb = 0;
  if (GEOM == 1) {
    const CT E1 = expm1_r(hl);
    rb += dx1b * E1 * (CT)(1.0 / g.dr);
    hlb += dx1b * M.r * (CT)(1.0 / g.dr) * (E1 + (CT)1);
    dthb += dx2b * (CT)(1.0 / g.dth);
  } else {
    if (g.r0 == 0.0) {
      hlb += dx1b * (CT)(1.0 / g.dR);
    } else {
      const CT E1 = expm1_r(hl);
      const CT den = M.r - (CT)g.r0;
      const CT Q = M.r * E1 / den;
      const CT Qb = dx1b * (CT)(1.0 / g.dR) / ((CT)1 + Q);
      rb += Qb * E1 * (-(CT)g.r0) / (den * den);
      hlb += Qb * M.r / den * (E1 + (CT)1);
    }
    // s solves a1 s + a2 s^2 + a3 s^3 = dth (T0 = x2 dT); dx2 = s / dT
    const CT T0 = x2 * (CT)g.dT;
    const CT tp = T0 * (CT)(1.0 / kPI);
    const CT vt = (CT)g.vt;
    const CT a1 = (CT)1 + (CT)2 * vt + (CT)12 * vt * tp * (tp - (CT)1);
    const CT a2 = (CT)(6.0 / (kPI * kPI)) * vt * ((CT)2 * T0 - (CT)kPI);
    const CT a3 = (CT)(4.0 / (kPI * kPI)) * vt;
    // the forward's dth and its Newton root
    CT dth;
    {
      const CT drho0 = ((CT)2 * rho_o * Dr + Dr * Dr + Dp * Dp);
      if (rho_n + rho_o > (CT)0)
        dth = atan2_r(drho0 / (rho_n + rho_o) * z_o - DZ * rho_o, rho_o * rho_n + z_o * z_n);
      else
        dth = ((CT)(kPI / 2) - atan2_r(z_n, rho_n)) - M.th;
    }
    CT s = dth / a1;
#pragma unroll
    for (int it = 0; it < 3; ++it) {
      const CT f = ((a3 * s + a2) * s + a1) * s - dth;
      const CT fp = ((CT)3 * a3 * s + (CT)2 * a2) * s + a1;
      s = s - f / fp;
    }
    const CT fp = ((CT)3 * a3 * s + (CT)2 * a2) * s + a1;
    const CT sb = dx2b * (CT)(1.0 / g.dT);
    dthb += sb / fp;
    const CT a1b = -sb * s / fp, a2b = -sb * s * s / fp;
    const CT T0b = a1b * (CT)12 * vt * ((CT)2 * tp - (CT)1) * (CT)(1.0 / kPI) +
                   a2b * (CT)(12.0 / (kPI * kPI)) * vt;
    x2b += T0b * (CT)g.dT;
  }
  // dphi = atan2(Dp, rx)
  CT Dpb = 0, rxb = 0, Drb = 0, rhoob = 0, zob = 0, rhonb = 0, znb = 0, DZb = 0;
  {
    const CT q2 = Dp * Dp + rx * rx;
    if (q2 > (CT)0) {
      Dpb += dphib * rx / q2;
      rxb -= dphib * Dp / q2;
    }
  }
  if (rho_n + rho_o > (CT)0) {
    const CT den = rho_n + rho_o;
    const CT num = (CT)2 * rho_o * Dr + Dr * Dr + Dp * Dp;
    const CT drho = num / den;
    const CT Y = drho * z_o - DZ * rho_o;
    const CT X = rho_o * rho_n + z_o * z_n;
    const CT q2 = X * X + Y * Y;
    const CT Yb = dthb * X / q2, Xb = -dthb * Y / q2;
    const CT drhob = Yb * z_o;
    zob += Yb * drho + Xb * z_n;
    DZb -= Yb * rho_o;
    rhoob += -Yb * DZ + Xb * rho_n;
    rhonb += Xb * rho_o;
    znb += Xb * z_o;
    const CT numb = drhob / den;
    const CT denb = -drhob * drho / den;
    rhonb += denb;
    rhoob += denb;
    rhoob += numb * (CT)2 * Dr;
    Drb += numb * (CT)2 * (rho_o + Dr);
    Dpb += numb * (CT)2 * Dp;
  } else {  // both points on the axis: theta from the literal map
    const CT q2 = z_n * z_n + rho_n * rho_n;
    if (q2 > (CT)0) {
      znb -= dthb * rho_n / q2;
      rhonb += dthb * z_n / q2;
    }
    Mb.th -= dthb;
  }
  // z_n = z_o + DZ; rho_n = |(rx, Dp)|
  zob += znb;
  DZb += znb;
  if (rho_n > (CT)0) {
    rxb += rhonb * rx / rho_n;
    Dpb += rhonb * Dp / rho_n;
  }
  // rx = rho_o + Dr
  rhoob += rxb;
  Drb += rxb;
  // hl = log1p(sig) / 2, sig = P / r^2
  const CT sigb = hlb * (CT)0.5 / ((CT)1 + sig);
  const CT Pb = sigb * ir2;
  rb -= (CT)2 * sigb * sig / M.r;
  rhoob += (CT)2 * Pb * Dr;
  Drb += (CT)2 * Pb * rho_o;
  zob += (CT)2 * Pb * DZ;
  DZb += (CT)2 * Pb * z_o;
  DXb[0] += (CT)2 * Pb * DX;
  DXb[1] += (CT)2 * Pb * DY;
  DZb += (CT)2 * Pb * DZ;
  // rho_o = r sin(theta), z_o = r cos(theta)
  rb += rhoob * M.st + zob * M.ct;
  Mb.st += rhoob * M.r;
  Mb.ct += zob * M.r;
  Mb.r += rb;
  // Dr = DX cp + DY sp, Dp = DY cp - DX sp
  DXb[0] += Drb * cp - Dpb * sp;
  DXb[1] += Drb * sp + Dpb * cp;
  DXb[2] += DZb;
  cpb += Drb * DX + Dpb * DY;
  spb += Drb * DY - Dpb * DX;
}

// Reverse of axi_to_cart: dL/dE, dL/dB (global Cartesian) -> dL/dF (the
// interpolated contravariant components) and the metric / azimuth adjoints.
template <class CT, class Real>
__device__ __forceinline__ void axi_to_cart_rev(const AxiMetric<CT> &M, CT sp, CT cp,
                                                const Real F[6], const Real Eb[3],
                                                const Real Bb[3], Real Fb[6],
                                                AxiMetricBar<CT> &Mb, CT &spb, CT &cpb) {
  const CT h[3] = {M.h1, M.h2, M.h3};
  CT hb[3] = {0, 0, 0};
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    const Real *ob = f ? Bb : Eb;
    const CT o0 = (CT)ob[0], o1 = (CT)ob[1], o2 = (CT)ob[2];
    const CT a = (CT)F[3 * f] * h[0], b = (CT)F[3 * f + 1] * h[1], cc = (CT)F[3 * f + 2] * h[2];
    const CT ax = a * M.st + b * M.ct;
    const CT axb = o0 * cp + o1 * sp;
    const CT ccb = -o0 * sp + o1 * cp;
    cpb += o0 * ax + o1 * cc;
    spb += -o0 * cc + o1 * ax;
    const CT ab = axb * M.st + o2 * M.ct;
    const CT bb = axb * M.ct - o2 * M.st;
    Mb.st += axb * a - o2 * b;
    Mb.ct += axb * b + o2 * a;
    Fb[3 * f] = (Real)(ab * h[0]);
    Fb[3 * f + 1] = (Real)(bb * h[1]);
    Fb[3 * f + 2] = (Real)(ccb * h[2]);
    hb[0] += ab * (CT)F[3 * f];
    hb[1] += bb * (CT)F[3 * f + 1];
    hb[2] += ccb * (CT)F[3 * f + 2];
  }
  Mb.h1 += hb[0];
  Mb.h2 += hb[1];
  Mb.h3 += hb[2];
}

}  // namespace picstep
