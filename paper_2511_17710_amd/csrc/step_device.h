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
template <class Real>
__device__ __forceinline__ void boris(Real k, const Real E[3], const Real B[3], Real u[3]) {
  Real um0 = u[0] + k * E[0], um1 = u[1] + k * E[1], um2 = u[2] + k * E[2];
  Real ig = rsqrt_r((Real)1 + um0 * um0 + um1 * um1 + um2 * um2);
  Real t0 = k * B[0] * ig, t1 = k * B[1] * ig, t2 = k * B[2] * ig;
  Real sf = (Real)2 * rcp_r((Real)1 + t0 * t0 + t1 * t1 + t2 * t2);
  Real s0 = t0 * sf, s1 = t1 * sf, s2 = t2 * sf;
  Real up0 = um0 + (um1 * t2 - um2 * t1);
  Real up1 = um1 + (um2 * t0 - um0 * t2);
  Real up2 = um2 + (um0 * t1 - um1 * t0);
  u[0] = um0 + (up1 * s2 - up2 * s1) + k * E[0];
  u[1] = um1 + (up2 * s0 - up0 * s2) + k * E[1];
  u[2] = um2 + (up0 * s1 - up1 * s0) + k * E[2];
}

// Cartesian in-cell displacement dt u_a / (gamma Delta_a) (steps 6-7); the
// FP32 build multiplies by the reciprocal spacing, the FP64 build divides
// (it matches the reference's rounding).  The forward and the adjoint
// recompute share this routine, so both take the same step.
__device__ __forceinline__ float cart_disp(const GridConst &g, int a, float dt, float u, float gi) {
  return dt * u * gi * (float)g.inv_dx[a];
}
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

}  // namespace picstep
