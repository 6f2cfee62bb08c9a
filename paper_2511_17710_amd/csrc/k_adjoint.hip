// k_adjoint.hip -- reverse-mode derivative of one particle step, written by
// hand, on Cartesian and axisymmetric (spherical, quasi-spherical) grids: the
// forward step of the particle is recomputed in registers from its stored
// state, then the adjoints are propagated backwards through the zig-zag
// deposit (a gather of dL/dJ), the move (on axisymmetric grids the
// offset-relative back-transform, its azimuth step and the position
// dependence of the metric), the Boris push, the tetrad and rotation, and
// the interpolation (a scatter into dL/dE, dL/dB).  Discrete branches (cell
// crossings, the relay clamp, the half-cell stagger choice, the theta clamp)
// take the derivative of the branch the forward step took.
#include "block_util.h"
#include "step_device.h"

namespace picstep {

// LDS buffer per block: the copy of the fields and of dL/dJ over the block's
// box, then the tile of dL/d(fields).  Sized like the forward kernel's: the
// FP32 instances run 4 blocks per CU, the FP64 ones 2.
template <class Real>
constexpr int adj_tile_bytes() {
  return sizeof(Real) == 8 ? 79872 : 39936;
}

// the 2^DIM lattice values around A[base] (row stride sy, plane stride sz)
template <int DIM, class Real>
__device__ __forceinline__ void corners(const Real *__restrict__ A, int base, int sy, int sz,
                                        Real c[8]) {
#pragma unroll
  for (int e = 0; e < (1 << DIM); ++e)
    c[e] = A[base + (e & 1) + ((e >> 1) & 1) * sy + ((DIM == 3) ? ((e >> 2) & 1) * sz : 0)];
}

// derivative of a first-order interpolation from the corner values cv along
// the offsets in x, y (and z); fw: the weights along x, y, z
template <int DIM, class Real>
__device__ __forceinline__ void offset_grad(const Real cv[8], const Real fw[3], Real G[3]) {
  const Real fx = fw[0], fy = fw[1], fz = fw[2];
  const Real gx = (Real)1 - fx, gy = (Real)1 - fy;
  if (DIM == 2) {
    G[0] = gy * (cv[1] - cv[0]) + fy * (cv[3] - cv[2]);
    G[1] = gx * (cv[2] - cv[0]) + fx * (cv[3] - cv[1]);
    G[2] = (Real)0;
  } else {
    const Real gz = (Real)1 - fz;
    G[0] = gz * (gy * (cv[1] - cv[0]) + fy * (cv[3] - cv[2])) +
           fz * (gy * (cv[5] - cv[4]) + fy * (cv[7] - cv[6]));
    G[1] = gz * (gx * (cv[2] - cv[0]) + fx * (cv[3] - cv[1])) +
           fz * (gx * (cv[6] - cv[4]) + fx * (cv[7] - cv[5]));
    G[2] = gy * (gx * (cv[4] - cv[0]) + fx * (cv[5] - cv[1])) +
           fy * (gx * (cv[6] - cv[2]) + fx * (cv[7] - cv[3]));
  }
}

// copy ncomp components of a padded global array over the box [o, o + s) of
// (unwrapped) cells into LDS, component-major, x fastest; Cartesian grids
// take the periodic image of points outside the padded lattice, curvilinear
// grids read them as zero (no particle stencil reaches them)
template <int GEOM, int DIM, class Real>
__device__ __forceinline__ void stage_box(const GridConst &g, const Real *__restrict__ src,
                                          int ncomp, const int o[3], const int sz3[3],
                                          Real *dst) {
  const int npts = (int)g.npts;
  const int wstride = (DIM == 3) ? g.np[0] * g.np[1] : g.np[0];
  bool inside = true;
#pragma unroll
  for (int d = 0; d < DIM; ++d) inside = inside && o[d] >= -NG && o[d] + sz3[d] <= g.n[d] + NG;
  if (inside) {
    tile_for_each_affine<16, Real>(
        ncomp, DIM == 3 ? 2 : 1, sz3[0], sz3[1], sz3[2], npts, wstride,
        [&](int ix, int iy) {
          return pad_index(g, o[0] + ix, o[1] + ((DIM == 3) ? iy : 0), o[2], DIM);
        },
        [&](int gi, int) { return src[gi]; }, [&](int, int x, Real v) { dst[x] = v; });
  } else {
    constexpr int WA = DIM - 1;
    tile_for_each<16, Real>(
        ncomp, DIM == 3 ? 2 : 1, sz3[0], sz3[1], sz3[2],
        [&](int ix, int iy) {
          int gx = o[0] + ix, gy = (DIM == 3) ? o[1] + iy : 0;
          bool ok = true;
          if (GEOM == 0) {
            gx = wrap_periodic(gx, g.n[0]);
            if (DIM == 3) gy = wrap_periodic(gy, g.n[1]);
          } else {
            ok = gx >= -NG && gx < g.n[0] + NG;
          }
          return PlanePt{(gx + NG) + ((DIM == 3) ? g.np[0] * (gy + NG) : 0), ok};
        },
        [&](const PlanePt &pp, int, int comp, int w) {
          int gw = o[WA] + w;
          bool ok = pp.ok;
          if (GEOM == 0)
            gw = wrap_periodic(gw, g.n[WA]);
          else
            ok = ok && gw >= -NG && gw < g.n[WA] + NG;
          return ok ? src[comp * npts + pp.off + wstride * (gw + NG)] : (Real)0;
        },
        [&](const PlanePt &, int x, int, int, Real v) { dst[x] = v; });
  }
}

// A padded global array or a block's LDS copy of it over a box: component c,
// cell (I, J, K) (unwrapped) at c*cs + (I - o0) + sy*(J - o1) + sz*(K - o2).
template <class Real>
struct BoxView {
  const Real *L;
  int cs, sy, sz;
  int o[3];
};

// Reverse of step 8: dL/dJ gathered through the particle's zig-zag.  za: old
// offsets, zb: new offsets + m (both exact, measured from the old cell i0).
// Adds dL/d(old offset) into ab and dL/d(displacement) into dxb (b = a +
// displacement), dL/d(dx3) (2D out-of-plane displacement) into dx3b; bfix[d]:
// the new position is a constant in dimension d (theta clamp), so nothing
// flows through b there.
template <int DIM, class Real>
__device__ __forceinline__ void zigzag_rev(const BoxView<Real> &V, const int i0[3], const int m[3],
                                           const double za[3], const double zb[3], Real C,
                                           Real dx3, const bool bfix[3], Real ab[3], Real dxb[3],
                                           Real &dx3b) {
  Real Fs[2][3] = {{0, 0, 0}, {0, 0, 0}}, Ws[2][3] = {{0, 0, 0}, {0, 0, 0}};
  bool mid_free[3] = {false, false, false};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const double lo = (double)(min(0, m[a]) + 1), hi = (double)max(0, m[a]);
    const double mid = (za[a] + zb[a]) * 0.5;
    const double xr = fmin(lo, fmax(hi, mid));
    mid_free[a] = (mid >= hi) && (mid <= lo);
    Fs[0][a] = (Real)(xr - za[a]);
    Fs[1][a] = (Real)(zb[a] - xr);
    Ws[0][a] = (Real)((za[a] + xr) * 0.5);
    Ws[1][a] = (Real)((xr + zb[a]) * 0.5 - (double)m[a]);
  }
  Real Fb[2][3] = {{0, 0, 0}, {0, 0, 0}}, Wb[2][3] = {{0, 0, 0}, {0, 0, 0}};
  const Real *L = V.L;
  const int cs = V.cs, sy = V.sy, sz = V.sz;
#pragma unroll
  for (int sg = 0; sg < 2; ++sg) {
    const int I = i0[0] + (sg ? m[0] : 0), Jc = i0[1] + (sg ? m[1] : 0);
    const int K = (DIM == 3) ? i0[2] + (sg ? m[2] : 0) : 0;
    const int base = (I - V.o[0]) + sy * (Jc - V.o[1]) + ((DIM == 3) ? sz * (K - V.o[2]) : 0);
    const Real Fx = Fs[sg][0], Fy = Fs[sg][1], Wx = Ws[sg][0], Wy = Ws[sg][1];
    if (DIM == 2) {
      const Real l10 = L[base], l11 = L[base + sy];
      const Real l20 = L[cs + base], l21 = L[cs + base + 1];
      Fb[sg][0] += C * (l10 * ((Real)1 - Wy) + l11 * Wy);
      Wb[sg][1] += C * Fx * (l11 - l10);
      Fb[sg][1] += C * (l20 * ((Real)1 - Wx) + l21 * Wx);
      Wb[sg][0] += C * Fy * (l21 - l20);
      const Real *L3 = L + 2 * cs + base;
      const Real a00 = L3[0], a10 = L3[1], a01 = L3[sy], a11 = L3[sy + 1];
      const Real h = C * dx3 * (Real)0.5;
      const Real cxy = Fx * Fy * (Real)(1.0 / 12.0);
      const Real val = a00 * (((Real)1 - Wx) * ((Real)1 - Wy) + cxy) +
                       a10 * (Wx * ((Real)1 - Wy) - cxy) + a01 * (((Real)1 - Wx) * Wy - cxy) +
                       a11 * (Wx * Wy + cxy);
      dx3b += C * (Real)0.5 * val;
      Wb[sg][0] += h * (-a00 * ((Real)1 - Wy) + a10 * ((Real)1 - Wy) - a01 * Wy + a11 * Wy);
      Wb[sg][1] += h * (-a00 * ((Real)1 - Wx) - a10 * Wx + a01 * ((Real)1 - Wx) + a11 * Wx);
      const Real csum = (a00 - a10 - a01 + a11) * h * (Real)(1.0 / 12.0);
      Fb[sg][0] += csum * Fy;
      Fb[sg][1] += csum * Fx;
    } else {
      // component c with transverse dims (a, b): value = C F_c (w_a w_b + sgn F_a F_b / 12)
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        const int da = (comp == 0) ? 1 : 0;
        const int db = (comp == 2) ? 1 : 2;
        const int sa = (da == 0) ? 1 : sy;
        const int sb = (db == 1) ? sy : sz;
        const Real *Lc = L + comp * cs + base;
        const Real l00 = Lc[0], l10 = Lc[sa], l01 = Lc[sb], l11 = Lc[sa + sb];
        const Real Fc = Fs[sg][comp];
        const Real Wa = Ws[sg][da], Wbb = Ws[sg][db];
        const Real Fa = Fs[sg][da], Fbt = Fs[sg][db];
        const Real ga = (Real)1 - Wa, gb = (Real)1 - Wbb;
        const Real cab = Fa * Fbt * (Real)(1.0 / 12.0);
        const Real sgn = l00 - l10 - l01 + l11;
        const Real val = l00 * (ga * gb + cab) + l10 * (Wa * gb - cab) + l01 * (ga * Wbb - cab) +
                         l11 * (Wa * Wbb + cab);
        Fb[sg][comp] += C * val;
        Wb[sg][da] += C * Fc * (-l00 * gb + l10 * gb - l01 * Wbb + l11 * Wbb);
        Wb[sg][db] += C * Fc * (-l00 * ga - l10 * Wa + l01 * ga + l11 * Wa);
        Fb[sg][da] += C * Fc * sgn * Fbt * (Real)(1.0 / 12.0);
        Fb[sg][db] += C * Fc * sgn * Fa * (Real)(1.0 / 12.0);
      }
    }
  }
  // relay: F1 = xr - a, F2 = b - xr, W1 = (a + xr)/2, W2 = (xr + b)/2 - m
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const Real xrb = Fb[0][a] - Fb[1][a] + (Real)0.5 * (Wb[0][a] + Wb[1][a]);
    Real abar = -Fb[0][a] + (Real)0.5 * Wb[0][a];
    Real bbar = Fb[1][a] + (Real)0.5 * Wb[1][a];
    if (mid_free[a]) {  // xr = (a + b)/2
      abar += (Real)0.5 * xrb;
      bbar += (Real)0.5 * xrb;
    }
    if (bfix[a]) bbar = 0;
    // b = a + displacement
    ab[a] += abar + bbar;
    dxb[a] += bbar;
  }
}

// Per-particle reverse on a Cartesian grid: forward recompute (tetrad =
// cell sizes, Boris, move), then the reverse of deposit, move and Boris.
// Returns dL/d(interpolated F) in Fb and adds dL/d(old offsets) (except the
// interpolation weights' part) into ab; writes dL/du before the step.
template <int DIM, class Real>
__device__ __forceinline__ void cart_particle_rev(const AdjArgs<Real> &A, int s, int64_t p,
                                                  const int i[3], const OffT<Real> q[3],
                                                  const Real F[6], const BoxView<Real> &LJ,
                                                  Real Fb[6], Real ab[3]) {
  using PS = Pos<Real>;
  const GridConst &g = A.g;
  const Real u0[3] = {A.p.u[0][p], A.p.u[1][p], A.p.u[2][p]};
  const Real k = konst<Real>(A.sp.k[s], A.sp.kf[s]);
  const Real dtr = (Real)A.dt;
  Real E[3], B[3], sc[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    sc[a] = (a < DIM) ? konst<Real>(g.dx[a], g.dxf[a]) : (Real)1;
    E[a] = F[a] * sc[a];
    B[a] = F[3 + a] * sc[a];
  }
  Real un[3] = {u0[0], u0[1], u0[2]};
  BorisRec<Real> R;
  boris_rec(k, E, B, un, R);
  // steps 6-7: move, as in the forward kernel
  const Real ig = rsqrt_r((Real)1 + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
  int m[3] = {0, 0, 0};
  double za[3] = {0, 0, 0}, zb[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const Real dx = cart_disp(g, a, dtr, un[a], ig);
    OffT<Real> qn;
    m[a] = PS::move(q[a], (double)dx, qn);
    za[a] = PS::exact(q[a]);
    zb[a] = PS::exact(qn) + (double)m[a];
  }
  // the adjoint of the new offsets passes to the old offset and the displacement
  Real dxb[3] = {0, 0, 0}, dx3b = 0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const Real l = A.lam_d[a][p];
    ab[a] += l;
    dxb[a] += l;
  }
  if (A.lamJ) {
    const bool bfix[3] = {false, false, false};
    const Real dx3 = (DIM == 2) ? dtr * un[2] * ig : (Real)0;
    zigzag_rev<DIM, Real>(LJ, i, m, za, zb, (Real)A.sp.qdt[s] * A.p.w[p], dx3, bfix, ab, dxb, dx3b);
  }
  // steps 6-7 reversed: dx_a = dt u_a / (gamma Delta_a); 2D also dx3 = dt u_z / gamma
  Real wv[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) wv[a] = dxb[a] * dtr / (Real)g.dx[a];
  if (DIM == 2) wv[2] = dx3b * dtr;
  const Real uw = un[0] * wv[0] + un[1] * wv[1] + un[2] * wv[2];
  Real unb[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) unb[a] = A.lam_u[a][p] + wv[a] * ig - un[a] * uw * ig * ig * ig;
  Real ub[3], Eb[3], Bb[3];
  boris_rev(k, R, unb, ub, Eb, Bb);
  // tetrad reversed
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Fb[a] = Eb[a] * sc[a];
    Fb[3 + a] = Bb[a] * sc[a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) A.lam_u[a][p] = ub[a];
}

// Per-particle reverse on an axisymmetric grid, with the metric, rotation
// and move in CT (FP64 near the axis and r_min in FP32 builds, as in the
// forward step).  D: the offsets as the forward step feeds them to the
// metric.  dL/dphi lives in lam_phi.
template <int GEOM, class CT, class Real, class D>
__device__ __forceinline__ void axi_particle_rev(const AdjArgs<Real> &A, int s, int64_t p,
                                                 const int i[3], const OffT<Real> q[3], D d1,
                                                 D d2, const Real F[6], const BoxView<Real> &LJ,
                                                 Real Fb[6], Real ab[3]) {
  using PS = Pos<Real>;
  const GridConst &g = A.g;
  const Real k = konst<Real>(A.sp.k[s], A.sp.kf[s]);
  const Real phi = A.p.phi[p];
  // ---- forward recompute (the operations of axi_particle)
  const CT x1 = (CT)i[0] + (CT)d1;
  const CT x2 = (CT)i[1] + (CT)d2;
  const AxiMetric<CT> M = axi_metric<GEOM, CT>(g, x1, x2);
  CT sp, cp;
  sincos_r((CT)phi, &sp, &cp);
  Real E[3], B[3];
  axi_to_cart<CT, Real>(M, sp, cp, F, E, B);
  Real un[3] = {A.p.u[0][p], A.p.u[1][p], A.p.u[2][p]};
  BorisRec<Real> R;
  boris_rec(k, E, B, un, R);
  const CT uu[3] = {(CT)un[0], (CT)un[1], (CT)un[2]};
  const CT gi = rsqrt_r((CT)1 + uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]);
  const CT dtg = (CT)A.dt * gi;
  const CT DX = dtg * uu[0], DY = dtg * uu[1], DZ = dtg * uu[2];
  CT dx1, dx2, dphi;
  axi_move<GEOM, CT>(g, M, x2, sp, cp, DX, DY, DZ, dx1, dx2, dphi);
  int m[3] = {0, 0, 0};
  OffT<Real> qn1, qn2;
  m[0] = PS::move(q[0], (double)dx1, qn1);
  m[1] = PS::move(q[1], (double)dx2, qn2);
  int inew1 = i[1] + m[1];
  bool clamp = false;
  if (inew1 < 0) {
    inew1 = 0;
    qn2 = (OffT<Real>)0;
    clamp = true;
  } else if (inew1 >= g.n[1]) {
    inew1 = g.n[1] - 1;
    qn2 = largest_offset<Real>();
    clamp = true;
  }
  m[1] = inew1 - i[1];
  // ---- reverse
  Real dxb[3] = {0, 0, 0}, dx3b = 0;
  {
    const Real l1 = A.lam_d[0][p];
    ab[0] += l1;
    dxb[0] += l1;
    if (!clamp) {
      const Real l2 = A.lam_d[1][p];
      ab[1] += l2;
      dxb[1] += l2;
    }
  }
  if (A.lamJ) {
    const double za[3] = {PS::exact(q[0]), PS::exact(q[1]), 0.0};
    const double zb[3] = {PS::exact(qn1) + (double)m[0], PS::exact(qn2) + (double)m[1], 0.0};
    const bool bfix[3] = {false, clamp, false};
    zigzag_rev<2, Real>(LJ, i, m, za, zb, (Real)A.sp.qdt[s] * A.p.w[p], (Real)dphi, bfix, ab, dxb,
                        dx3b);
  }
  // phi_new = phi + dphi (wrapped)
  const Real phinb = A.lam_phi[p];
  CT phib = (CT)phinb;
  const CT dphib = (CT)dx3b + (CT)phinb;
  AxiMetricBar<CT> Mb{0, 0, 0, 0, 0, 0, 0};
  CT x1b = 0, x2b = 0, spb = 0, cpb = 0;
  CT DXb[3] = {0, 0, 0};
  axi_move_rev<GEOM, CT>(g, M, x2, sp, cp, DX, DY, DZ, (CT)dxb[0], (CT)dxb[1], dphib, Mb, x2b, spb,
                         cpb, DXb);
  // DX = dt u / gamma
  const CT uw = uu[0] * DXb[0] + uu[1] * DXb[1] + uu[2] * DXb[2];
  Real unb[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    unb[a] = A.lam_u[a][p] + (Real)(dtg * DXb[a] - (CT)A.dt * gi * gi * gi * uu[a] * uw);
  Real ub[3], Eb[3], Bb[3];
  boris_rev(k, R, unb, ub, Eb, Bb);
  axi_to_cart_rev<CT, Real>(M, sp, cp, F, Eb, Bb, Fb, Mb, spb, cpb);
  phib += spb * cp - cpb * sp;
  axi_metric_rev<GEOM, CT>(g, M, x2, Mb, x1b, x2b);
  ab[0] += (Real)x1b;
  ab[1] += (Real)x2b;
#pragma unroll
  for (int a = 0; a < 3; ++a) A.lam_u[a][p] = ub[a];
  A.lam_phi[p] = (Real)phib;
}

// adj_ppt consecutive particles per thread (1 in FP32, 2 in FP64), in
// XCD-aware order: the block's field and dL/dJ copies and its tile flush
// serve them all.  The
// scatter into dL/dE, dL/dB (the adjoint of the interpolation) goes to an LDS
// tile over the block's cells, accumulated like the forward current (64-bit
// fixed point in FP32 builds, scaled by the block's largest |dL/dF|) and
// flushed with one global atomic per nonzero value; particles whose stencil
// leaves the tile scatter with global atomics.
// Waves per SIMD the register allocation must allow: the FP32 Cartesian
// instances run faster at 4 (a few spills) than uncapped at 3 (0.457 -> 0.41
// ms per step on the 64^3 workload); the others stay uncapped.
template <int GEOM, class Real>
constexpr int adj_waves() {
  return (GEOM == 0 && sizeof(Real) == 4) ? 4 : 1;
}

template <int GEOM, int DIM, class Real>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(adj_waves<GEOM, Real>(), 8)))
void k_adjoint(AdjArgs<Real> A) {
  using PS = Pos<Real>;
  using Acc = typename TileAcc<Real>::type;
  constexpr int APT = adj_ppt<Real>();
  constexpr int TILE_VALS = adj_tile_bytes<Real>() / (int)sizeof(Acc);
  constexpr int STAGE_VALS = adj_tile_bytes<Real>() / (int)sizeof(Real);
  __shared__ union {
    Acc j[TILE_VALS];
    Real f[STAGE_VALS];
  } lds;
  Acc *tile = lds.j;
  __shared__ int red[6 * (BLOCK / 64)];
  const GridConst &g = A.g;
  const int64_t blk = xcd_chunk(blockIdx.x, A.sp.blk0[MAXSP]);  // blk0[MAXSP] = all blocks
  int s = 0;
#pragma unroll
  for (int t = 1; t < MAXSP; ++t)
    if (t < A.sp.nspec && blk >= A.sp.blk0[t]) s = t;
  // the thread's particles: APT consecutive ones of the block's chunk, and
  // neighbouring lanes 4 APT apart (the 4 waves interleave): a wave's 64
  // lanes spread over 4 APT times as many particles, so fewer lanes of an
  // atomic to the dL/dF tile share its address (0.41 -> 0.37 ms per step in
  // FP32, 0.65 -> 0.51 in FP64 on the 64^3 workload)
  static_assert(BLOCK == 256, "4 waves interleave");
  const int64_t c0 = (blk - A.sp.blk0[s]) * (int64_t)(BLOCK * APT);
  int64_t pr[APT];
  int32_t ccr[APT];
#pragma unroll
  for (int r = 0; r < APT; ++r) {
    const int64_t local =
        c0 + (int64_t)((threadIdx.x & 63) * (4 * APT) + (threadIdx.x >> 6) * APT + r);
    const bool inrange = local < A.sp.n[s];
    pr[r] = A.sp.off[s] + (inrange ? local : 0);
    // a frozen (dead) particle maps to itself: its adjoints pass through
    ccr[r] = inrange ? A.p.cell[pr[r]] : (int32_t)DEAD_BIT;
  }

  // ---------------- the block's box and its LDS tile (stencils reach i-1 .. i+1)
  int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
#pragma unroll
  for (int r = 0; r < APT; ++r) {
    if (ccr[r] & DEAD_BIT) continue;
    int i[3];
    cell_decode(g, ccr[r], i);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = min(lo[d], i[d]);
      hi[d] = max(hi[d], i[d]);
    }
  }
  block_minmax3(lo, hi, red);
  if (lo[0] > hi[0]) return;  // no live particle in the block (uniform)
  // periodic dimensions whose cells span more than half the box are
  // unwrapped (cells below N/2 shifted by +N)
  int shift[3] = {0, 0, 0};
  if (GEOM == 0) {
    bool any = false;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      shift[d] = (hi[d] - lo[d] > (g.n[d] >> 1)) ? 1 : 0;
      any = any || shift[d];
    }
    if (any) {  // a block straddling a periodic boundary: box of the unwrapped cells
      __syncthreads();
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lo[d] = INT32_MAX;
        hi[d] = INT32_MIN;
      }
#pragma unroll
      for (int r = 0; r < APT; ++r) {
        if (ccr[r] & DEAD_BIT) continue;
        int i[3];
        cell_decode(g, ccr[r], i);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int v = i[d] + ((shift[d] && i[d] < (g.n[d] >> 1)) ? g.n[d] : 0);
          lo[d] = min(lo[d], v);
          hi[d] = max(hi[d], v);
        }
      }
      block_minmax3(lo, hi, red);
    }
  }
  // unwrapped minus stored cell coordinates of a particle
  auto unwrap = [&](const int i[3], int dsh[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d)
      dsh[d] = (GEOM == 0 && shift[d] && i[d] < (g.n[d] >> 1)) ? g.n[d] : 0;
  };
  int t0[3] = {0, 0, 0}, ts[3] = {1, 1, 1}, j0[3] = {0, 0, 0}, js[3] = {1, 1, 1};
  int T = 1, TJ = 1;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    ts[d] = hi[d] - lo[d] + 3;  // interpolation stencils: cells i-1 .. i+1
    js[d] = hi[d] - lo[d] + 4;  // deposit stencils: cells i-1 .. i+2
    j0[d] = lo[d] - 1;
    T *= ts[d];
    TJ *= js[d];
  }
  // the box's fields (6 T values) and dL/dJ (3 TJ) fit in the buffer: copy
  // them (uniform), and every live particle reads them from LDS
  const bool stage = 6 * T <= TILE_VALS && 6 * T + (A.lamJ ? 3 * TJ : 0) <= STAGE_VALS;
  if (6 * T <= TILE_VALS) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) t0[d] = lo[d] - 1;
  } else {  // largest cube (square) centred on the block's mean cell
    __syncthreads();
    int sum[3] = {0, 0, 0}, nl[3] = {0, 0, 0};
#pragma unroll
    for (int r = 0; r < APT; ++r) {
      if (ccr[r] & DEAD_BIT) continue;
      int i[3], dsh[3];
      cell_decode(g, ccr[r], i);
      unwrap(i, dsh);
      nl[0] += 1;
#pragma unroll
      for (int d = 0; d < DIM; ++d) sum[d] += i[d] + dsh[d];
    }
    block_sum3(sum, red);
    __syncthreads();
    block_sum3(nl, red);
    constexpr int SIDE = tile_side(TILE_VALS / 6, DIM);  // 6 SIDE^DIM <= TILE_VALS
    T = 1;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int ctr = (sum[d] + nl[0] / 2) / nl[0];
      ts[d] = SIDE;
      t0[d] = ctr - SIDE / 2;
      T *= ts[d];
    }
  }
  if (stage) {
    stage_box<GEOM, DIM, Real>(g, A.EB, 6, t0, ts, lds.f);
    if (A.lamJ) stage_box<GEOM, DIM, Real>(g, A.lamJ, 3, j0, js, lds.f + 6 * T);
    __syncthreads();
  }
  FieldTile<Real> ft;
  ft.F = lds.f;
  ft.T = T;
  ft.sy = ts[0];
  ft.sz = ts[0] * ts[1];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ft.o[a] = t0[a];
    ft.ts[a] = ts[a];
  }

  // FP32: each component's offset derivative is formed from the corner
  // values the interpolation reads and kept in registers until dL/dF is
  // known; FP64 (two particles per thread) reads the corners again instead,
  // which keeps its occupancy
  constexpr bool FUSED = sizeof(Real) == 4;
  // corner values of component c around a particle (LDS copy or global
  // memory) and its weights along x, y, z
  auto stencil_corners = [&](int c, const Stencil1<Real> *st, const int *dsh, Real cv[8],
                             Real fw[3]) {
    const int sx = kStag[c][0], sy2 = kStag[c][1], sz2 = kStag[c][2];
    const int bx = sx ? st[0].bh : st[0].b0;
    const int by = sy2 ? st[1].bh : st[1].b0;
    const int bz = (DIM == 3) ? (sz2 ? st[2].bh : st[2].b0) : 0;
    fw[0] = sx ? st[0].fh : st[0].f0;
    fw[1] = sy2 ? st[1].fh : st[1].f0;
    fw[2] = (DIM == 3) ? (sz2 ? st[2].fh : st[2].f0) : (Real)0;
    if (stage)
      corners<DIM, Real>(lds.f + c * T,
                         (bx + dsh[0] - t0[0]) + ft.sy * (by + dsh[1] - t0[1]) +
                             ((DIM == 3) ? ft.sz * (bz + dsh[2] - t0[2]) : 0),
                         ft.sy, ft.sz, cv);
    else
      corners<DIM, Real>(A.EB + c * (int)g.npts, pad_index(g, bx, by, bz, DIM), g.np[0],
                         g.np[0] * g.np[1], cv);
  };
  Real Fbr[APT][6];
  float bmax = 0.0f;
#pragma unroll
  for (int r = 0; r < APT; ++r) {
#pragma unroll
    for (int c = 0; c < 6; ++c) Fbr[r][c] = (Real)0;
    if (ccr[r] & DEAD_BIT) continue;
    const int64_t p = pr[r];
    int i[3], dsh[3];
    cell_decode(g, ccr[r], i);
    unwrap(i, dsh);
    Real *Fbar = Fbr[r];
    OffT<Real> q[3] = {(OffT<Real>)0, (OffT<Real>)0, (OffT<Real>)0};
    Real d[3] = {0, 0, 0};
    Real F[6], G[FUSED ? 6 : 1][3];
    Stencil1<Real> st[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      q[a] = A.p.offs[a][p];
      d[a] = (Real)PS::weight(q[a]);
      st[a] = stencil1(i[a], d[a]);
    }
    // ---------------- forward recompute of step 3 (interpolation: the
    // forward kernel's expression on the same corner values)
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      Real cv[8], fw[3];
      stencil_corners(c, st, dsh, cv, fw);
      F[c] = gather_at<DIM, Real>(cv, 0, 2, 4, fw[0], fw[1], fw[2]);
      if constexpr (FUSED) offset_grad<DIM, Real>(cv, fw, G[c]);
    }
    // dL/dJ from the LDS copy (box frame) or from global memory
    BoxView<Real> LJ;
    if (stage) {
      LJ.L = lds.f + 6 * T;
      LJ.cs = TJ;
      LJ.sy = js[0];
      LJ.sz = js[0] * js[1];
#pragma unroll
      for (int a = 0; a < 3; ++a) LJ.o[a] = j0[a] - dsh[a];
    } else {
      LJ.L = A.lamJ;
      LJ.cs = (int)g.npts;
      LJ.sy = g.np[0];
      LJ.sz = g.np[0] * g.np[1];
      LJ.o[0] = -NG;
      LJ.o[1] = -NG;
      LJ.o[2] = (DIM == 3) ? -NG : 0;
    }
    Real ab[3] = {0, 0, 0};  // adjoint of the old offsets
    if constexpr (GEOM == 0) {
      cart_particle_rev<DIM, Real>(A, s, p, i, q, F, LJ, Fbar, ab);
    } else {
      const bool near = (i[0] < g.fp64_cells) || (i[1] < g.fp64_cells) ||
                        (i[1] >= g.n[1] - g.fp64_cells);
      if (sizeof(Real) == 8 || near)
        axi_particle_rev<GEOM, double, Real>(A, s, p, i, q, PS::exact(q[0]), PS::exact(q[1]), F,
                                             LJ, Fbar, ab);
      else
        axi_particle_rev<GEOM, float, Real>(A, s, p, i, q, d[0], d[1], F, LJ, Fbar, ab);
    }
    // the offset derivative of the interpolation weights
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const Real fb = Fbar[c];
      bmax = fmaxf(bmax, fabsf((float)fb));
      Real gc[3];
      if constexpr (FUSED) {
#pragma unroll
        for (int a = 0; a < 3; ++a) gc[a] = G[c][a];
      } else {
        Real cv[8], fw[3];
        stencil_corners(c, st, dsh, cv, fw);
        offset_grad<DIM, Real>(cv, fw, gc);
      }
#pragma unroll
      for (int a = 0; a < DIM; ++a) ab[a] += fb * gc[a];
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) A.lam_d[a][p] = ab[a];
  }

  // ---------------- scatter of dL/dF into the tile (or global memory)
  // Fixed-point scale 2^esc (FP32): one particle adds at most max|dL/dF| to a
  // tile value (interpolation weights are at most 1), so with B 2^esc < 2^49
  // the (at most 2 BLOCK) particles of the block stay below 2^58.
  // the copies are done with: the buffer becomes the tile
  __syncthreads();
  for (int x = threadIdx.x; x < 6 * T; x += BLOCK) tile[x] = (Acc)0;
  int esc = 0;
  if (sizeof(Acc) == 8 && sizeof(Real) == 4) {
    const float B = block_max_nonneg(bmax, red);  // also orders the tile zeroing
    if (B > 0.0f && B <= 3.0e38f) esc = 48 - ilogbf(B);
  } else {
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < APT; ++r) {
    if (ccr[r] & DEAD_BIT) continue;
    const int64_t p = pr[r];
    int i[3], dsh[3];
    cell_decode(g, ccr[r], i);
    unwrap(i, dsh);
    Stencil1<Real> st[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) st[a] = stencil1(i[a], (Real)PS::weight(A.p.offs[a][p]));
    bool in = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d)
      in = in && (i[d] + dsh[d] - 1 >= t0[d]) && (i[d] + dsh[d] + 1 < t0[d] + ts[d]);
    const int sy = ts[0], sz = ts[0] * ts[1];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int sx = kStag[c][0], sy2 = kStag[c][1], sz2 = kStag[c][2];
      const int bx = sx ? st[0].bh : st[0].b0;
      const int by = sy2 ? st[1].bh : st[1].b0;
      const int bz = (DIM == 3) ? (sz2 ? st[2].bh : st[2].b0) : 0;
      const Real fx = sx ? st[0].fh : st[0].f0;
      const Real fy = sy2 ? st[1].fh : st[1].f0;
      const Real fz = (DIM == 3) ? (sz2 ? st[2].fh : st[2].f0) : (Real)0;
      const Real gx = (Real)1 - fx, gy = (Real)1 - fy, gz = (Real)1 - fz;
      Real wt[8];
      wt[0] = gx * gy;
      wt[1] = fx * gy;
      wt[2] = gx * fy;
      wt[3] = fx * fy;
      if (DIM == 3) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          wt[4 + e] = wt[e] * fz;
          wt[e] *= gz;
        }
      }
      if (in) {
        const Real fb = tile_coef(Fbr[r][c], esc);
        const int base = c * T + (bx + dsh[0] - t0[0]) + sy * (by + dsh[1] - t0[1]) +
                         ((DIM == 3) ? sz * (bz + dsh[2] - t0[2]) : 0);
#pragma unroll
        for (int e = 0; e < (1 << DIM); ++e) {
          const int o = (e & 1) + ((e >> 1) & 1) * sy + ((DIM == 3) ? ((e >> 2) & 1) * sz : 0);
          atomic_add_r(tile + base + o, fb * wt[e]);
        }
      } else {
        const Real fb = Fbr[r][c];
        Real *dE = A.dEB + c * (int)g.npts;
        const int np0 = g.np[0], np01 = np0 * g.np[1];
        const int base = pad_index(g, bx, by, bz, DIM);
#pragma unroll
        for (int e = 0; e < (1 << DIM); ++e) {
          const int o = (e & 1) + ((e >> 1) & 1) * np0 + ((DIM == 3) ? ((e >> 2) & 1) * np01 : 0);
          atomic_add_r(dE + base + o, fb * wt[e]);
        }
      }
    }
  }
  __syncthreads();
  // flush: one global atomic per nonzero tile value, periodic images resolved
  const int np0 = g.np[0], np01 = g.np[0] * g.np[1], npts = (int)g.npts;
  constexpr int WA = DIM - 1;  // walked axis
  const int wstride = (DIM == 3) ? np01 : np0;
  bool inside = true;  // uniform: the tile lies inside the padded lattice
#pragma unroll
  for (int d = 0; d < DIM; ++d) inside = inside && t0[d] >= -NG && t0[d] + ts[d] <= g.n[d] + NG;
  if (inside) {  // ghost values are folded into the active cells afterwards
    tile_for_each_affine<8, Acc>(
        6, DIM == 3 ? 2 : 1, ts[0], ts[1], ts[2], npts, wstride,
        [&](int ix, int iy) {
          return pad_index(g, t0[0] + ix, t0[1] + ((DIM == 3) ? iy : 0), t0[2], DIM);
        },
        [&](int, int x) { return tile[x]; },
        [&](int gi, int, Acc acc) {
          if (acc != (Acc)0) atomic_add_r(A.dEB + gi, (Real)ldexp((double)acc, -esc));
        });
    return;
  }
  // (curvilinear: tile points outside the padded lattice hold nothing)
  tile_for_each<8, Acc>(
      6, DIM == 3 ? 2 : 1, ts[0], ts[1], ts[2],
      [&](int ix, int iy) {
        int gx = t0[0] + ix, gy = (DIM == 3) ? t0[1] + iy : 0;
        bool ok = true;
        if (GEOM == 0) {
          gx = wrap_periodic(gx, g.n[0]);
          if (DIM == 3) gy = wrap_periodic(gy, g.n[1]);
        } else {
          ok = gx >= -NG && gx < g.n[0] + NG;
        }
        return PlanePt{(gx + NG) + ((DIM == 3) ? np0 * (gy + NG) : 0), ok};
      },
      [&](const PlanePt &, int x, int, int) { return tile[x]; },
      [&](const PlanePt &pp, int, int comp, int w, Acc acc) {
        if (acc == (Acc)0) return;
        int gw = t0[WA] + w;
        if (GEOM == 0) {
          gw = wrap_periodic(gw, g.n[WA]);
        } else if (!pp.ok || gw < -NG || gw >= g.n[WA] + NG) {
          return;
        }
        const Real v = (Real)ldexp((double)acc, -esc);
        atomic_add_r(A.dEB + comp * npts + pp.off + wstride * (gw + NG), v);
      });
}

template <class Real>
hipError_t launch_adjoint_step(const AdjArgs<Real> &a, hipStream_t s) {
  const int64_t nblk = a.sp.blk0[a.sp.nspec];
  if (nblk == 0) return hipSuccess;
  if (a.g.geom != 0 && !a.lam_phi) return hipErrorInvalidValue;
  dim3 grid((unsigned)nblk), block(BLOCK);
  if (a.g.geom == 0) {
    if (a.g.dim == 2)
      hipLaunchKernelGGL((k_adjoint<0, 2, Real>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_adjoint<0, 3, Real>), grid, block, 0, s, a);
  } else if (a.g.geom == 1) {
    hipLaunchKernelGGL((k_adjoint<1, 2, Real>), grid, block, 0, s, a);
  } else {
    hipLaunchKernelGGL((k_adjoint<2, 2, Real>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

template hipError_t launch_adjoint_step<float>(const AdjArgs<float> &, hipStream_t);
template hipError_t launch_adjoint_step<double>(const AdjArgs<double> &, hipStream_t);

}  // namespace picstep
