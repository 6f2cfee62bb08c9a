// k_push.hip -- fused particle step: interpolate, rotate, Boris, move, deposit
// (arXiv 2511.17710, Sec. 2.3 steps 3-8), one thread per particle, one launch
// for all species.
#include "step_device.h"

namespace picstep {

// ---------------------------------------------------------------- Cartesian grids
// Tetrad on a Cartesian grid: F^i_hat = Delta_i F^i (eq. curvspace-tetradtrans,
// Sec. 2.4 Cartesian metric; h33 = 1 in 2D); the basis is already global.
template <int DIM, class Real>
__global__ __launch_bounds__(BLOCK) void k_push_cart(StepArgs<Real> A) {
  using PS = Pos<Real>;
  int s;
  int64_t local;
  if (!locate(A.sp, s, local)) return;
  const int64_t p = A.sp.off[s] + local;
  const GridConst &g = A.g;
  const int32_t c = A.p.cell[p];
  OffT<Real> q[3];
  Real d[3];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    q[a] = A.p.offs[a][p];
    d[a] = (Real)PS::weight(q[a]);
  }
  if (A.write_prev) {
    A.prev_cell[p] = c;
#pragma unroll
    for (int a = 0; a < DIM; ++a) A.prev_offs[a][p] = q[a];
  }
  if (c & DEAD_BIT) return;
  int i[3];
  cell_decode(g, c, i);

  Stencil1<Real> st[3];
#pragma unroll
  for (int a = 0; a < DIM; ++a) st[a] = stencil1(i[a], d[a]);
  Real F[6];
  interp6<DIM, Real>(A.EB, g, st, F);

  Real E[3], B[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const Real sc = (a < DIM) ? (Real)g.dx[a] : (Real)1;
    E[a] = F[a] * sc;
    B[a] = F[3 + a] * sc;
  }
  Real u[3] = {A.p.u[0][p], A.p.u[1][p], A.p.u[2][p]};
  const Real k = (Real)A.sp.k[s];
  boris(k, E, B, u);

  // move (steps 6-7): offsets advance by dt u / (gamma Delta)
  const Real gi = rsqrt_r((Real)1 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const Real dtr = (Real)A.dt;
  int m[3] = {0, 0, 0};
  OffT<Real> qn[3];
  double za[3] = {0, 0, 0}, zb[3] = {0, 0, 0};
  int inew[3] = {i[0], i[1], i[2]};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const Real dx = dtr * u[a] * gi / (Real)g.dx[a];
    m[a] = PS::move(q[a], (double)dx, qn[a]);
    za[a] = PS::exact(q[a]);
    zb[a] = PS::exact(qn[a]) + (double)m[a];
    int v = i[a] + m[a];
    v = (v < 0) ? v + g.n[a] : ((v >= g.n[a]) ? v - g.n[a] : v);  // periodic wrap
    inew[a] = v;
  }
  const Real dx3 = (DIM == 2) ? dtr * u[2] * gi : (Real)0;

  // deposit (step 8) with the unwrapped step m; ghosts are folded afterwards
  ZigZag<Real> z;
  zigzag<DIM, Real>(za, m, zb, z);
  const Real C = (Real)A.sp.qdt[s] * A.p.w[p];
  deposit<DIM, Real>(A.J, g, C, i, m, z, dx3);

  A.p.cell[p] = cell_encode(g, inew);
#pragma unroll
  for (int a = 0; a < DIM; ++a) A.p.offs[a][p] = qn[a];
  A.p.u[0][p] = u[0];
  A.p.u[1][p] = u[1];
  A.p.u[2][p] = u[2];
}

// ---------------------------------------------------------------- axisymmetric grids
// Tetrad (F^i_hat = sqrt(h_ii) F^i at x_p) and rotation of (r, theta, phi)_hat
// into (x, y, z)_hat (Sec. 2.3 step 4), Boris in the global basis, then the
// offset-relative move.  Metric and move run in CT (FP64 near the axis and
// r_min when Real is float).
template <int GEOM, class CT, class Real, class D>
__device__ __forceinline__ void axi_particle(const GridConst &g, Real k, double dt, int i1, int i2,
                                             D d1, D d2, Real phi, const Real F[6],
                                             Real u[3], CT &dx1, CT &dx2, CT &dphi) {
  const CT x1 = (CT)i1 + (CT)d1;
  const CT x2 = (CT)i2 + (CT)d2;
  const AxiMetric<CT> M = axi_metric<GEOM, CT>(g, x1, x2);
  CT sp, cp;
  sincos_r((CT)phi, &sp, &cp);
  Real E[3], B[3];
  {
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
  boris(k, E, B, u);
  const CT uu0 = (CT)u[0], uu1 = (CT)u[1], uu2 = (CT)u[2];
  const CT gi = rsqrt_r((CT)1 + uu0 * uu0 + uu1 * uu1 + uu2 * uu2);
  const CT dtg = (CT)dt * gi;
  axi_move<GEOM, CT>(g, M, x2, sp, cp, dtg * uu0, dtg * uu1, dtg * uu2, dx1, dx2, dphi);
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

template <int GEOM, class Real>
__global__ __launch_bounds__(BLOCK) void k_push_axi(StepArgs<Real> A) {
  using PS = Pos<Real>;
  int s;
  int64_t local;
  if (!locate(A.sp, s, local)) return;
  const int64_t p = A.sp.off[s] + local;
  const GridConst &g = A.g;
  const int32_t c = A.p.cell[p];
  const OffT<Real> q1 = A.p.offs[0][p], q2 = A.p.offs[1][p];
  if (A.write_prev) {
    A.prev_cell[p] = c;
    A.prev_offs[0][p] = q1;
    A.prev_offs[1][p] = q2;
  }
  if (c & DEAD_BIT) return;
  const Real d1 = (Real)PS::weight(q1), d2 = (Real)PS::weight(q2);
  int i[3];
  cell_decode(g, c, i);
  Stencil1<Real> st[3];
  st[0] = stencil1(i[0], d1);
  st[1] = stencil1(i[1], d2);
  Real F[6];
  interp6<2, Real>(A.EB, g, st, F);
  Real u[3] = {A.p.u[0][p], A.p.u[1][p], A.p.u[2][p]};
  const Real phi = A.p.phi[p];
  const Real k = (Real)A.sp.k[s];

  double dx1, dx2;
  Real phinew, dx3;
  const bool near = (i[0] < g.fp64_cells) || (i[1] < g.fp64_cells) ||
                    (i[1] >= g.n[1] - g.fp64_cells);
  if (sizeof(Real) == 8 || near) {
    double dphi;
    axi_particle<GEOM, double, Real>(g, k, A.dt, i[0], i[1], PS::exact(q1), PS::exact(q2), phi, F,
                                     u, dx1, dx2, dphi);
    phinew = next_phi<Real, double>(phi, dphi);
    dx3 = (Real)dphi;
  } else {
    float f1, f2, dphi;
    axi_particle<GEOM, float, Real>(g, k, A.dt, i[0], i[1], d1, d2, phi, F, u, f1, f2, dphi);
    dx1 = f1;
    dx2 = f2;
    phinew = next_phi<Real, float>(phi, dphi);
    dx3 = (Real)dphi;
  }
  int m[3] = {0, 0, 0};
  OffT<Real> qn1, qn2;
  m[0] = PS::move(q1, dx1, qn1);
  m[1] = PS::move(q2, dx2, qn2);
  int inew[3] = {i[0] + m[0], i[1] + m[1], 0};
  // theta stays in [0, pi]: clamp rounding excursions
  if (inew[1] < 0) {
    inew[1] = 0;
    qn2 = (OffT<Real>)0;
  } else if (inew[1] >= g.n[1]) {
    inew[1] = g.n[1] - 1;
    qn2 = largest_offset<Real>();
  }
  m[1] = inew[1] - i[1];
  const bool alive = inew[0] >= 0 && inew[0] < g.n[0];  // radial exit

  const double za[3] = {PS::exact(q1), PS::exact(q2), 0.0};
  const double zb[3] = {PS::exact(qn1) + (double)m[0], PS::exact(qn2) + (double)m[1], 0.0};
  ZigZag<Real> z;
  zigzag<2, Real>(za, m, zb, z);
  const Real C = (Real)A.sp.qdt[s] * A.p.w[p];
  deposit<2, Real>(A.J, g, C, i, m, z, dx3);

  A.p.cell[p] = cell_encode(g, inew) | (alive ? 0 : DEAD_BIT);
  A.p.offs[0][p] = qn1;
  A.p.offs[1][p] = qn2;
  A.p.phi[p] = phinew;
  A.p.u[0][p] = u[0];
  A.p.u[1][p] = u[1];
  A.p.u[2][p] = u[2];
}

template <class Real>
hipError_t launch_push_deposit(const StepArgs<Real> &a, hipStream_t s) {
  const int64_t nblk = a.sp.blk0[a.sp.nspec];
  if (nblk == 0) return hipSuccess;
  dim3 grid((unsigned)nblk), block(BLOCK);
  if (a.g.geom == 0) {
    if (a.g.dim == 2)
      hipLaunchKernelGGL((k_push_cart<2, Real>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_push_cart<3, Real>), grid, block, 0, s, a);
  } else if (a.g.geom == 1) {
    hipLaunchKernelGGL((k_push_axi<1, Real>), grid, block, 0, s, a);
  } else {
    hipLaunchKernelGGL((k_push_axi<2, Real>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

template hipError_t launch_push_deposit<float>(const StepArgs<float> &, hipStream_t);
template hipError_t launch_push_deposit<double>(const StepArgs<double> &, hipStream_t);

}  // namespace picstep
