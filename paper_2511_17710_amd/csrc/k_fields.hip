// k_fields.hip -- the field update around the particle step (Sec. 2.3 steps
// 2, 9-11): Faraday's and Ampere's laws on the curvilinear Yee lattice in the
// discretized forms of App. A, the polar-axis rules of Sec. 2.6, and the
// digital filter of the conformal current (Sec. 2.5).
//
// These are streaming stencil sweeps over the field arrays (a few bytes per
// lattice point against the tens per particle of the particle step): one
// thread per lattice point (the filter of 3D periodic grids: per column run
// along z), x fastest so that neighbouring lanes read
// neighbouring addresses, every component of the point handled by its thread,
// geometry and dimension fixed at compile time; metric factors are evaluated
// on the fly in FP64 (they are never stored between calls, as in the
// paper), once per row and column of a block's stencils, in LDS; values are
// combined in FP64 and rounded once to the storage precision.
#include "step_device.h"

namespace picstep {

// Yee offsets of (E1, E2, E3, B1, B2, B3) in code units (App. A)
__device__ constexpr double kYee[6][3] = {{0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 0.5},
                                          {0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}};

// the solver's node range along dimension d for a component staggered by
// `half` there: periodic Cartesian [0, N); (quasi-)spherical nodes [0, N]
// (integer points) or cells [0, N) (half-integer points)
template <int GEOM, int DIM>
__device__ __forceinline__ bool in_range(const GridConst &g, int d, int v, bool half) {
  if (d >= DIM) return v == 0;
  if (GEOM == 0) return v >= 0 && v < g.n[d];
  return v >= 0 && v < g.n[d] + (half ? 0 : 1);
}

template <int GEOM, int DIM, int c>
__device__ __forceinline__ bool comp_in_range(const GridConst &g, int i, int j, int k) {
  return in_range<GEOM, DIM>(g, 0, i, kYee[c][0] != 0.0) &&
         in_range<GEOM, DIM>(g, 1, j, kYee[c][1] != 0.0) &&
         in_range<GEOM, DIM>(g, 2, k, kYee[c][2] != 0.0);
}

// The (quasi-)spherical metric factors into a function of x1 (r and
// sqrt(h11)) and one of x2 (the factor of r in sqrt(h22), and sin theta):
// sqrt(h22) = h2f(x2) r(x1), sqrt(h33) = r(x1) sin theta(x2), with the
// arithmetic of the particle step's metric.  A thread evaluates them once
// for each x1 and x2 its stencil touches instead of once per stencil point.
struct MetricRow {
  double r, h1;
};
struct MetricCol {
  double h2f, st;
};
template <int GEOM>
__device__ __forceinline__ MetricRow metric_row(const GridConst &g, double x1) {
  if (GEOM == 1) {
    return {g.rmin + x1 * g.dr, g.dr};
  } else {
    const double eR = exp(g.Rmin + x1 * g.dR);
    return {g.r0 + eR, g.dR * eR};
  }
}
template <int GEOM>
__device__ __forceinline__ MetricCol metric_col(const GridConst &g, double x2) {
  double th, h2f;
  if (GEOM == 1) {
    th = x2 * g.dth;
    h2f = g.dth;
  } else {
    const double T = x2 * g.dT;
    const double tp = T * (1.0 / kPI);
    const double vt = g.vt;
    th = T + 2.0 * vt * T * (1.0 - 2.0 * tp) * (1.0 - tp);
    h2f = g.dT * (1.0 + 2.0 * vt + 12.0 * vt * tp * (tp - 1.0));
  }
  double st, ct;
  sincos(th, &st, &ct);
  return {h2f, st};
}

// The solver kernels take one thread per lattice point on a 2D (3D) launch
// grid: x (the fastest index) over blocks of FX lanes, y over FY rows per
// block, z over planes, so a point's indices need no division.
constexpr int FX = 64, FY = 4;

// A block's metric rows x1 = i0 - 1/2 + t/2 and columns x2 = j0 - 1/2 + t/2
// ((i0, j0) its first point), every half step its threads' stencils touch,
// evaluated once per block in LDS (an exponential per row and a sine per
// column on the quasi-spherical grid, against one per stencil point).
template <int GEOM>
struct MetricTables {
  static constexpr int NR = GEOM != 0 ? 2 * FX + 4 : 1, NC = GEOM != 0 ? 2 * FY + 4 : 1;
  MetricRow r[NR];
  MetricCol c[NC];
};
template <int GEOM>
__device__ __forceinline__ void fill_metric_tables(const GridConst &g, MetricTables<GEOM> &T) {
  if constexpr (GEOM != 0) {
    constexpr int NR = MetricTables<GEOM>::NR, NC = MetricTables<GEOM>::NC;
    const int tid = (int)(threadIdx.x + FX * threadIdx.y);
    const double x0 = (double)(blockIdx.x * FX) - 0.5, y0 = (double)(blockIdx.y * FY) - 0.5;
    if (tid < NR)
      T.r[tid] = metric_row<GEOM>(g, x0 + 0.5 * tid);
    else if (tid < NR + NC)
      T.c[tid - NR] = metric_col<GEOM>(g, y0 + 0.5 * (tid - NR));
    __syncthreads();
  }
}

// The lattice around a thread's point (i, j, k): covariant components and
// sqrt(h) at Yee points addressed relative to it, the metric from the rows
// x1 = i + (q - 1)/2 and columns x2 = j + (q - 1)/2, q = 0..3, of the
// block's tables (the compiler keeps the ones a kernel uses).
template <int GEOM, int DIM, class Real>
struct FieldView {
  const GridConst &g;
  const Real *A;
  int i, j, k;
  MetricRow R[4];
  MetricCol C[4];
  __device__ __forceinline__ FieldView(const GridConst &g_, const Real *A_, int i_, int j_, int k_,
                                       const MetricTables<GEOM> &T)
      : g(g_), A(A_), i(i_), j(j_), k(k_) {
    if constexpr (GEOM != 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        R[q] = T.r[2 * threadIdx.x + q];
        C[q] = T.c[2 * threadIdx.y + q];
      }
    }
  }
  // sqrt(h_mm) at the Yee point of component c of element (i+di, j+dj)
  __device__ __forceinline__ double hm(int c, int m, int di, int dj) const {
    if constexpr (GEOM == 0) {
      return g.dx[m];
    } else {
      const int q1 = 2 * di + (kYee[c][0] != 0.0 ? 1 : 0) + 1;
      const int q2 = 2 * dj + (kYee[c][1] != 0.0 ? 1 : 0) + 1;
      return m == 0 ? R[q1].h1 : (m == 1 ? C[q2].h2f * R[q1].r : R[q1].r * C[q2].st);
    }
  }
  // covariant component m of block f (0: E, 1: B) at element (i+di, j+dj, k+dk)
  __device__ __forceinline__ double cov(int f, int m, int di, int dj, int dk) const {
    const int c = 3 * f + m;
    const double h = hm(c, m, di, dj);
    return h * h * (double)A[c * (int)g.npts + pad_index(g, i + di, j + dj, k + dk, DIM)];
  }
  // sqrt(h) = sqrt(h11 h22 h33) at the Yee point of component c of the point
  __device__ __forceinline__ double sqrt_det(int c) const {
    return hm(c, 0, 0, 0) * hm(c, 1, 0, 0) * hm(c, 2, 0, 0);
  }
};

template <int GEOM>
__device__ __forceinline__ bool axis_node(const GridConst &g, int j) {
  return GEOM != 0 && (j == 0 || j == g.n[1]);
}

// the extents of the points the solver updates (any component)
template <int GEOM, int DIM>
__device__ __forceinline__ bool solver_point(const GridConst &g, int &i, int &j, int &k) {
  i = (int)(blockIdx.x * FX + threadIdx.x);
  j = (int)(blockIdx.y * FY + threadIdx.y);
  k = (int)blockIdx.z;
  return i < g.n[0] + (GEOM != 0 ? 1 : 0) && j < g.n[1] + (GEOM != 0 ? 1 : 0);
}

// Faraday (App. A, eq. discretized-faraday): B^i -= f (curl E)^i / sqrt(h),
// the curl of the covariant E_m = h_mm E^m over unit code cells; B2 on the
// axis nodes stays 0 (Sec. 2.6)
template <int GEOM, int DIM, class Real>
__global__ __launch_bounds__(FX *FY) void k_faraday(GridConst g, Real *EB, double f) {
  __shared__ MetricTables<GEOM> mt;
  fill_metric_tables<GEOM>(g, mt);  // every thread of the block, before any returns
  int i, j, k;
  if (!solver_point<GEOM, DIM>(g, i, j, k)) return;
  const FieldView<GEOM, DIM, Real> V(g, EB, i, j, k, mt);
  constexpr bool d3 = DIM == 3;
  const int npts = (int)g.npts;
  const int at = pad_index(g, i, j, k, DIM);
  if (comp_in_range<GEOM, DIM, 3>(g, i, j, k)) {  // B1 at (i, j+1/2, k+1/2)
    double curl = V.cov(0, 2, 0, 1, 0) - V.cov(0, 2, 0, 0, 0);
    if (d3) curl -= V.cov(0, 1, 0, 0, 1) - V.cov(0, 1, 0, 0, 0);
    Real *dst = EB + 3 * npts + at;
    *dst = (Real)((double)*dst - f * curl / V.sqrt_det(3));
  }
  if (comp_in_range<GEOM, DIM, 4>(g, i, j, k)) {  // B2 at (i+1/2, j, k+1/2)
    Real *dst = EB + 4 * npts + at;
    if (axis_node<GEOM>(g, j)) {
      *dst = (Real)0;
    } else {
      double curl = -(V.cov(0, 2, 1, 0, 0) - V.cov(0, 2, 0, 0, 0));
      if (d3) curl += V.cov(0, 0, 0, 0, 1) - V.cov(0, 0, 0, 0, 0);
      *dst = (Real)((double)*dst - f * curl / V.sqrt_det(4));
    }
  }
  if (comp_in_range<GEOM, DIM, 5>(g, i, j, k)) {  // B3 at (i+1/2, j+1/2, k)
    const double curl = (V.cov(0, 1, 1, 0, 0) - V.cov(0, 1, 0, 0, 0)) -
                        (V.cov(0, 0, 0, 1, 0) - V.cov(0, 0, 0, 0, 0));
    Real *dst = EB + 5 * npts + at;
    *dst = (Real)((double)*dst - f * curl / V.sqrt_det(5));
  }
}

// Sec. 2.6: integral over x2 in [0, 1/2] of sqrt(h), in closed form
template <int GEOM>
__device__ __forceinline__ double polar_area(const GridConst &g, double x1) {
  if (GEOM == 1) {
    const double r = g.rmin + x1 * g.dr;
    return r * r * g.dr * (1.0 - cos(0.5 * g.dth));
  }
  const double eR = exp(g.Rmin + x1 * g.dR);
  const double r = g.r0 + eR;
  const double tt = 0.5 * g.dT + g.vt * g.dT * (1.0 - g.dT / kPI) * (1.0 - g.dT / (2.0 * kPI));
  return r * r * eR * g.dR * (1.0 - cos(tt));
}

// Ampere (App. A, eq. discretized-ampere): E^i += dt ((curl B)^i - coupling
// J^i) / sqrt(h); on the axis nodes E3 = 0 and E1 takes the update
// integrated over the half cell next to the axis, A dE1/dt = +-B_3 -
// (coupling / 2) J1 (Sec. 2.6)
template <int GEOM, int DIM, class Real>
__global__ __launch_bounds__(FX *FY) void k_ampere(GridConst g, Real *EB, const Real *J, double dt,
                                                  double coupling) {
  __shared__ MetricTables<GEOM> mt;
  fill_metric_tables<GEOM>(g, mt);  // every thread of the block, before any returns
  int i, j, k;
  if (!solver_point<GEOM, DIM>(g, i, j, k)) return;
  const FieldView<GEOM, DIM, Real> V(g, EB, i, j, k, mt);
  constexpr bool d3 = DIM == 3;
  const int npts = (int)g.npts;
  const int pt = pad_index(g, i, j, k, DIM);
  if (comp_in_range<GEOM, DIM, 0>(g, i, j, k)) {  // E1 at (i+1/2, j, k)
    const double Jc = (double)J[pt];
    double v = (double)EB[pt];
    if (axis_node<GEOM>(g, j)) {
      const double b3 = (j == 0) ? V.cov(1, 2, 0, 0, 0) : -V.cov(1, 2, 0, -1, 0);
      if constexpr (GEOM != 0) v += dt * (b3 - 0.5 * coupling * Jc) / polar_area<GEOM>(g, i + 0.5);
    } else {
      double curl = V.cov(1, 2, 0, 0, 0) - V.cov(1, 2, 0, -1, 0);
      if (d3) curl -= V.cov(1, 1, 0, 0, 0) - V.cov(1, 1, 0, 0, -1);
      v += dt * (curl - coupling * Jc) / V.sqrt_det(0);
    }
    EB[pt] = (Real)v;
  }
  if (comp_in_range<GEOM, DIM, 1>(g, i, j, k)) {  // E2 at (i, j+1/2, k)
    const int at = npts + pt;
    double curl = -(V.cov(1, 2, 0, 0, 0) - V.cov(1, 2, -1, 0, 0));
    if (d3) curl += V.cov(1, 0, 0, 0, 0) - V.cov(1, 0, 0, 0, -1);
    EB[at] = (Real)((double)EB[at] + dt * (curl - coupling * (double)J[at]) /
                                         V.sqrt_det(1));
  }
  if (comp_in_range<GEOM, DIM, 2>(g, i, j, k)) {  // E3 at (i, j, k+1/2)
    const int at = 2 * npts + pt;
    if (axis_node<GEOM>(g, j)) {
      EB[at] = (Real)0;
    } else {
      const double curl = (V.cov(1, 1, 0, 0, 0) - V.cov(1, 1, -1, 0, 0)) -
                          (V.cov(1, 0, 0, 0, 0) - V.cov(1, 0, 0, -1, 0));
      EB[at] = (Real)((double)EB[at] + dt * (curl - coupling * (double)J[at]) /
                                           V.sqrt_det(2));
    }
  }
}

// J of component c at element (i, j, k) as the filter sees it: periodic
// Cartesian grids wrap; (quasi-)spherical grids mirror across the axes
// (J1 even about an axis node, J2 odd about it, J3 zero on it) and read the
// stored values across the radial edges
template <int GEOM, int DIM, class Real>
__device__ __forceinline__ double j_filter_at(const GridConst &g, const Real *J, int c, int i, int j,
                                              int k) {
  if constexpr (GEOM == 0) {
    int ii[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      ii[d] += (ii[d] < 0) ? g.n[d] : 0;
      ii[d] -= (ii[d] >= g.n[d]) ? g.n[d] : 0;
    }
    return (double)J[c * (int)g.npts + pad_index(g, ii[0], ii[1], ii[2], DIM)];
  } else {
    const int n2 = g.n[1];
    int jj = j;
    double sgn = 1.0;
    if (c == 2 && (j == 0 || j == n2)) return 0.0;
    if (c == 1) {
      if (j < 0) {
        jj = -1 - j;
        sgn = -1.0;
      } else if (j >= n2) {
        jj = 2 * n2 - 1 - j;
        sgn = -1.0;
      }
    } else {
      if (j < 0) jj = -j;
      else if (j > n2) jj = 2 * n2 - j;
    }
    return sgn * (double)J[c * (int)g.npts + pad_index(g, i, jj, k, DIM)];
  }
}

// one filter pass (Sec. 2.5, eq. 2d-filter and its 3D form): weights
// (1/2)^(D + |di| + |dj| + |dk|) = prod_d (1/2)^(1 + |d|) over the 3^D
// neighbours of each point of the solver's node ranges; every other point
// (ghosts, the extra node of half-staggered components) is copied.  One
// thread per padded lattice point; z runs over component x plane.
template <int GEOM, int DIM, class Real>
__global__ __launch_bounds__(FX *FY) void k_filter(GridConst g, const Real *in, Real *out, int np2) {
  const int ip = (int)(blockIdx.x * FX + threadIdx.x), jp = (int)(blockIdx.y * FY + threadIdx.y);
  if (ip >= g.np[0] || jp >= g.np[1]) return;
  const int c = (int)blockIdx.z / np2, kp = (int)blockIdx.z - c * np2;
  const int i = ip - NG, j = jp - NG, k = (DIM == 3) ? kp - NG : 0;
  const int q = c * (int)g.npts + ip + g.np[0] * (jp + g.np[1] * kp);
  const bool upd = in_range<GEOM, DIM>(g, 0, i, kYee[c][0] != 0.0) &&
                   in_range<GEOM, DIM>(g, 1, j, kYee[c][1] != 0.0) &&
                   in_range<GEOM, DIM>(g, 2, k, kYee[c][2] != 0.0);
  if (!upd) {
    out[q] = in[q];
    return;
  }
  if (c == 2 && axis_node<GEOM>(g, j)) {
    out[q] = (Real)0;
    return;
  }
  constexpr int kr = (DIM == 3) ? 1 : 0;
  double acc = 0.0;
  // a stencil whose rows and planes are clear of the periodic seams
  // (Cartesian) or of the axis rows (where the mirror rules apply; a wave is
  // one row, so this is uniform over it) reads its neighbours at fixed
  // offsets, the x neighbours wrapped per lane on periodic grids
  bool clear;
  if constexpr (GEOM == 0) {
    clear = j >= 1 && j <= g.n[1] - 2;
    if (DIM == 3) clear = clear && k >= 1 && k <= g.n[2] - 2;
  } else {
    clear = j >= 2 && j <= g.n[1] - 2;
  }
  if (clear) {
    const Real *b = in + q;
    const int s1 = g.np[0], s2 = g.np[0] * g.np[1];
    const int om = (GEOM == 0 && i == 0) ? g.n[0] - 1 : -1;
    const int op = (GEOM == 0 && i == g.n[0] - 1) ? 1 - g.n[0] : 1;
#pragma unroll
    for (int dk = -kr; dk <= kr; ++dk) {
      const double wz = (DIM == 3) ? (dk == 0 ? 0.5 : 0.25) : 1.0;
#pragma unroll
      for (int dj = -1; dj <= 1; ++dj) {
        const double wyz = wz * (dj == 0 ? 0.5 : 0.25);
        const Real *row = b + dj * s1 + dk * s2;
        acc += wyz * 0.25 * (double)row[om];
        acc += wyz * 0.5 * (double)row[0];
        acc += wyz * 0.25 * (double)row[op];
      }
    }
    out[q] = (Real)acc;
    return;
  }
#pragma unroll
  for (int dk = -kr; dk <= kr; ++dk) {
    const double wz = (DIM == 3) ? (dk == 0 ? 0.5 : 0.25) : 1.0;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      const double wyz = wz * (dj == 0 ? 0.5 : 0.25);
#pragma unroll
      for (int di = -1; di <= 1; ++di)
        acc += wyz * (di == 0 ? 0.5 : 0.25) *
               j_filter_at<GEOM, DIM, Real>(g, in, c, i + di, j + dj, k + dk);
    }
  }
  out[q] = (Real)acc;
}

// The filter pass on 3D periodic Cartesian grids as a sweep along z: a
// thread owns an (x, y) column of one component over a run of planes,
// forms each plane's 3x3 weighted sum once (9 reads) and combines three
// consecutive plane sums per output (the weights factor per dimension), so
// an output costs 9 reads instead of 27.  Columns outside the updated range
// (ghosts) and ghost planes are copied.  z of the launch grid: component x
// run of ZRUN planes.
constexpr int ZRUN = 16;
template <class Real>
__global__ __launch_bounds__(FX *FY) void k_filter_zsweep(GridConst g, const Real *in, Real *out,
                                                          int nrun) {
  const int ip = (int)(blockIdx.x * FX + threadIdx.x), jp = (int)(blockIdx.y * FY + threadIdx.y);
  if (ip >= g.np[0] || jp >= g.np[1]) return;
  const int c = (int)blockIdx.z / nrun, run = (int)blockIdx.z - c * nrun;
  const int np2 = g.np[2];
  const int kp0 = run * ZRUN, kp1 = min(np2, kp0 + ZRUN);
  const int s1 = g.np[0], s2 = g.np[0] * g.np[1];
  const Real *src = in + (int64_t)c * g.npts;
  Real *dst = out + (int64_t)c * g.npts;
  const int col = ip + s1 * jp;
  const int i = ip - NG, j = jp - NG;
  if (i < 0 || i >= g.n[0] || j < 0 || j >= g.n[1]) {  // a ghost column: copied
    for (int kp = kp0; kp < kp1; ++kp) dst[col + s2 * kp] = src[col + s2 * kp];
    return;
  }
  // x and y neighbours of the column, wrapped
  const int xm = (i == 0) ? g.n[0] - 1 : -1, xp = (i == g.n[0] - 1) ? 1 - g.n[0] : 1;
  const int ym = ((j == 0) ? g.n[1] - 1 : -1) * s1, yp = ((j == g.n[1] - 1) ? 1 - g.n[1] : 1) * s1;
  const int n2 = g.n[2];
  // weighted 3x3 sum of plane k (wrapped into [0, n2))
  auto plane = [&](int k) {
    k += (k < 0) ? n2 : 0;
    k -= (k >= n2) ? n2 : 0;
    const Real *b = src + col + s2 * (k + NG);
    const Real *rows[3] = {b + ym, b, b + yp};
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double wy = (r == 1) ? 0.5 : 0.25;
      acc += wy * 0.25 * (double)rows[r][xm];
      acc += wy * 0.5 * (double)rows[r][0];
      acc += wy * 0.25 * (double)rows[r][xp];
    }
    return acc;
  };
  double pm = 0.0, pc = 0.0;
  bool primed = false;
  for (int kp = kp0; kp < kp1; ++kp) {
    const int k = kp - NG;
    if (k < 0 || k >= n2) {  // a ghost plane: copied
      dst[col + s2 * kp] = src[col + s2 * kp];
      continue;
    }
    if (!primed) {
      pm = plane(k - 1);
      pc = plane(k);
      primed = true;
    }
    const double pn = plane(k + 1);
    dst[col + s2 * kp] = (Real)(0.25 * pm + 0.5 * pc + 0.25 * pn);
    pm = pc;
    pc = pn;
  }
}

dim3 solver_grid(const GridConst &g) {
  const unsigned e0 = (unsigned)(g.n[0] + (g.geom != 0 ? 1 : 0));
  const unsigned e1 = (unsigned)(g.n[1] + (g.geom != 0 ? 1 : 0));
  const unsigned e2 = (unsigned)((g.dim == 3) ? g.n[2] : 1);
  return dim3((e0 + FX - 1) / FX, (e1 + FY - 1) / FY, e2);
}

// the instance of a solver kernel for the grid's geometry and dimension
#define PIC_FIELD_LAUNCH(KERNEL, GRID, ...)                                                \
  do {                                                                                     \
    if (g.geom == 0 && g.dim == 3)                                                         \
      hipLaunchKernelGGL((KERNEL<0, 3, Real>), GRID, dim3(FX, FY), 0, s, __VA_ARGS__);     \
    else if (g.geom == 0)                                                                  \
      hipLaunchKernelGGL((KERNEL<0, 2, Real>), GRID, dim3(FX, FY), 0, s, __VA_ARGS__);     \
    else if (g.geom == 1)                                                                  \
      hipLaunchKernelGGL((KERNEL<1, 2, Real>), GRID, dim3(FX, FY), 0, s, __VA_ARGS__);     \
    else                                                                                   \
      hipLaunchKernelGGL((KERNEL<2, 2, Real>), GRID, dim3(FX, FY), 0, s, __VA_ARGS__);     \
  } while (0)

template <class Real>
hipError_t launch_faraday(const GridConst &g, Real *EB, double f, hipStream_t s) {
  PIC_FIELD_LAUNCH(k_faraday, solver_grid(g), g, EB, f);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_fill_ghosts<Real>(g, EB + 3 * g.npts, 3, s);
  return e;
}

template <class Real>
hipError_t launch_ampere(const GridConst &g, Real *EB, const Real *J, double dt, double coupling,
                         hipStream_t s) {
  PIC_FIELD_LAUNCH(k_ampere, solver_grid(g), g, EB, J, dt, coupling);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_fill_ghosts<Real>(g, EB, 3, s);
  return e;
}

template <class Real>
hipError_t launch_filter(const GridConst &g, const Real *in, Real *out, hipStream_t s) {
  if (g.geom == 0 && g.dim == 3) {
    const int nrun = (g.np[2] + ZRUN - 1) / ZRUN;
    const dim3 grid((unsigned)((g.np[0] + FX - 1) / FX), (unsigned)((g.np[1] + FY - 1) / FY),
                    (unsigned)(3 * nrun));
    hipLaunchKernelGGL(k_filter_zsweep<Real>, grid, dim3(FX, FY), 0, s, g, in, out, nrun);
    return hipGetLastError();
  }
  const int np2 = (int)(g.npts / ((int64_t)g.np[0] * g.np[1]));
  const dim3 grid((unsigned)((g.np[0] + FX - 1) / FX), (unsigned)((g.np[1] + FY - 1) / FY),
                  (unsigned)(3 * np2));
  PIC_FIELD_LAUNCH(k_filter, grid, g, in, out, np2);
  return hipGetLastError();
}

#undef PIC_FIELD_LAUNCH

template hipError_t launch_faraday<float>(const GridConst &, float *, double, hipStream_t);
template hipError_t launch_faraday<double>(const GridConst &, double *, double, hipStream_t);
template hipError_t launch_ampere<float>(const GridConst &, float *, const float *, double, double,
                                         hipStream_t);
template hipError_t launch_ampere<double>(const GridConst &, double *, const double *, double,
                                          double, hipStream_t);
template hipError_t launch_filter<float>(const GridConst &, const float *, float *, hipStream_t);
template hipError_t launch_filter<double>(const GridConst &, const double *, double *,
                                          hipStream_t);

}  // namespace picstep
