// k_fields.hip -- the field update around the particle step (Sec. 2.3 steps
// 2, 9-11): Faraday's and Ampere's laws on the curvilinear Yee lattice in the
// discretized forms of App. A, the polar-axis rules of Sec. 2.6, and the
// digital filter of the conformal current (Sec. 2.5).
//
// These are streaming stencil sweeps over the field arrays (a few bytes per
// lattice point against the tens per particle of the particle step): one
// thread per lattice point, x fastest so that neighbouring lanes read
// neighbouring addresses, every component of the point handled by its thread;
// metric factors are evaluated on the fly in FP64 (they are never stored,
// as in the paper), values are combined in FP64 and rounded once to the
// storage precision.
#include "step_device.h"

namespace picstep {

constexpr int FT = 256;

// Yee offsets of (E1, E2, E3, B1, B2, B3) in code units (App. A)
__device__ constexpr double kYee[6][3] = {{0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 0.5},
                                          {0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}};

// sqrt(h_ii) at code coordinates (Sec. 2.4; x3 plays no role)
__device__ __forceinline__ void metric_at(const GridConst &g, double x1, double x2, double h[3]) {
  if (g.geom == 0) {
    h[0] = g.dx[0];
    h[1] = g.dx[1];
    h[2] = g.dx[2];
    return;
  }
  const AxiMetric<double> M =
      g.geom == 1 ? axi_metric<1, double>(g, x1, x2) : axi_metric<2, double>(g, x1, x2);
  h[0] = M.h1;
  h[1] = M.h2;
  h[2] = M.h3;
}

// the solver's node range along dimension d for a component staggered by
// `half` there: periodic Cartesian [0, N); (quasi-)spherical nodes [0, N]
// (integer points) or cells [0, N) (half-integer points)
__device__ __forceinline__ bool in_range(const GridConst &g, int d, int v, bool half) {
  if (d >= g.dim) return v == 0;
  if (g.geom == 0) return v >= 0 && v < g.n[d];
  return v >= 0 && v < g.n[d] + (half ? 0 : 1);
}

template <class Real>
struct FieldView {
  const GridConst &g;
  const Real *A;
  // covariant component m of block f (0: E, 1: B) at element (i, j, k)
  __device__ __forceinline__ double cov(int f, int m, int i, int j, int k) const {
    const int c = 3 * f + m;
    double h[3];
    metric_at(g, i + kYee[c][0], j + kYee[c][1], h);
    return h[m] * h[m] * (double)A[c * (int)g.npts + pad_index(g, i, j, k, g.dim)];
  }
};

__device__ __forceinline__ double sqrt_det(const GridConst &g, int c, int i, int j) {
  double h[3];
  metric_at(g, i + kYee[c][0], j + kYee[c][1], h);
  return h[0] * h[1] * h[2];
}

__device__ __forceinline__ bool axis_node(const GridConst &g, int j) {
  return g.geom != 0 && (j == 0 || j == g.n[1]);
}

// thread -> lattice point over the extents the solver updates
__device__ __forceinline__ bool point_of(const GridConst &g, int q, int &i, int &j, int &k) {
  const int e0 = g.n[0] + (g.geom != 0 ? 1 : 0);
  const int e1 = g.n[1] + (g.geom != 0 ? 1 : 0);
  const int e2 = (g.dim == 3) ? g.n[2] : 1;
  if (q >= e0 * e1 * e2) return false;
  i = q % e0;
  q /= e0;
  j = q % e1;
  k = q / e1;
  return true;
}

// Faraday (App. A, eq. discretized-faraday): B^i -= f (curl E)^i / sqrt(h),
// the curl of the covariant E_m = h_mm E^m over unit code cells; B2 on the
// axis nodes stays 0 (Sec. 2.6)
template <class Real>
__global__ __launch_bounds__(FT) void k_faraday(GridConst g, Real *EB, double f) {
  int i, j, k;
  if (!point_of(g, blockIdx.x * FT + threadIdx.x, i, j, k)) return;
  const FieldView<Real> V{g, EB};
  const bool d3 = g.dim == 3;
  const int npts = (int)g.npts;
  for (int c = 3; c < 6; ++c) {
    if (!in_range(g, 0, i, kYee[c][0] != 0.0) || !in_range(g, 1, j, kYee[c][1] != 0.0) ||
        !in_range(g, 2, k, kYee[c][2] != 0.0))
      continue;
    Real *dst = EB + c * npts + pad_index(g, i, j, k, g.dim);
    if (c == 4 && axis_node(g, j)) {
      *dst = (Real)0;
      continue;
    }
    double curl;
    if (c == 3) {  // B1 at (i, j+1/2, k+1/2)
      curl = V.cov(0, 2, i, j + 1, k) - V.cov(0, 2, i, j, k);
      if (d3) curl -= V.cov(0, 1, i, j, k + 1) - V.cov(0, 1, i, j, k);
    } else if (c == 4) {  // B2 at (i+1/2, j, k+1/2)
      curl = -(V.cov(0, 2, i + 1, j, k) - V.cov(0, 2, i, j, k));
      if (d3) curl += V.cov(0, 0, i, j, k + 1) - V.cov(0, 0, i, j, k);
    } else {  // B3 at (i+1/2, j+1/2, k)
      curl = (V.cov(0, 1, i + 1, j, k) - V.cov(0, 1, i, j, k)) -
             (V.cov(0, 0, i, j + 1, k) - V.cov(0, 0, i, j, k));
    }
    *dst = (Real)((double)*dst - f * curl / sqrt_det(g, c, i, j));
  }
}

// Sec. 2.6: integral over x2 in [0, 1/2] of sqrt(h), in closed form
__device__ __forceinline__ double polar_area(const GridConst &g, double x1) {
  if (g.geom == 1) {
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
template <class Real>
__global__ __launch_bounds__(FT) void k_ampere(GridConst g, Real *EB, const Real *J, double dt,
                                              double coupling) {
  int i, j, k;
  if (!point_of(g, blockIdx.x * FT + threadIdx.x, i, j, k)) return;
  const FieldView<Real> V{g, EB};
  const bool d3 = g.dim == 3;
  const int npts = (int)g.npts;
  for (int c = 0; c < 3; ++c) {
    if (!in_range(g, 0, i, kYee[c][0] != 0.0) || !in_range(g, 1, j, kYee[c][1] != 0.0) ||
        !in_range(g, 2, k, kYee[c][2] != 0.0))
      continue;
    const int at = c * npts + pad_index(g, i, j, k, g.dim);
    const double Jc = (double)J[at];
    double v = (double)EB[at];
    if (c == 2 && axis_node(g, j)) {
      v = 0.0;
    } else if (c == 0 && axis_node(g, j)) {
      const double b3 = (j == 0) ? V.cov(1, 2, i, 0, k) : -V.cov(1, 2, i, j - 1, k);
      v += dt * (b3 - 0.5 * coupling * Jc) / polar_area(g, i + 0.5);
    } else {
      double curl;
      if (c == 0) {  // E1 at (i+1/2, j, k)
        curl = V.cov(1, 2, i, j, k) - V.cov(1, 2, i, j - 1, k);
        if (d3) curl -= V.cov(1, 1, i, j, k) - V.cov(1, 1, i, j, k - 1);
      } else if (c == 1) {  // E2 at (i, j+1/2, k)
        curl = -(V.cov(1, 2, i, j, k) - V.cov(1, 2, i - 1, j, k));
        if (d3) curl += V.cov(1, 0, i, j, k) - V.cov(1, 0, i, j, k - 1);
      } else {  // E3 at (i, j, k+1/2)
        curl = (V.cov(1, 1, i, j, k) - V.cov(1, 1, i - 1, j, k)) -
               (V.cov(1, 0, i, j, k) - V.cov(1, 0, i, j - 1, k));
      }
      v += dt * (curl - coupling * Jc) / sqrt_det(g, c, i, j);
    }
    EB[at] = (Real)v;
  }
}

// J of component c at element (i, j, k) as the filter sees it: periodic
// Cartesian grids wrap; (quasi-)spherical grids mirror across the axes
// (J1 even about an axis node, J2 odd about it, J3 zero on it) and read the
// stored values across the radial edges
template <class Real>
__device__ __forceinline__ double j_filter_at(const GridConst &g, const Real *J, int c, int i, int j,
                                              int k) {
  if (g.geom == 0) {
    int ii[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (d < g.dim) {
        ii[d] += (ii[d] < 0) ? g.n[d] : 0;
        ii[d] -= (ii[d] >= g.n[d]) ? g.n[d] : 0;
      }
    return (double)J[c * (int)g.npts + pad_index(g, ii[0], ii[1], ii[2], g.dim)];
  }
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
  return sgn * (double)J[c * (int)g.npts + pad_index(g, i, jj, k, g.dim)];
}

// one filter pass (Sec. 2.5, eq. 2d-filter and its 3D form): weights
// (1/2)^(D + |di| + |dj| + |dk|) over the 3^D neighbours of each point of the
// solver's node ranges; every other point is copied
template <class Real>
__global__ __launch_bounds__(FT) void k_filter(GridConst g, const Real *in, Real *out) {
  const int q = blockIdx.x * FT + threadIdx.x;
  const int npts = (int)g.npts;
  if (q >= 3 * npts) return;
  const int c = q / npts;
  int r = q - c * npts;
  const int i = r % g.np[0] - NG;
  r /= g.np[0];
  const int j = r % g.np[1] - NG;
  const int k = (g.dim == 3) ? r / g.np[1] - NG : 0;
  const bool upd = in_range(g, 0, i, kYee[c][0] != 0.0) && in_range(g, 1, j, kYee[c][1] != 0.0) &&
                   in_range(g, 2, k, kYee[c][2] != 0.0);
  if (!upd) {
    out[q] = in[q];
    return;
  }
  if (c == 2 && axis_node(g, j)) {
    out[q] = (Real)0;
    return;
  }
  const int D = g.dim;
  const int kr = (D == 3) ? 1 : 0;
  double acc = 0.0;
  for (int dk = -kr; dk <= kr; ++dk)
    for (int dj = -1; dj <= 1; ++dj)
      for (int di = -1; di <= 1; ++di) {
        const int e = D + abs(di) + abs(dj) + abs(dk);
        acc += ldexp(1.0, -e) * j_filter_at(g, in, c, i + di, j + dj, k + dk);
      }
  out[q] = (Real)acc;
}

unsigned field_blocks(const GridConst &g) {
  const int64_t e0 = g.n[0] + (g.geom != 0 ? 1 : 0);
  const int64_t e1 = g.n[1] + (g.geom != 0 ? 1 : 0);
  const int64_t e2 = (g.dim == 3) ? g.n[2] : 1;
  return (unsigned)((e0 * e1 * e2 + FT - 1) / FT);
}

template <class Real>
hipError_t launch_faraday(const GridConst &g, Real *EB, double f, hipStream_t s) {
  hipLaunchKernelGGL(k_faraday<Real>, dim3(field_blocks(g)), dim3(FT), 0, s, g, EB, f);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_fill_ghosts<Real>(g, EB + 3 * g.npts, 3, s);
  return e;
}

template <class Real>
hipError_t launch_ampere(const GridConst &g, Real *EB, const Real *J, double dt, double coupling,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_ampere<Real>, dim3(field_blocks(g)), dim3(FT), 0, s, g, EB, J, dt,
                     coupling);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_fill_ghosts<Real>(g, EB, 3, s);
  return e;
}

template <class Real>
hipError_t launch_filter(const GridConst &g, const Real *in, Real *out, hipStream_t s) {
  const unsigned nb = (unsigned)((3 * g.npts + FT - 1) / FT);
  hipLaunchKernelGGL(k_filter<Real>, dim3(nb), dim3(FT), 0, s, g, in, out);
  return hipGetLastError();
}

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
