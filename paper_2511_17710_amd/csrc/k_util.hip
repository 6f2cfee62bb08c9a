// k_util.hip -- periodic ghost fill of the fields, periodic fold of the
// current ghosts into their images, and zeroing.
#include "step_device.h"

namespace picstep {

constexpr int UT = 256;

__device__ __forceinline__ void unpad(const GridConst &g, int64_t q, int ii[3]) {
  ii[0] = (int)(q % g.np[0]) - NG;
  const int64_t r = q / g.np[0];
  ii[1] = (int)(r % g.np[1]) - NG;
  ii[2] = (g.dim == 3) ? (int)(r / g.np[1]) - NG : 0;
}

// copy the periodic image into every ghost point of dimension dd
template <class Real>
__global__ __launch_bounds__(UT) void k_fill_ghosts(GridConst g, Real *A, int ncomp, int dd) {
  const int64_t q = (int64_t)blockIdx.x * UT + threadIdx.x;
  if (q >= g.npts * ncomp) return;
  const int64_t c = q / g.npts, pt = q % g.npts;
  int ii[3];
  unpad(g, pt, ii);
  const int v = ii[dd];
  if (v >= 0 && v < g.n[dd]) return;
  int s = v % g.n[dd];
  if (s < 0) s += g.n[dd];
  ii[dd] = s;
  A[q] = A[c * g.npts + (int64_t)pad_index(g, ii[0], ii[1], ii[2], g.dim)];
}

// add every ghost point of dimension dd into its periodic image, zero the ghost
template <class Real>
__global__ __launch_bounds__(UT) void k_fold_ghosts(GridConst g, Real *A, int ncomp, int dd) {
  const int64_t q = (int64_t)blockIdx.x * UT + threadIdx.x;
  if (q >= g.npts * ncomp) return;
  const int64_t c = q / g.npts, pt = q % g.npts;
  int ii[3];
  unpad(g, pt, ii);
  const int v = ii[dd];
  if (v >= 0 && v < g.n[dd]) return;
  const Real x = A[q];
  A[q] = (Real)0;
  if (x == (Real)0) return;
  int s = v % g.n[dd];
  if (s < 0) s += g.n[dd];
  ii[dd] = s;
  atomic_add_r(A + c * g.npts + (int64_t)pad_index(g, ii[0], ii[1], ii[2], g.dim), x);
}

template <class Real>
__global__ __launch_bounds__(UT) void k_zero(Real *A, int64_t n) {
  const int64_t q = (int64_t)blockIdx.x * UT + threadIdx.x;
  if (q < n) A[q] = (Real)0;
}

template <class Real>
hipError_t launch_fill_ghosts(const GridConst &g, Real *A, int ncomp, hipStream_t s) {
  if (g.geom != 0) return hipSuccess;
  const int64_t tot = g.npts * ncomp;
  const unsigned nb = (unsigned)((tot + UT - 1) / UT);
  for (int dd = 0; dd < g.dim; ++dd)
    hipLaunchKernelGGL((k_fill_ghosts<Real>), dim3(nb), dim3(UT), 0, s, g, A, ncomp, dd);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_fold_ghosts(const GridConst &g, Real *A, int ncomp, hipStream_t s) {
  if (g.geom != 0) return hipSuccess;
  const int64_t tot = g.npts * ncomp;
  const unsigned nb = (unsigned)((tot + UT - 1) / UT);
  for (int dd = g.dim - 1; dd >= 0; --dd)
    hipLaunchKernelGGL((k_fold_ghosts<Real>), dim3(nb), dim3(UT), 0, s, g, A, ncomp, dd);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_zero(Real *A, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_zero<Real>), dim3((unsigned)((n + UT - 1) / UT)), dim3(UT), 0, s, A, n);
  return hipGetLastError();
}

template hipError_t launch_fill_ghosts<float>(const GridConst &, float *, int, hipStream_t);
template hipError_t launch_fill_ghosts<double>(const GridConst &, double *, int, hipStream_t);
template hipError_t launch_fold_ghosts<float>(const GridConst &, float *, int, hipStream_t);
template hipError_t launch_fold_ghosts<double>(const GridConst &, double *, int, hipStream_t);
template hipError_t launch_zero<float>(float *, int64_t, hipStream_t);
template hipError_t launch_zero<double>(double *, int64_t, hipStream_t);

}  // namespace picstep
