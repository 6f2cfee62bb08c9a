// k_util.hip -- periodic ghost fill of the fields, periodic fold of the
// current ghosts into their images, and zeroing.
#include "step_device.h"

namespace picstep {

constexpr int UT = 256;

// Ghost slab of dimension dd: its 2*NG ghost layers times the padded extent
// of the other dimensions.  Thread q of ncomp * slab_points(g, dd) maps to
// component c and unpadded coordinates ii (ii[dd] in [-NG, 0) or [n, n + NG)).
__device__ __forceinline__ int slab_points(const GridConst &g, int dd) {
  int e = 2 * NG;
  for (int d = 0; d < g.dim; ++d)
    if (d != dd) e *= g.np[d];
  return e;
}
__device__ __forceinline__ void slab_point(const GridConst &g, int dd, int r, int ii[3]) {
  int ext[3] = {g.np[0], g.np[1], (g.dim == 3) ? g.np[2] : 1};
  ext[dd] = 2 * NG;
  ii[0] = r % ext[0] - NG;
  r /= ext[0];
  ii[1] = r % ext[1] - NG;
  ii[2] = (g.dim == 3) ? r / ext[1] - NG : 0;
  if (ii[dd] >= 0) ii[dd] += g.n[dd];  // the high layers
}

// copy the periodic image into every ghost point of dimension dd
template <class Real>
__global__ __launch_bounds__(UT) void k_fill_ghosts(GridConst g, Real *A, int ncomp, int dd) {
  const int per = slab_points(g, dd);
  const int q = blockIdx.x * UT + threadIdx.x;
  if (q >= per * ncomp) return;
  const int c = q / per;
  int ii[3];
  slab_point(g, dd, q - c * per, ii);
  const int64_t at = c * g.npts + (int64_t)pad_index(g, ii[0], ii[1], ii[2], g.dim);
  int s = ii[dd] % g.n[dd];
  if (s < 0) s += g.n[dd];
  ii[dd] = s;
  A[at] = A[c * g.npts + (int64_t)pad_index(g, ii[0], ii[1], ii[2], g.dim)];
}

// add every ghost point into its periodic image (wrapped in every
// dimension at once), zero the ghost.  One launch: thread q walks the ghost
// slabs of the dimensions in turn and takes each point in the slab of its
// lowest ghost dimension only, so every ghost point is visited once; the
// images are active points, which no thread reads.
template <class Real>
__global__ __launch_bounds__(UT) void k_fold_ghosts(GridConst g, Real *A, int ncomp) {
  int q = blockIdx.x * UT + threadIdx.x;
  int dd = 0, per = slab_points(g, 0);
  while (q >= per * ncomp) {  // at most DIM iterations
    q -= per * ncomp;
    if (++dd >= g.dim) return;
    per = slab_points(g, dd);
  }
  const int c = q / per;
  int ii[3];
  slab_point(g, dd, q - c * per, ii);
  for (int d = 0; d < dd; ++d)
    if (ii[d] < 0 || ii[d] >= g.n[d]) return;  // taken in the slab of dimension d
  const int64_t at = c * g.npts + (int64_t)pad_index(g, ii[0], ii[1], ii[2], g.dim);
  const Real x = A[at];
  A[at] = (Real)0;
  if (x == (Real)0) return;
  for (int d = 0; d < g.dim; ++d) {
    int s = ii[d] % g.n[d];
    if (s < 0) s += g.n[d];
    ii[d] = s;
  }
  atomic_add_r(A + c * g.npts + (int64_t)pad_index(g, ii[0], ii[1], ii[2], g.dim), x);
}

template <class Real>
__global__ __launch_bounds__(UT) void k_zero(Real *A, int64_t n) {
  const int64_t q = (int64_t)blockIdx.x * UT + threadIdx.x;
  if (q < n) A[q] = (Real)0;
}

// blocks for the ghost slab of dimension dd (host side of slab_points)
unsigned slab_blocks(const GridConst &g, int dd, int ncomp) {
  int64_t e = 2 * NG;
  for (int d = 0; d < g.dim; ++d)
    if (d != dd) e *= g.np[d];
  return (unsigned)((e * ncomp + UT - 1) / UT);
}

template <class Real>
hipError_t launch_fill_ghosts(const GridConst &g, Real *A, int ncomp, hipStream_t s) {
  if (g.geom != 0) return hipSuccess;
  for (int dd = 0; dd < g.dim; ++dd)
    hipLaunchKernelGGL((k_fill_ghosts<Real>), dim3(slab_blocks(g, dd, ncomp)), dim3(UT), 0, s, g,
                       A, ncomp, dd);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_fold_ghosts(const GridConst &g, Real *A, int ncomp, hipStream_t s) {
  if (g.geom != 0) return hipSuccess;
  int64_t threads = 0;  // all ghost slabs, one after the other
  for (int dd = 0; dd < g.dim; ++dd) threads += (int64_t)slab_blocks(g, dd, ncomp) * UT;
  hipLaunchKernelGGL((k_fold_ghosts<Real>), dim3((unsigned)((threads + UT - 1) / UT)), dim3(UT), 0,
                     s, g, A, ncomp);
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
template hipError_t launch_zero<int32_t>(int32_t *, int64_t, hipStream_t);

}  // namespace picstep
