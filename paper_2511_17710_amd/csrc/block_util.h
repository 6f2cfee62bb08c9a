// block_util.h -- workgroup-level helpers shared by the particle kernels:
// XCD-aware block order and block-wide reductions (256 threads, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace picstep {

// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD
// b mod 8), and each XCD has its own L2.  Block b = 8k + x is given the k-th
// chunk of XCD x's contiguous share of the chunk sequence, so that one XCD
// works through neighbouring chunks (neighbouring cells after the sort) and
// its L2 holds the fields and current around them.
constexpr int NXCD = 8;
__device__ __forceinline__ int64_t xcd_chunk(int64_t b, int64_t nblk) {
  const int64_t q = nblk / NXCD, r = nblk % NXCD;
  const int64_t x = b % NXCD, k = b / NXCD;
  return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Segments of seg consecutive chunks dealt to the XCDs round robin: XCD x
// takes segments x, x + 8, x + 16, ... in turn (blocks b = 8k + x, k-th
// block of XCD x), so the XCDs together sweep the chunks in order while each
// L2 serves runs of seg neighbouring chunks; the blocks past the last whole
// round of 8 segments keep the plain order (a bijection on [0, nblk)).
__device__ __forceinline__ int64_t xcd_segment_chunk(int64_t b, int64_t nblk, int64_t seg) {
  const int64_t whole = nblk / (NXCD * seg) * (NXCD * seg);
  if (b >= whole) return b;
  const int64_t x = b % NXCD, k = b / NXCD;
  return ((k / seg) * NXCD + x) * seg + k % seg;
}

// largest s with s^dim <= vals
constexpr int tile_side(int vals, int dim) {
  int s = 1;
  while (true) {
    int p = 1;
    for (int d = 0; d < dim; ++d) p *= s + 1;
    if (p > vals) return s;
    ++s;
  }
}
static_assert(tile_side(1331, 3) == 11 && tile_side(1330, 3) == 10 && tile_side(1365, 2) == 36,
              "tile_side");

// v mod n in [0, n): tile coordinates lie within one period of the active
// range except on tiny grids, which take the general remainder
__device__ __forceinline__ int wrap_periodic(int v, int n) {
  v += (v < 0) ? n : 0;
  v -= (v >= n) ? n : 0;
  if ((unsigned)v >= (unsigned)n) v = ((v % n) + n) % n;
  return v;
}

// block-wide min/max of three ints (256 threads); the results, equal in every
// lane, are made wave-uniform so that they and what derives from them live
// in scalar registers (the reverse-step kernel's spills 60 -> 47 VGPRs,
// 0.367 -> 0.347 ms per step on the 64^3 workload)
__device__ __forceinline__ void block_minmax3(int lo[3], int hi[3], int *red) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      lo[d] = min(lo[d], __shfl_xor(lo[d], o, 64));
      hi[d] = max(hi[d], __shfl_xor(hi[d], o, 64));
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      red[w * 6 + d] = lo[d];
      red[w * 6 + 3 + d] = hi[d];
    }
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = red[d];
    hi[d] = red[3 + d];
#pragma unroll
    for (int ww = 1; ww < BLOCK / 64; ++ww) {
      lo[d] = min(lo[d], red[ww * 6 + d]);
      hi[d] = max(hi[d], red[ww * 6 + 3 + d]);
    }
    lo[d] = __builtin_amdgcn_readfirstlane(lo[d]);
    hi[d] = __builtin_amdgcn_readfirstlane(hi[d]);
  }
}

// block-wide maximum of a non-negative float (its bit pattern orders like
// the value)
__device__ __forceinline__ float block_max_nonneg(float v, int *red) {
  __syncthreads();  // earlier reductions may still be reading red
  int x = __float_as_int(v);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  x = red[0];
#pragma unroll
  for (int ww = 1; ww < BLOCK / 64; ++ww) x = max(x, red[ww]);
  return __int_as_float(__builtin_amdgcn_readfirstlane(x));
}

// q = x / d for 0 <= x < 2^23 with a float reciprocal and one correction
__device__ __forceinline__ int div_small(int x, int d, float inv) {
  int q = (int)((float)x * inv);
  if (q * d > x) --q;
  else if ((q + 1) * d <= x) ++q;
  return q;
}

// Visits every element x = comp*T + ix + s0*iy + s0*s1*iz (T = s0 s1 s2) of
// an ncomp-component tile, spread over the block.  Each thread owns one point
// of the plane of the first pdims axes (the x row in 2D, the (x, y) plane in
// 3D) and walks the last axis (w: y in 2D, z in 3D) and the components, so
// elements need no division; per thread ps = plane(ix, iy) is formed once
// (iy = 0 in 2D).  Elements go in batches of NB per thread: v = get(ps, x,
// comp, w) for the whole batch first (so that NB global loads are in flight
// together instead of one waiting after another), then put(ps, x, comp, w,
// v).  A plane wider than the block falls back to an element loop with
// divisions.
template <int NB, class V, class Plane, class Get, class Put>
__device__ __forceinline__ void tile_for_each(int ncomp, int pdims, int s0, int s1, int s2,
                                              Plane plane, Get get, Put put) {
  const int T = s0 * s1 * s2;
  const int P = (pdims == 2) ? s0 * s1 : s0;
  const int L = (pdims == 2) ? s2 : s1;
  if (P <= BLOCK) {
    const int G = BLOCK / P;
    const int grp = div_small((int)threadIdx.x, P, 1.0f / (float)P);
    if (grp >= G) return;
    const int pt = (int)threadIdx.x - grp * P;
    const int iy0 = div_small(pt, s0, 1.0f / (float)s0);
    const int ix = pt - iy0 * s0;
    const auto ps = plane(ix, pdims == 2 ? iy0 : 0);
    // elements per component of this thread: w = grp, grp + G, ... < L
    const int nw = (L > grp) ? div_small(L - grp + G - 1, G, 1.0f / (float)G) : 0;
    const int n = ncomp * nw;
    int comp = 0, w = grp;
    for (int k = 0; k < n; k += NB) {
      V v[NB];
      int c1 = comp, w1 = w;  // the put phase replays the walk from here
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (k + j < n) {
          v[j] = get(ps, comp * T + pt + P * w, comp, w);
          w += G;
          if (w >= L) {
            w = grp;
            ++comp;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (k + j < n) {
          put(ps, c1 * T + pt + P * w1, c1, w1, v[j]);
          w1 += G;
          if (w1 >= L) {
            w1 = grp;
            ++c1;
          }
        }
      }
    }
  } else {
    const float iT = 1.0f / (float)T, i0f = 1.0f / (float)s0, i01 = 1.0f / (float)(s0 * s1);
    for (int x = threadIdx.x; x < ncomp * T; x += BLOCK) {
      const int comp = div_small(x, T, iT);
      int rem = x - comp * T;
      const int iz = div_small(rem, s0 * s1, i01);
      rem -= iz * s0 * s1;
      const int iy = div_small(rem, s0, i0f);
      const auto ps = plane(rem - iy * s0, pdims == 2 ? iy : 0);
      const int w = (pdims == 2) ? iz : iy;
      put(ps, x, comp, w, get(ps, x, comp, w));
    }
  }
}

// tile_for_each for a tile that maps affinely onto a global array: element
// (comp, plane point, w) sits at g = plane(ix, iy) + comp*cstride + w*wstride
// there.  x and g advance by additions only, so an element costs a few
// instructions: v = get(g, x) for a batch of NB, then put(g, x, v).  Same
// walk and the same element loop fallback as tile_for_each.
template <int NB, class V, class Plane, class Get, class Put>
__device__ __forceinline__ void tile_for_each_affine(int ncomp, int pdims, int s0, int s1, int s2,
                                                     int cstride, int wstride, Plane plane,
                                                     Get get, Put put) {
  const int T = s0 * s1 * s2;
  const int P = (pdims == 2) ? s0 * s1 : s0;
  const int L = (pdims == 2) ? s2 : s1;
  if (P <= BLOCK) {
    const int G = BLOCK / P;
    const int grp = div_small((int)threadIdx.x, P, 1.0f / (float)P);
    if (grp >= G) return;
    const int pt = (int)threadIdx.x - grp * P;
    const int iy0 = div_small(pt, s0, 1.0f / (float)s0);
    const int ix = pt - iy0 * s0;
    const int nw = (L > grp) ? div_small(L - grp + G - 1, G, 1.0f / (float)G) : 0;
    const int n = ncomp * nw;
    // steps along the walk and from the last w of a component to the first
    // of the next
    const int dx = P * G, dg = wstride * G;
    const int dxc = T - dx * (nw - 1), dgc = cstride - dg * (nw - 1);
    // unsigned: the offset one step past the last element may exceed 2^31
    unsigned x = pt + P * grp;
    unsigned gi = plane(ix, pdims == 2 ? iy0 : 0) + wstride * grp;
    int cw = 0;  // position along the walk within the component
    for (int k = 0; k < n; k += NB) {
      V v[NB];
      unsigned x1 = x, g1 = gi;  // the put phase replays the walk from here
      int c1 = cw;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (k + j < n) {
          v[j] = get((int)gi, (int)x);
          const bool last = ++cw == nw;
          x += last ? dxc : dx;
          gi += last ? dgc : dg;
          cw = last ? 0 : cw;
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (k + j < n) {
          put((int)g1, (int)x1, v[j]);
          const bool last = ++c1 == nw;
          x1 += last ? dxc : dx;
          g1 += last ? dgc : dg;
          c1 = last ? 0 : c1;
        }
      }
    }
  } else {
    const float iT = 1.0f / (float)T, i0f = 1.0f / (float)s0, i01 = 1.0f / (float)(s0 * s1);
    for (int x = threadIdx.x; x < ncomp * T; x += BLOCK) {
      const int comp = div_small(x, T, iT);
      int rem = x - comp * T;
      const int iz = div_small(rem, s0 * s1, i01);
      rem -= iz * s0 * s1;
      const int iy = div_small(rem, s0, i0f);
      const int w = (pdims == 2) ? iz : iy;
      const int gi = plane(rem - iy * s0, pdims == 2 ? iy : 0) + comp * cstride + w * wstride;
      put(gi, x, get(gi, x));
    }
  }
}

// a thread's point of a tile plane: its padded-lattice offset and whether it
// lies on the lattice
struct PlanePt {
  int off;
  bool ok;
};

// block-wide sum of three ints (256 threads), wave-uniform results
__device__ __forceinline__ void block_sum3(int v[3], int *red) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v[d] += __shfl_xor(v[d], o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) red[w * 6 + d] = v[d];
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    v[d] = 0;
#pragma unroll
    for (int ww = 0; ww < BLOCK / 64; ++ww) v[d] += red[ww * 6 + d];
    v[d] = __builtin_amdgcn_readfirstlane(v[d]);
  }
}

}  // namespace picstep
