// k_sort.hip -- stable per-cell counting sort of a particle species.
//
// Least-significant-digit radix sort on a cell key that orders cells brick by
// brick (8-bit digits; dead particles carry the largest key; the first pass
// forms the keys from the cells), so equal keys keep their previous order and
// the permutation is unique.  Per pass: tile histograms (one row of 256
// counts per tile), an exclusive scan of the matrix in digit-major order (the
// start of every digit of every tile), and a stable in-tile ranking with
// wave ballots followed by a scatter.  A gather then reorders every SoA array into
// the second particle set.
#include "step_device.h"

namespace picstep {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = SORT_TILE / SORT_THREADS;  // 16 keys per thread
constexpr int RADIX = 256;

// block-wide exclusive scan of one int per thread (256 threads, wave64)
__device__ __forceinline__ int block_exclusive_scan(int v, int *total, int *sh_warp) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh_warp[wid] = x;
  __syncthreads();
  int pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < SORT_THREADS / 64; ++w) {
    const int t = sh_warp[w];
    if (w < wid) pre += t;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return pre + x - v;
}

// The first radix pass reads the cells and forms key and index on the fly
// (cells != nullptr); later passes read the previous pass's keys and values.
struct KeySource {
  const uint32_t *keys;
  const int32_t *vals;
  const int32_t *cells;
  GridConst g;
  uint32_t deadkey;
  __device__ __forceinline__ uint32_t key(int64_t i) const {
    return cells ? brick_key(g, cells[i], deadkey) : keys[i];
  }
  __device__ __forceinline__ int32_t val(int64_t i) const {
    return cells ? (int32_t)i : vals[i];
  }
};

__global__ __launch_bounds__(SORT_THREADS) void k_radix_hist(KeySource src, int64_t n, int shift,
                                                             int32_t *__restrict__ hist,
                                                             int64_t ntiles) {
  __shared__ int h[RADIX];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * SORT_TILE;
#pragma unroll
  for (int j = 0; j < SORT_ITEMS; ++j) {
    const int64_t i = t0 + (int64_t)j * SORT_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(src.key(i) >> shift) & (RADIX - 1)], 1);
  }
  __syncthreads();
  hist[(int64_t)blockIdx.x * RADIX + threadIdx.x] = h[threadIdx.x];  // one 1 KB row
}

// Exclusive scan of the tile-major histogram matrix H[tile][digit] in
// digit-major order: H[t][d] becomes the number of keys with a smaller digit
// plus those with digit d in earlier tiles.  Thread = digit throughout, so
// every access is a coalesced row.  (1) column sums of chunks of ct tiles,
// (2) one block scans those sums down the chunks and across the digits,
// (3) each chunk rescans its rows from its chunk start.
__global__ __launch_bounds__(RADIX) void k_col_sums(const int32_t *__restrict__ H, int64_t ntiles,
                                                    int64_t ct, int32_t *__restrict__ S) {
  const int64_t t0 = (int64_t)blockIdx.x * ct, t1 = min(t0 + ct, ntiles);
  int sum = 0;
#pragma unroll 16
  for (int64_t t = t0; t < t1; ++t) sum += H[t * RADIX + threadIdx.x];
  S[(int64_t)blockIdx.x * RADIX + threadIdx.x] = sum;
}

__global__ __launch_bounds__(RADIX) void k_col_scan(int32_t *__restrict__ S, int nchunks) {
  __shared__ int sw[RADIX / 64];
  int v[SCAN_CHUNKS];  // the whole column in registers: loads issued together
#pragma unroll
  for (int c = 0; c < SCAN_CHUNKS; ++c) v[c] = (c < nchunks) ? S[c * RADIX + threadIdx.x] : 0;
  int run = 0;
#pragma unroll
  for (int c = 0; c < SCAN_CHUNKS; ++c) {
    const int x = v[c];
    v[c] = run;
    run += x;
  }
  int all;
  const int base = block_exclusive_scan(run, &all, sw);  // keys with a smaller digit
#pragma unroll
  for (int c = 0; c < SCAN_CHUNKS; ++c)
    if (c < nchunks) S[c * RADIX + threadIdx.x] = v[c] + base;
}

__global__ __launch_bounds__(RADIX) void k_col_apply(int32_t *__restrict__ H, int64_t ntiles,
                                                     int64_t ct, const int32_t *__restrict__ S) {
  const int64_t t0 = (int64_t)blockIdx.x * ct, t1 = min(t0 + ct, ntiles);
  int run = S[(int64_t)blockIdx.x * RADIX + threadIdx.x];
#pragma unroll 16
  for (int64_t t = t0; t < t1; ++t) {
    const int v = H[t * RADIX + threadIdx.x];
    H[t * RADIX + threadIdx.x] = run;
    run += v;
  }
}

// Stable scatter of one tile.  Wave w ranks the keys [w*1024, (w+1)*1024) of
// the tile in 16 rounds of 64 consecutive keys: eight ballots find the lanes
// holding the same digit, a lane's rank is the count of those peers below it
// plus the wave's running count of the digit (a wave-private LDS counter
// advanced by the lowest peer).  Rounds run in key order and waves are
// ordered by their per-digit prefix, so equal digits keep their order.  Then
// either (STAGE) the tile is staged in digit order in LDS and written with
// consecutive threads on consecutive destinations -- the first pass, whose
// low digit is spread over many short runs after the particles have drifted
// -- or each key goes straight from registers to its slot: lanes of a round
// holding the same digit write consecutive addresses, and the higher digits
// of nearly sorted keys come in long runs.
template <bool STAGE>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(
    KeySource src, uint32_t *__restrict__ kout, int32_t *__restrict__ vout, int64_t n, int shift,
    const int32_t *__restrict__ hist, int64_t ntiles) {
  constexpr int NW = SORT_THREADS / 64;
  constexpr int PER_WAVE = SORT_TILE / NW;
  constexpr int ROUNDS = PER_WAVE / 64;
  __shared__ int cnt[NW][RADIX];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int64_t t0 = (int64_t)blockIdx.x * SORT_TILE;
  const int nvalid = (int)min((int64_t)SORT_TILE, n - t0);
#pragma unroll
  for (int ww = 0; ww < NW; ++ww) cnt[ww][threadIdx.x] = 0;
  const int goff = hist[(int64_t)blockIdx.x * RADIX + threadIdx.x];
  __syncthreads();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t k[ROUNDS];
  int32_t v[ROUNDS];
  int rk[ROUNDS];
#pragma unroll
  for (int j = 0; j < ROUNDS; ++j) {
    const int e = w * PER_WAVE + j * 64 + lane;
    const bool ok = e < nvalid;
    k[j] = ok ? src.key(t0 + e) : 0u;
    v[j] = ok ? src.val(t0 + e) : -1;
  }
#pragma unroll
  for (int j = 0; j < ROUNDS; ++j) {
    const int e = w * PER_WAVE + j * 64 + lane;
    const bool ok = e < nvalid;
    const uint32_t dg = (k[j] >> shift) & (RADIX - 1);
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool set = (dg >> b) & 1u;
      const uint64_t bb = __ballot(set);
      peers &= set ? bb : ~bb;
    }
    const int r = __popcll(peers & below);
    int base = 0;
    if (ok) base = cnt[w][dg];
    rk[j] = base + r;
    if (ok && r == 0) cnt[w][dg] = base + __popcll(peers);
  }
  __syncthreads();
  if constexpr (STAGE) {
    __shared__ uint32_t sk[SORT_TILE];
    __shared__ int32_t sv[SORT_TILE];
    __shared__ int dstart[RADIX];
    __shared__ int sw[NW];
    {  // per digit (one per thread): tile start and the waves' prefixes
      const int d = threadIdx.x;
      int c[NW], tot = 0;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) {
        c[ww] = cnt[ww][d];
        tot += c[ww];
      }
      int all;
      const int st = block_exclusive_scan(tot, &all, sw);
      dstart[d] = st;
      int run = st;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) {
        cnt[ww][d] = run;
        run += c[ww];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ROUNDS; ++j) {
      const int e = w * PER_WAVE + j * 64 + lane;
      if (e < nvalid) {
        const int lp = cnt[w][(k[j] >> shift) & (RADIX - 1)] + rk[j];
        sk[lp] = k[j];
        sv[lp] = v[j];
      }
    }
    __syncthreads();
    cnt[0][threadIdx.x] = goff;  // the digit's start of the tile in the global order
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; ++j) {
      const int e = j * SORT_THREADS + threadIdx.x;
      if (e < nvalid) {
        const uint32_t key = sk[e];
        const uint32_t dg = (key >> shift) & (RADIX - 1);
        const int64_t dst = (int64_t)cnt[0][dg] + (e - dstart[dg]);
        if (kout) kout[dst] = key;  // the last pass keeps only the permutation
        vout[dst] = sv[e];
      }
    }
  } else {
    {  // per digit (one per thread): global start of each wave's keys of the digit
      const int d = threadIdx.x;
      int run = goff;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) {
        const int c = cnt[ww][d];
        cnt[ww][d] = run;
        run += c;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ROUNDS; ++j) {
      const int e = w * PER_WAVE + j * 64 + lane;
      if (e < nvalid) {
        const uint32_t dg = (k[j] >> shift) & (RADIX - 1);
        const int64_t dst = (int64_t)cnt[w][dg] + rk[j];
        if (kout) kout[dst] = k[j];  // the last pass keeps only the permutation
        vout[dst] = v[j];
      }
    }
  }
}

hipError_t launch_sort_species(const GridConst &g, const int32_t *cell, int64_t n,
                               const SortScratch &S, int32_t *perm_out, int keybits,
                               hipStream_t s, const uint32_t **keys_out) {
  if (n <= 0) return hipSuccess;
  const int64_t ntiles = (n + SORT_TILE - 1) / SORT_TILE;
  if (ntiles > S.max_tiles) return hipErrorInvalidValue;
  const int64_t ct = (ntiles + SCAN_CHUNKS - 1) / SCAN_CHUNKS;  // tiles per chunk
  const int64_t nchunks = (ntiles + ct - 1) / ct;                // <= SCAN_CHUNKS
  const uint32_t deadkey = 1u << (keybits - 1);
  const int passes = (keybits + 7) / 8;
  for (int ps = 0; ps < passes; ++ps) {
    const int shift = 8 * ps;
    const int src = ps & 1, dst = src ^ 1;
    KeySource ks{S.keys[src], S.vals[src], ps == 0 ? cell : nullptr, g, deadkey};
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(SORT_THREADS), 0, s, ks, n,
                       shift, S.hist, ntiles);
    hipLaunchKernelGGL(k_col_sums, dim3((unsigned)nchunks), dim3(RADIX), 0, s, S.hist, ntiles, ct,
                       S.bsum);
    hipLaunchKernelGGL(k_col_scan, dim3(1), dim3(RADIX), 0, s, S.bsum, (int)nchunks);
    hipLaunchKernelGGL(k_col_apply, dim3((unsigned)nchunks), dim3(RADIX), 0, s, S.hist, ntiles,
                       ct, S.bsum);
    int32_t *vdst = (ps == passes - 1) ? perm_out : S.vals[dst];
    // the last pass keeps the keys only when the caller wants them
    uint32_t *kdst = (ps == passes - 1 && !keys_out) ? nullptr : S.keys[dst];
    if (ps == passes - 1 && keys_out) *keys_out = S.keys[dst];
    if (ps == 0)
      hipLaunchKernelGGL(k_radix_scatter<true>, dim3((unsigned)ntiles), dim3(SORT_THREADS), 0, s,
                         ks, kdst, vdst, n, shift, S.hist, ntiles);
    else
      hipLaunchKernelGGL(k_radix_scatter<false>, dim3((unsigned)ntiles), dim3(SORT_THREADS), 0, s,
                         ks, kdst, vdst, n, shift, S.hist, ntiles);
  }
  return hipGetLastError();
}

// Brick starts of sorted keys: index i opens every bin in (bin(i-1), bin(i)]
// (bin = brick, or nb for the dead); i = n closes the rest.
__global__ __launch_bounds__(SORT_THREADS) void k_brick_bounds(const uint32_t *__restrict__ keys,
                                                               int64_t n, int nb, int localbits,
                                                               uint32_t deadkey,
                                                               int32_t *__restrict__ bstart) {
  const int64_t i = (int64_t)blockIdx.x * SORT_THREADS + threadIdx.x;
  if (i > n) return;
  auto bin = [&](int64_t j) {
    const uint32_t k = keys[j];
    return k == deadkey ? nb : (int)(k >> localbits);
  };
  const int lo = (i == 0) ? -1 : bin(i - 1);
  const int hi = (i == n) ? nb + 1 : bin(i);
  for (int b = lo + 1; b <= hi; ++b) bstart[b] = (int32_t)i;
}

hipError_t launch_brick_bounds(const uint32_t *keys, int64_t n, int nb, int localbits,
                               uint32_t deadkey, int32_t *bstart, hipStream_t s) {
  hipLaunchKernelGGL(k_brick_bounds, dim3((unsigned)(n / SORT_THREADS + 1)), dim3(SORT_THREADS), 0,
                     s, keys, n, nb, localbits, deadkey, bstart);
  return hipGetLastError();
}

// reorder every SoA array of one species range: dst[off+i] = src[off+perm[i]].
// Four elements per thread, strided by the block size (coalesced stores),
// with all loads of an array issued before its stores.
constexpr int GATHER_PER_THREAD = 4;

template <class T>
__device__ __forceinline__ void gather_array(const T *__restrict__ src, T *__restrict__ dst,
                                             int64_t off, const int64_t i[GATHER_PER_THREAD],
                                             const int32_t pj[GATHER_PER_THREAD]) {
  T v[GATHER_PER_THREAD];
#pragma unroll
  for (int k = 0; k < GATHER_PER_THREAD; ++k)
    if (pj[k] >= 0) v[k] = src[off + pj[k]];
#pragma unroll
  for (int k = 0; k < GATHER_PER_THREAD; ++k)
    if (pj[k] >= 0) dst[off + i[k]] = v[k];
}

template <class Real>
__global__ __launch_bounds__(SORT_THREADS) void k_gather(PSet<Real> src, PSet<Real> dst, int dim,
                                                         int has_phi, int64_t off, int64_t n,
                                                         const int32_t *__restrict__ perm) {
  int64_t i[GATHER_PER_THREAD];
  int32_t pj[GATHER_PER_THREAD];
#pragma unroll
  for (int k = 0; k < GATHER_PER_THREAD; ++k) {
    i[k] = ((int64_t)blockIdx.x * GATHER_PER_THREAD + k) * SORT_THREADS + threadIdx.x;
    pj[k] = (i[k] < n) ? perm[i[k]] : -1;
    if (pj[k] >= n) pj[k] = -1;  // never read outside the species range
  }
  gather_array(src.cell, dst.cell, off, i, pj);
  for (int a = 0; a < dim; ++a) gather_array(src.offs[a], dst.offs[a], off, i, pj);
#pragma unroll
  for (int a = 0; a < 3; ++a) gather_array(src.u[a], dst.u[a], off, i, pj);
  gather_array(src.w, dst.w, off, i, pj);
  if (has_phi) gather_array(src.phi, dst.phi, off, i, pj);
  gather_array(src.id, dst.id, off, i, pj);
}

template <class Real>
hipError_t launch_gather(const PSet<Real> &src, const PSet<Real> &dst, int dim, int has_phi,
                         int64_t off, int64_t n, const int32_t *perm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t per = (int64_t)SORT_THREADS * GATHER_PER_THREAD;
  hipLaunchKernelGGL((k_gather<Real>), dim3((unsigned)((n + per - 1) / per)), dim3(SORT_THREADS),
                     0, s, src, dst, dim, has_phi, off, n, perm);
  return hipGetLastError();
}

// inverse of the gather for one array: dst[off+perm[i]] = src[off+i]
template <class Real>
__global__ __launch_bounds__(SORT_THREADS) void k_scatter_back(const Real *__restrict__ src,
                                                               Real *__restrict__ dst, int64_t off,
                                                               int64_t n,
                                                               const int32_t *__restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * SORT_THREADS + threadIdx.x;
  if (i >= n) return;
  const int32_t pi = perm[i];
  if (pi < 0 || pi >= n) return;
  dst[off + pi] = src[off + i];
}

template <class Real>
hipError_t launch_scatter_back(const Real *src, Real *dst, int64_t off, int64_t n,
                               const int32_t *perm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_scatter_back<Real>),
                     dim3((unsigned)((n + SORT_THREADS - 1) / SORT_THREADS)), dim3(SORT_THREADS),
                     0, s, src, dst, off, n, perm);
  return hipGetLastError();
}

template hipError_t launch_gather<float>(const PSet<float> &, const PSet<float> &, int, int,
                                         int64_t, int64_t, const int32_t *, hipStream_t);
template hipError_t launch_gather<double>(const PSet<double> &, const PSet<double> &, int, int,
                                          int64_t, int64_t, const int32_t *, hipStream_t);
template hipError_t launch_scatter_back<float>(const float *, float *, int64_t, int64_t,
                                               const int32_t *, hipStream_t);
template hipError_t launch_scatter_back<double>(const double *, double *, int64_t, int64_t,
                                                const int32_t *, hipStream_t);

}  // namespace picstep
