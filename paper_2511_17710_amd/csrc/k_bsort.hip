// k_bsort.hip -- the per-cell sort of a species whose particles are still in
// the order of the previous sort and have since moved by at most one brick
// in every dimension (the usual case: a particle crosses at most one cell per
// step and dimension, and sorts come every few steps).
//
// The particles of a new brick then come from the old ranges of its 3^D
// neighbour bricks, and in the stable order (ties keep the previous order)
// they arrive source by source, in the order of the old bricks.  So instead
// of radix passes over the whole key:
//   count    one block per old brick: how many of its particles go to each
//            neighbour, how many died, and an error flag when one went
//            further (cells changed behind the library's back)
//   totals   one thread per new brick: the sum over its sources
//   scan     one block: the new brick starts and the dead particles' starts
//   offsets  one thread per new brick: its sources in increasing old order,
//            and where each source's particles start in it
//   scatter  one block per old brick: every particle's slot in the
//            brick-grouped order (its stable rank among the block's particles
//            with the same destination)
//   local    one block per new brick: stable counting sort of its particles
//            by the cell inside the brick (64 cells), writing the permutation
//            and, when asked, moving every particle record into the other
//            particle set (in slot order; the reads follow the previous order
//            inside each cell).
// The result equals the stable sort by the brick key (the radix sort of
// k_sort.hip).  When the error flag is raised, the later kernels copy every
// particle unchanged instead (the identity permutation, the brick starts
// kept), and the sticky error word tells the host.
#include "block_util.h"
#include "step_device.h"

namespace picstep {

constexpr int BS_THREADS = 256;
constexpr int BS_BATCH = 4;  // rounds whose loads a thread issues together

__device__ __forceinline__ void brick_coords(const GridConst &g, int b, int c[3]) {
  c[0] = b % g.nbrick[0];
  b /= g.nbrick[0];
  c[1] = b % g.nbrick[1];
  c[2] = b / g.nbrick[1];
}

// destination code of a live particle of old brick ob: (dx+1) + 3 (dy+1)
// [+ 9 (dz+1)] for a move by (dx, dy, dz) bricks (the shorter way round a
// periodic dimension, which holds at least 3 bricks), or -1 beyond the
// neighbours
template <int DIM>
__device__ __forceinline__ int brick_move(const GridConst &g, const int ob[3], int32_t c) {
  int i[3];
  cell_decode(g, c, i);
  int code = 0, mul = 1;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    int d = (i[a] >> g.brick_shift[a]) - ob[a];
    if (g.geom == 0) {
      if (d > 1) d -= g.nbrick[a];
      else if (d < -1) d += g.nbrick[a];
    }
    if (d < -1 || d > 1) return -1;
    code += (d + 1) * mul;
    mul *= 3;
  }
  return code;
}

// The sources of new brick nbk in increasing old order: per dimension the
// source offsets o in the order of increasing source coordinate (a periodic
// dimension wraps at its ends; elsewhere sources outside the grid do not
// exist); f(source brick, destination code of the move source -> nbk).
template <int DIM, class F>
__device__ __forceinline__ void for_each_source(const GridConst &g, const int nbk[3], F f) {
  int ord[3][3], cnt[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ord[a][0] = -1;
    ord[a][1] = 0;
    ord[a][2] = 1;
    cnt[a] = 3;
    if (a >= DIM) {
      ord[a][0] = 0;
      cnt[a] = 1;
      continue;
    }
    const int n = g.nbrick[a], x = nbk[a];
    if (g.geom == 0) {
      if (x == 0) {  // x - 1 wraps to the largest
        ord[a][0] = 0;
        ord[a][1] = 1;
        ord[a][2] = -1;
      } else if (x == n - 1) {  // x + 1 wraps to the smallest
        ord[a][0] = 1;
        ord[a][1] = -1;
        ord[a][2] = 0;
      }
    } else {
      int k = 0;
      if (x > 0) ord[a][k++] = -1;
      ord[a][k++] = 0;
      if (x < n - 1) ord[a][k++] = 1;
      cnt[a] = k;
    }
  }
#pragma unroll
  for (int kz = 0; kz < 3; ++kz) {
    if (kz >= cnt[2]) break;
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      if (ky >= cnt[1]) break;
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        if (kx >= cnt[0]) break;
        const int o[3] = {ord[0][kx], ord[1][ky], ord[2][kz]};
        int s[3], code = 0, mul = 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          s[a] = nbk[a] + o[a];
          if (a < DIM) {
            if (s[a] < 0) s[a] += g.nbrick[a];
            if (s[a] >= g.nbrick[a]) s[a] -= g.nbrick[a];
            code += (1 - o[a]) * mul;  // the move from the source is -o
            mul *= 3;
          }
        }
        f(s[0] + g.nbrick[0] * (s[1] + g.nbrick[1] * s[2]), code);
      }
    }
  }
}

// lanes of the wave that are valid and hold the same code (bits wide)
__device__ __forceinline__ uint64_t same_code(int code, int bits, bool ok) {
  uint64_t m = __ballot(ok);
  for (int b = 0; b < bits; ++b) {
    const bool set = (code >> b) & 1;
    const uint64_t bb = __ballot(set);
    m &= set ? bb : ~bb;
  }
  return m;
}

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__global__ void k_bs_clear(int32_t *flag) { *flag = 0; }

template <int DIM>
__global__ __launch_bounds__(BS_THREADS) void k_bs_count(BrickSortArgs a) {
  constexpr int NN = (DIM == 3 ? 27 : 9) + 1;
  __shared__ int hc[NN];
  const int b = blockIdx.x;  // old bin; b == nb holds the particles already dead
  if (threadIdx.x < NN) hc[threadIdx.x] = 0;
  __syncthreads();
  int ob[3] = {0, 0, 0};
  if (b < a.nb) brick_coords(a.g, b, ob);
  const int i0 = a.bold[b], i1 = a.bold[b + 1];
  const uint64_t below = lanes_below();
  bool bad = false;
  for (int r0 = i0; r0 < i1; r0 += BS_BATCH * BS_THREADS) {
    int32_t cb[BS_BATCH];
#pragma unroll
    for (int k = 0; k < BS_BATCH; ++k) {
      const int i = r0 + k * BS_THREADS + (int)threadIdx.x;
      cb[k] = i < i1 ? a.cell[i] : 0;
    }
#pragma unroll
    for (int k = 0; k < BS_BATCH; ++k) {
      const int i = r0 + k * BS_THREADS + (int)threadIdx.x;
      bool ok = i < i1;
      int code = 0;
      if (ok) {
        const int32_t c = cb[k];
        code = (c & DEAD_BIT) ? NN - 1 : (b < a.nb ? brick_move<DIM>(a.g, ob, c) : -1);
        if (code < 0) {
          bad = true;
          ok = false;
          code = 0;
        }
      }
      const uint64_t peers = same_code(code, 5, ok);
      if (ok && (peers & below) == 0) atomicAdd(&hc[code], (int)__popcll(peers));
    }
  }
  if (bad) {
    a.flag[0] = 1;
    atomicOr(a.err, PIC_DEVERR_SORT_MOVE);
  }
  __syncthreads();
  if (threadIdx.x < NN) a.cnt[(int64_t)b * NN + threadIdx.x] = hc[threadIdx.x];
  if (threadIdx.x == 0) a.dpre[b] = hc[NN - 1];  // scanned in place
}

template <int DIM>
__global__ __launch_bounds__(BS_THREADS) void k_bs_totals(BrickSortArgs a) {
  constexpr int NN = (DIM == 3 ? 27 : 9) + 1;
  const int b = (int)(blockIdx.x * BS_THREADS + threadIdx.x);
  if (a.flag[0] || b >= a.nb) return;
  int nbk[3];
  brick_coords(a.g, b, nbk);
  int t = 0;
  for_each_source<DIM>(a.g, nbk, [&](int src, int code) { t += a.cnt[(int64_t)src * NN + code]; });
  a.tot[b] = t;
}

// exclusive scans of two arrays at once (src may be dst), 1024 threads, in
// chunks of 4096 elements with 4 consecutive elements per thread; the totals
// come back in tot[2]
__device__ void block_scan2(const int32_t *src0, int32_t *dst0, int L0, const int32_t *src1,
                            int32_t *dst1, int L1, int (*sh)[16], int tot[2]) {
  constexpr int T = 1024, E = 4;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int carry0 = 0, carry1 = 0;
  for (int base = 0; base < max(L0, L1); base += T * E) {
    const int i0 = base + (int)threadIdx.x * E;
    int v0[E], v1[E], s0 = 0, s1 = 0;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      v0[k] = (i0 + k < L0) ? src0[i0 + k] : 0;
      v1[k] = (i0 + k < L1) ? src1[i0 + k] : 0;
    }
#pragma unroll
    for (int k = 0; k < E; ++k) {
      s0 += v0[k];
      s1 += v1[k];
    }
    int x0 = s0, x1 = s1;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y0 = __shfl_up(x0, o, 64), y1 = __shfl_up(x1, o, 64);
      if (lane >= o) {
        x0 += y0;
        x1 += y1;
      }
    }
    if (lane == 63) {
      sh[0][w] = x0;
      sh[1][w] = x1;
    }
    __syncthreads();
    int p0 = 0, p1 = 0, t0 = 0, t1 = 0;
#pragma unroll
    for (int ww = 0; ww < T / 64; ++ww) {
      const int a = sh[0][ww], b = sh[1][ww];
      if (ww < w) {
        p0 += a;
        p1 += b;
      }
      t0 += a;
      t1 += b;
    }
    __syncthreads();
    int r0 = carry0 + p0 + x0 - s0, r1 = carry1 + p1 + x1 - s1;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      if (i0 + k < L0) dst0[i0 + k] = r0;
      if (i0 + k < L1) dst1[i0 + k] = r1;
      r0 += v0[k];
      r1 += v1[k];
    }
    carry0 += t0;
    carry1 += t1;
  }
  tot[0] = carry0;
  tot[1] = carry1;
}

__global__ __launch_bounds__(1024) void k_bs_scan(BrickSortArgs a) {
  __shared__ int sh[2][16];
  if (a.flag[0]) return;
  int tot[2];
  block_scan2(a.tot, a.bnew, a.nb, a.dpre, a.dpre, a.nb + 1, sh, tot);
  const int live = tot[0], dead = tot[1];
  if (threadIdx.x == 0) {
    a.bnew[a.nb] = live;
    a.bnew[a.nb + 1] = live + dead;
    // a particle counted towards a brick outside a non-periodic grid
    if ((int64_t)live + dead != a.n) {
      a.flag[0] = 1;
      atomicOr(a.err, PIC_DEVERR_SORT_MOVE);
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(BS_THREADS) void k_bs_offsets(BrickSortArgs a) {
  constexpr int NN = (DIM == 3 ? 27 : 9) + 1;
  const int b = (int)(blockIdx.x * BS_THREADS + threadIdx.x);
  if (a.flag[0] || b >= a.nb) return;
  int nbk[3];
  brick_coords(a.g, b, nbk);
  int run = a.bnew[b];
  // each (source, code) entry belongs to exactly one destination: in place
  for_each_source<DIM>(a.g, nbk, [&](int src, int code) {
    const int64_t k = (int64_t)src * NN + code;
    const int c = a.cnt[k];
    a.cnt[k] = run;
    run += c;
  });
}

template <int DIM>
__global__ __launch_bounds__(BS_THREADS) void k_bs_scatter(BrickSortArgs a) {
  constexpr int NN = (DIM == 3 ? 27 : 9) + 1;
  constexpr int NW = BS_THREADS / 64;
  __shared__ int base[NN];
  __shared__ int wcnt[NW][NN], wst[NW][NN];
  if (a.flag[0]) return;
  const int b = blockIdx.x;
  const int w = threadIdx.x >> 6;
  int ob[3] = {0, 0, 0};
  if (b < a.nb) brick_coords(a.g, b, ob);
  if (threadIdx.x < NN) {
    const int t = threadIdx.x;
    base[t] = (t < NN - 1) ? a.cnt[(int64_t)b * NN + t] : a.bnew[a.nb] + a.dpre[b];
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) wcnt[ww][t] = 0;
  }
  __syncthreads();
  const int i0 = a.bold[b], i1 = a.bold[b + 1];
  const uint64_t below = lanes_below();
  for (int rb = i0; rb < i1; rb += BS_BATCH * BS_THREADS) {
   int32_t cb[BS_BATCH];
#pragma unroll
   for (int k = 0; k < BS_BATCH; ++k) {
     const int i = rb + k * BS_THREADS + (int)threadIdx.x;
     cb[k] = i < i1 ? a.cell[i] : 0;
   }
#pragma unroll
   for (int k = 0; k < BS_BATCH; ++k) {
    const int i = rb + k * BS_THREADS + (int)threadIdx.x;
    const bool ok = i < i1;
    int code = 0;
    uint32_t key = 0;
    if (ok) {
      const int32_t c = cb[k];
      code = (c & DEAD_BIT) ? NN - 1 : brick_move<DIM>(a.g, ob, c);  // >= 0: the flag is clear
      key = brick_key(a.g, c, a.deadkey);
    }
    const uint64_t peers = same_code(code, 5, ok);
    const int r = (int)__popcll(peers & below);
    if (ok && r == 0) wcnt[w][code] = (int)__popcll(peers);
    __syncthreads();
    if (threadIdx.x < NN) {  // per code: the waves' starts in this round
      const int t = threadIdx.x;
      int run = base[t];
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) {
        const int x = wcnt[ww][t];
        wcnt[ww][t] = 0;
        wst[ww][t] = run;
        run += x;
      }
      base[t] = run;
    }
    __syncthreads();
    if (ok) {
      const int dst = wst[w][code] + r;
      a.tkey[dst] = key;
      a.tval[dst] = i;
    }
   }
  }
}

// one particle record from slot `from` of src to slot `to` of dst (all loads
// issued before the stores)
template <class Real>
__device__ __forceinline__ void move_record(const PSet<Real> &s, const PSet<Real> &d, int64_t off,
                                            int from, int to, int dim, int has_phi) {
  const int64_t f = off + from, t = off + to;
  const int32_t c = s.cell[f], id = s.id[f];
  OffT<Real> q[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) q[a] = (a < dim) ? s.offs[a][f] : (OffT<Real>)0;
  Real u[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = s.u[a][f];
  const Real w = s.w[f];
  const Real ph = has_phi ? s.phi[f] : (Real)0;
  d.cell[t] = c;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (a < dim) d.offs[a][t] = q[a];
#pragma unroll
  for (int a = 0; a < 3; ++a) d.u[a][t] = u[a];
  d.w[t] = w;
  if (has_phi) d.phi[t] = ph;
  d.id[t] = id;
}

// dest slots of the brick staged in LDS per window: the records are then
// moved in slot order (consecutive lanes write consecutive slots; the reads
// follow the previous order, which inside a cell is increasing)
constexpr int BS_WIN = 4096;

// NB records at once (every load before the first store): record from[k]
// (skipped when negative) to slot to0 + k * step
template <class Real, int NB>
__device__ __forceinline__ void move_records(const PSet<Real> &s, const PSet<Real> &d, int64_t off,
                                             const int from[NB], int to0, int step, int dim,
                                             int has_phi) {
  int32_t c[NB], id[NB];
  OffT<Real> q[3][NB];
  Real u[3][NB], w[NB], ph[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (from[k] < 0) continue;
    const int64_t f = off + from[k];
    c[k] = s.cell[f];
    id[k] = s.id[f];
#pragma unroll
    for (int a = 0; a < 3; ++a) q[a][k] = (a < dim) ? s.offs[a][f] : (OffT<Real>)0;
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a][k] = s.u[a][f];
    w[k] = s.w[f];
    ph[k] = has_phi ? s.phi[f] : (Real)0;
  }
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (from[k] < 0) continue;
    const int64_t t = off + to0 + (int64_t)k * step;
    d.cell[t] = c[k];
    d.id[t] = id[k];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (a < dim) d.offs[a][t] = q[a][k];
#pragma unroll
    for (int a = 0; a < 3; ++a) d.u[a][t] = u[a][k];
    d.w[t] = w[k];
    if (has_phi) d.phi[t] = ph[k];
  }
}

// MOVE: also move every particle record into dst (else only the permutation,
// which the next step then reads through)
template <class Real, bool MOVE>
__global__ __launch_bounds__(BS_THREADS) void k_bs_local(BrickSortArgs a, PSet<Real> src,
                                                         PSet<Real> dst, int64_t off, int dim,
                                                         int has_phi) {
  constexpr int NW = BS_THREADS / 64;
  constexpr int NC = 64;  // cells per brick
  __shared__ int cst[NC], cur[NC];
  __shared__ int wcnt[NW][NC], wst[NW][NC];
  __shared__ int lperm[BS_WIN];
  const int b = blockIdx.x;
  if (a.flag[0]) {  // the identity, over the old ranges (they cover every particle),
                    // whose starts stay those of the order
    for (int i = a.bold[b] + (int)threadIdx.x; i < a.bold[b + 1]; i += BS_THREADS) {
      a.perm[i] = i;
      if (MOVE) move_record(src, dst, off, i, i, dim, has_phi);
    }
    if (threadIdx.x == 0) {
      a.bnew[b] = a.bold[b];
      if (b == a.nb) a.bnew[b + 1] = a.bold[b + 1];
    }
    return;
  }
  const int j0 = a.bnew[b], j1 = a.bnew[b + 1];
  if (b == a.nb) {  // the dead keep their order
    for (int i = j0 + (int)threadIdx.x; i < j1; i += BS_THREADS) {
      const int v = a.tval[i];
      a.perm[i] = v;
      if (MOVE) move_record(src, dst, off, v, i, dim, has_phi);
    }
    return;
  }
  const int w = threadIdx.x >> 6;
  const uint32_t lmask = (1u << a.localbits) - 1;
  const uint64_t below = lanes_below();
  if (threadIdx.x < NC) {
    cst[threadIdx.x] = 0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) wcnt[ww][threadIdx.x] = 0;
  }
  __syncthreads();
  // cells' counts
  for (int rb = j0; rb < j1; rb += BS_BATCH * BS_THREADS) {
    uint32_t kb[BS_BATCH];
#pragma unroll
    for (int k = 0; k < BS_BATCH; ++k) {
      const int i = rb + k * BS_THREADS + (int)threadIdx.x;
      kb[k] = i < j1 ? a.tkey[i] : 0u;
    }
#pragma unroll
    for (int k = 0; k < BS_BATCH; ++k) {
      const int i = rb + k * BS_THREADS + (int)threadIdx.x;
      const bool ok = i < j1;
      const int lc = (int)(kb[k] & lmask);
      const uint64_t peers = same_code(lc, 6, ok);
      if (ok && (peers & below) == 0) atomicAdd(&cst[lc], (int)__popcll(peers));
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) {  // exclusive scan over the cells (one wave)
    const int v = cst[threadIdx.x];
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if ((int)threadIdx.x >= o) x += y;
    }
    cst[threadIdx.x] = j0 + x - v;
  }
  // windows of BS_WIN slots (one unless the brick holds more particles):
  // rank every particle (stable per cell), keep the slots of the window
  for (int w0 = j0; w0 < j1; w0 += BS_WIN) {
    __syncthreads();
    if (threadIdx.x < NC) cur[threadIdx.x] = cst[threadIdx.x];
    __syncthreads();
    for (int rb = j0; rb < j1; rb += BS_BATCH * BS_THREADS) {
     uint32_t kb[BS_BATCH];
     int vb[BS_BATCH];
#pragma unroll
     for (int k = 0; k < BS_BATCH; ++k) {
       const int i = rb + k * BS_THREADS + (int)threadIdx.x;
       kb[k] = i < j1 ? a.tkey[i] : 0u;
       vb[k] = i < j1 ? a.tval[i] : 0;
     }
#pragma unroll
     for (int k = 0; k < BS_BATCH; ++k) {
      const int i = rb + k * BS_THREADS + (int)threadIdx.x;
      const bool ok = i < j1;
      const int lc = (int)(kb[k] & lmask), v = vb[k];
      const uint64_t peers = same_code(lc, 6, ok);
      const int r = (int)__popcll(peers & below);
      if (ok && r == 0) wcnt[w][lc] = (int)__popcll(peers);
      __syncthreads();
      if (threadIdx.x < NC) {
        const int t = threadIdx.x;
        int run = cur[t];
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
          const int x = wcnt[ww][t];
          wcnt[ww][t] = 0;
          wst[ww][t] = run;
          run += x;
        }
        cur[t] = run;
      }
      __syncthreads();
      if (ok) {
        const int d = wst[w][lc] + r;
        if (d >= w0 && d < w0 + BS_WIN) lperm[d - w0] = v;
      }
     }
    }
    __syncthreads();
    const int we = min(j1, w0 + BS_WIN);
    for (int db = w0; db < we; db += BS_BATCH * BS_THREADS) {
      int vb[BS_BATCH];
#pragma unroll
      for (int k = 0; k < BS_BATCH; ++k) {
        const int d = db + k * BS_THREADS + (int)threadIdx.x;
        vb[k] = d < we ? lperm[d - w0] : -1;
        if (d < we) a.perm[d] = vb[k];
      }
      if (MOVE)
        move_records<Real, BS_BATCH>(src, dst, off, vb, db + (int)threadIdx.x, BS_THREADS, dim,
                                     has_phi);
    }
  }
}

template <int DIM, class Real>
hipError_t brick_sort_dim(const BrickSortArgs &a, const PSet<Real> &src, const PSet<Real> &dst,
                          int64_t off, int has_phi, bool move, hipStream_t s) {
  const unsigned bins = (unsigned)a.nb + 1, thr = (unsigned)((a.nb + BS_THREADS - 1) / BS_THREADS);
  hipLaunchKernelGGL(k_bs_clear, dim3(1), dim3(1), 0, s, a.flag);
  hipLaunchKernelGGL(k_bs_count<DIM>, dim3(bins), dim3(BS_THREADS), 0, s, a);
  hipLaunchKernelGGL(k_bs_totals<DIM>, dim3(thr), dim3(BS_THREADS), 0, s, a);
  hipLaunchKernelGGL(k_bs_scan, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(k_bs_offsets<DIM>, dim3(thr), dim3(BS_THREADS), 0, s, a);
  hipLaunchKernelGGL(k_bs_scatter<DIM>, dim3(bins), dim3(BS_THREADS), 0, s, a);
  if (move)
    hipLaunchKernelGGL((k_bs_local<Real, true>), dim3(bins), dim3(BS_THREADS), 0, s, a, src, dst,
                       off, a.g.dim, has_phi);
  else
    hipLaunchKernelGGL((k_bs_local<Real, false>), dim3(bins), dim3(BS_THREADS), 0, s, a, src, dst,
                       off, a.g.dim, has_phi);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_brick_sort(const BrickSortArgs &a, const PSet<Real> &src, const PSet<Real> &dst,
                             int64_t off, int has_phi, bool move, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  return a.g.dim == 3 ? brick_sort_dim<3, Real>(a, src, dst, off, has_phi, move, s)
                      : brick_sort_dim<2, Real>(a, src, dst, off, has_phi, move, s);
}

template hipError_t launch_brick_sort<float>(const BrickSortArgs &, const PSet<float> &,
                                             const PSet<float> &, int64_t, int, bool, hipStream_t);
template hipError_t launch_brick_sort<double>(const BrickSortArgs &, const PSet<double> &,
                                              const PSet<double> &, int64_t, int, bool,
                                              hipStream_t);

}  // namespace picstep
