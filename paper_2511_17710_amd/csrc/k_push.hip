// k_push.hip -- fused particle step: interpolate, rotate, Boris, move, deposit
// (arXiv 2511.17710, Sec. 2.3 steps 3-8), one launch for all species.
//
// A block owns a chunk of consecutive particles of one species (4 per
// thread in FP32, 2 in FP64, loaded with 16-byte vector accesses, or fewer
// for sparse species; read through the permutation of a sort on the step
// that follows it).  Particles are kept in brick order by the per-cell sort,
// so the chunk's cells form a compact box.  One LDS buffer
// serves in turn as the block's copy of the fields over that box (when it
// fits) for the push pass, and as the block's current tile over the box
// (plus the stencil halo) for the deposit pass: exact 64-bit fixed-point
// accumulation in FP32 builds, double in FP64 builds, flushed with one global
// atomic per nonzero value.  When the box outgrows the tile (particles
// drifted far since the last sort) the particles whose stencil leaves the
// tile read the fields and deposit in global memory; the sums are the same.
#include <type_traits>

#include "block_util.h"
#include "step_device.h"

namespace picstep {

// most particles per thread of the dense instance: 4 in FP32 contexts, 2 in
// FP64 ones (their registers: 4 particles need about 240 per lane, which
// holds a SIMD at 2 waves)
template <class Real>
constexpr int push_ppt() {
  return sizeof(Real) == 4 ? 4 : 2;
}
// LDS buffer per block (field copy, then current tile), sized so that the
// blocks a CU holds at once share its 160 KB: 4 blocks per CU (the FP64
// chunks of 512 particles need half the FP32 field copy's points).
template <class Real>
constexpr int tile_bytes() {
  return 39936;
}

// ---------------------------------------------------------------- vector I/O
__device__ __forceinline__ void ld4(const float *p, float v[4]) {
  const float4 x = *reinterpret_cast<const float4 *>(p);
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}
__device__ __forceinline__ void ld4(const uint32_t *p, uint32_t v[4]) {
  const uint4 x = *reinterpret_cast<const uint4 *>(p);
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}
__device__ __forceinline__ void ld4(const int32_t *p, int32_t v[4]) {
  const int4 x = *reinterpret_cast<const int4 *>(p);
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}
__device__ __forceinline__ void ld4(const double *p, double v[4]) {
  const double2 a = *reinterpret_cast<const double2 *>(p);
  const double2 b = *reinterpret_cast<const double2 *>(p + 2);
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void st4(float *p, const float v[4]) {
  *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st4(uint32_t *p, const uint32_t v[4]) {
  *reinterpret_cast<uint4 *>(p) = make_uint4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st4(int32_t *p, const int32_t v[4]) {
  *reinterpret_cast<int4 *>(p) = make_int4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st4(double *p, const double v[4]) {
  *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
  *reinterpret_cast<double2 *>(p + 2) = make_double2(v[2], v[3]);
}
__device__ __forceinline__ void ld2(const double *p, double v[2]) {
  const double2 a = *reinterpret_cast<const double2 *>(p);
  v[0] = a.x; v[1] = a.y;
}
__device__ __forceinline__ void ld2(const int32_t *p, int32_t v[2]) {
  const int2 a = *reinterpret_cast<const int2 *>(p);
  v[0] = a.x; v[1] = a.y;
}
__device__ __forceinline__ void ld2(const float *p, float v[2]) {
  const float2 a = *reinterpret_cast<const float2 *>(p);
  v[0] = a.x; v[1] = a.y;
}
__device__ __forceinline__ void ld2(const uint32_t *p, uint32_t v[2]) {
  const uint2 a = *reinterpret_cast<const uint2 *>(p);
  v[0] = a.x; v[1] = a.y;
}
__device__ __forceinline__ void st2(double *p, const double v[2]) {
  *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
}
__device__ __forceinline__ void st2(int32_t *p, const int32_t v[2]) {
  *reinterpret_cast<int2 *>(p) = make_int2(v[0], v[1]);
}
__device__ __forceinline__ void st2(float *p, const float v[2]) {
  *reinterpret_cast<float2 *>(p) = make_float2(v[0], v[1]);
}
__device__ __forceinline__ void st2(uint32_t *p, const uint32_t v[2]) {
  *reinterpret_cast<uint2 *>(p) = make_uint2(v[0], v[1]);
}
template <int N, class T>
__device__ __forceinline__ void ldv(const T *p, T v[N]) {
  if constexpr (N == 4) ld4(p, v); else ld2(p, v);
}
template <int N, class T>
__device__ __forceinline__ void stv(T *p, const T v[N]) {
  if constexpr (N == 4) st4(p, v); else st2(p, v);
}

template <int N, class T>
__device__ __forceinline__ void load_n(const T *p, int cnt, T v[N], T fill) {
  if (cnt == N) {
    ldv<N>(p, v);
  } else {
#pragma unroll
    for (int r = 0; r < N; ++r) v[r] = (r < cnt) ? p[r] : fill;
  }
}
template <int N, class T>
__device__ __forceinline__ void store_n(T *p, int cnt, const T v[N]) {
  if (cnt == N) {
    stv<N>(p, v);
  } else {
#pragma unroll
    for (int r = 0; r < N; ++r)
      if (r < cnt) p[r] = v[r];
  }
}

// ---------------------------------------------------------------- block -> chunk
// XCD-aware order (each XCD's L2 keeps the fields and current around its
// neighbouring chunks), except on the step that reads through a sort's
// permutation: there the blocks in flight on all XCDs sweep about one plane
// of bricks at a time, so the particles that came from the plane before are
// read while it is still cached (under the XCD order they were last touched
// many L2 capacities earlier: push 3.4 -> 3.2 ms on that step), and the
// chunks are dealt to the XCDs in segments of 32 (neighbouring chunks read
// much the same source lines, which one L2 then serves: 3.2 -> 3.05 ms).
// The debug launch with one block in flight takes the plain order.
constexpr int64_t GATHER_SEGMENT = 32;
template <bool SPARSE, int PPT>
__device__ __forceinline__ bool locate_chunk(const SpeciesTable &sp, int &s, int64_t &c0,
                                             bool gather, bool serial, int64_t base) {
  // blk0[MAXSP] = all blocks
  const int64_t bid = base + (int64_t)blockIdx.x;
  const int64_t nb = sp.blk0[MAXSP];
  const int64_t b = serial   ? bid
                    : gather ? xcd_segment_chunk(bid, nb, GATHER_SEGMENT)
                             : xcd_chunk(bid, nb);
  s = 0;
#pragma unroll
  for (int t = 1; t < MAXSP; ++t)
    if (t < sp.nspec && b >= sp.blk0[t]) s = t;
  c0 = (b - sp.blk0[s]) * ((int64_t)BLOCK * (SPARSE ? sp.ppt[s] : PPT));
  return c0 < sp.n[s];
}

// ---------------------------------------------------------------- per-particle steps
// Cartesian: tetrad F^i_hat = Delta_i F^i (eq. curvspace-tetradtrans with the
// Sec. 2.4 Cartesian metric, h33 = 1 in 2D); the basis is already global.
// A particle deposits into the block's LDS tile when its whole stencil (cell
// -1 ... cell +2 in every dimension, in the tile's unwrapped frame) lies
// inside it, else straight into the global current.
template <int DIM, class Acc>
__device__ __forceinline__ bool in_tile(const DepTarget<Acc> &tile, const int ts[3],
                                        const int ib[3]) {
  bool in = true;
#pragma unroll
  for (int a = 0; a < DIM; ++a) in = in && (ib[a] - 1 >= tile.o[a]) && (ib[a] + 2 < tile.o[a] + ts[a]);
  return in;
}


template <class Real>
using TileT = DepTarget<typename TileAcc<Real>::type>;

// Step m of every dimension packed two bits each (m + 1)
__device__ __forceinline__ int pack_m(const int m[3]) {
  return (m[0] + 1) | ((m[1] + 1) << 2) | ((m[2] + 1) << 4);
}
__device__ __forceinline__ void unpack_m(int p, int m[3]) {
  m[0] = (p & 3) - 1;
  m[1] = ((p >> 2) & 3) - 1;
  m[2] = ((p >> 4) & 3) - 1;
}

// fields at the particle: from the block's LDS copy when it covers the
// particle's stencil (always, unless CHK: the copy is a cube smaller than the
// chunk's box), else from global memory
template <int DIM, class Real, bool CHK>
__device__ __forceinline__ void particle_fields(const StepArgs<Real> &A, const FieldTile<Real> &ft,
                                                const int i[3], const int shift[3],
                                                const Stencil1<Real> st[3], Real F[6]) {
  int dsh[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a)
    if (shift[a] && i[a] < (A.g.n[a] >> 1)) dsh[a] = A.g.n[a];
  bool in = true;
  if (CHK) {
    int ib[3] = {i[0] + dsh[0], i[1] + dsh[1], i[2] + dsh[2]};
    in = fields_in_tile<DIM, Real>(ft, ib);
  }
  if (in)
    interp6_tile<DIM, Real>(ft, dsh, st, F);
  else
    interp6<DIM, Real>(A.EB, A.g, st, F);
}

template <int DIM, class Real, bool CHK, bool PUSHERS>
__device__ __forceinline__ int32_t cart_push(const StepArgs<Real> &A, const FieldTile<Real> &ft,
                                             const int shift[3], int s, int32_t c,
                                             OffT<Real> q[3], Real u[3], int &mp, Real &dx3,
                                             float &span) {
  using PS = Pos<Real>;
  const GridConst &g = A.g;
  int i[3];
  cell_decode(g, c, i);
  Stencil1<Real> st[3];
#pragma unroll
  for (int a = 0; a < DIM; ++a) st[a] = stencil1(i[a], (Real)PS::weight(q[a]));
  Real F[6];
  particle_fields<DIM, Real, CHK>(A, ft, i, shift, st, F);
  Real E[3], B[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const Real sc = (a < DIM) ? konst<Real>(g.dx[a], g.dxf[a]) : (Real)1;
    E[a] = F[a] * sc;
    B[a] = F[3 + a] * sc;
  }
  if (PUSHERS)
    push_momentum<Real>(A.sp, s, konst<Real>(A.sp.k[s], A.sp.kf[s]), A.dt, E, B, u);
  else
    boris(konst<Real>(A.sp.k[s], A.sp.kf[s]), E, B, u);
  // move (steps 6-7): offsets advance by dt u / (gamma Delta)
  const Real gi = rsqrt_r((Real)1 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const Real dtr = konst<Real>(A.dt, A.dtf);
  int m[3] = {0, 0, 0};
  int inew[3] = {i[0], i[1], i[2]};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const Real dx = cart_disp(g, a, dtr, u[a], gi);
    OffT<Real> qn;
    m[a] = PS::move(q[a], (double)dx, qn);
    // bound of the stored displacement: |dx| plus the rounding of the new
    // offset (2^-32 in the FP32 build, an ulp of 1 in the FP64 one)
    span = fmaxf(span, fabsf((float)dx) * 1.0001f + 0x1p-31f);
    q[a] = qn;
    int v = i[a] + m[a];
    v = (v < 0) ? v + g.n[a] : ((v >= g.n[a]) ? v - g.n[a] : v);  // periodic wrap
    inew[a] = v;
  }
  dx3 = (DIM == 2) ? dtr * u[2] * gi : (Real)0;
  mp = pack_m(m);
  return cell_encode(g, inew);
}

template <int GEOM, class Real, bool CHK, bool PUSHERS>
__device__ __forceinline__ int32_t axi_push(const StepArgs<Real> &A, const FieldTile<Real> &ft,
                                            int s, int32_t c, OffT<Real> q[3], Real u[3],
                                            Real &phi, int &mp, Real &dx3, float &span) {
  using PS = Pos<Real>;
  const GridConst &g = A.g;
  int i[3];
  cell_decode(g, c, i);
  const Real d1 = (Real)PS::weight(q[0]), d2 = (Real)PS::weight(q[1]);
  Stencil1<Real> st[3];
  st[0] = stencil1(i[0], d1);
  st[1] = stencil1(i[1], d2);
  Real F[6];
  const int noshift[3] = {0, 0, 0};
  particle_fields<2, Real, CHK>(A, ft, i, noshift, st, F);
  double dx1, dx2;
  Real phinew;
  const bool near = (i[0] < g.fp64_cells) || (i[1] < g.fp64_cells) ||
                    (i[1] >= g.n[1] - g.fp64_cells);
  if (sizeof(Real) == 8 || near) {
    double dphi;
    axi_particle<GEOM, double, Real, double, PUSHERS>(g, A.sp, s, A.dt, i[0], i[1],
                                                      PS::exact(q[0]), PS::exact(q[1]),
                                     phi, F, u, dx1, dx2, dphi);
    phinew = next_phi<Real, double>(phi, dphi);
    dx3 = (Real)dphi;
  } else {
    float f1, f2, dphi;
    axi_particle<GEOM, float, Real, Real, PUSHERS>(g, A.sp, s, A.dt, i[0], i[1], d1, d2, phi, F,
                                                   u, f1, f2, dphi);
    dx1 = f1;
    dx2 = f2;
    phinew = next_phi<Real, float>(phi, dphi);
    dx3 = (Real)dphi;
  }
  int m[3] = {0, 0, 0};
  OffT<Real> qn1, qn2;
  m[0] = PS::move(q[0], dx1, qn1);
  m[1] = PS::move(q[1], dx2, qn2);
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
  span = fmaxf(span, (float)fabs(PS::exact(qn1) + (double)m[0] - PS::exact(q[0])));
  span = fmaxf(span, (float)fabs(PS::exact(qn2) + (double)m[1] - PS::exact(q[1])));  // theta clamp
  q[0] = qn1;
  q[1] = qn2;
  phi = phinew;
  mp = pack_m(m);
  return cell_encode(g, inew) | (alive ? 0 : DEAD_BIT);
}

// Deposit (step 8) of one pushed particle from its old and new positions:
// zig-zag with the unwrapped step m; periodic ghosts are folded after the
// step, and a tile uses the image of the old cell that keeps the box compact.
template <int GEOM, int DIM, class Real>
__device__ __forceinline__ void deposit_particle(const StepArgs<Real> &A, int s, int32_t c_old,
                                                 const OffT<Real> qo[3], const OffT<Real> qn[3],
                                                 int mp, Real w, Real dx3,
                                                 const TileT<Real> &tile,
                                                 const DepTarget<Real> &glob, const int ts[3],
                                                 const int shift[3], int esc) {
  using PS = Pos<Real>;
  const GridConst &g = A.g;
  int i[3], m[3];
  cell_decode(g, c_old, i);
  unpack_m(mp, m);
  double za[3] = {0, 0, 0}, zb[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    za[a] = PS::exact(qo[a]);
    zb[a] = PS::exact(qn[a]) + (double)m[a];
  }
  // segment data in FP64 (exact differences of exact positions), rounded to
  // Real only where a float contribution is formed
  ZigZag<double> z;
  const int nseg = (m[0] | m[1] | m[2]) ? 2 : 1;
  if (nseg == 1)
    straight<DIM, double>(za, zb, z);
  else
    zigzag<DIM, double>(za, m, zb, z);
  int ib[3] = {i[0], i[1], i[2]};
  if (GEOM == 0) {
#pragma unroll
    for (int a = 0; a < DIM; ++a)
      if (shift[a] && i[a] < (g.n[a] >> 1)) ib[a] += g.n[a];
  }
  const Real C = (Real)A.sp.qdt[s] * w;
  if (in_tile<DIM>(tile, ts, ib)) {
    if constexpr (sizeof(Real) == 4)
      deposit_fixed<DIM>(tile, ldexp((double)A.sp.qdt[s] * (double)w, esc), ib, m, z,
                         (double)dx3, nseg);
    else
      deposit<DIM>(tile, C, ib, m, z, dx3, nseg);
  } else {
    deposit<DIM>(glob, C, i, m, z, dx3, nseg);
    if (A.stats) atomicAdd(A.stats + 1, 1);
  }
}

// ---------------------------------------------------------------- the kernel
// Waves per SIMD the register allocation must allow: the LDS buffer
// already limits a CU to 4 blocks of 4 waves, and the Cartesian FP32 kernel
// runs faster capped at that occupancy (128 VGPRs) than uncapped at 3 waves;
// the FP64 instances (2 particles per thread) are held to 3 (168 VGPRs); the
// other instances would spill heavily.
template <int GEOM, int DIM, class Real>
constexpr int push_waves() {
  return sizeof(Real) == 8 ? 3 : (GEOM == 0 ? 4 : 1);
}

// PUSHERS: some species uses another pusher than Boris (a separate instance,
// so the plain Boris kernel carries no code for them).  SPARSE: some species
// has fewer than 4 particles per thread (the dense instance keeps the
// constant layout of 4).
template <int GEOM, int DIM, class Real, bool PUSHERS, bool SPARSE>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(push_waves<GEOM, DIM, Real>(), 8)))
void k_push(StepArgs<Real> A) {
  using Acc = typename TileAcc<Real>::type;
  constexpr int TILE_VALS = tile_bytes<Real>() / (int)sizeof(Acc);
  constexpr int FIELD_VALS = tile_bytes<Real>() / (int)sizeof(Real);
  // one LDS buffer: the block's copy of the fields during the push pass,
  // then its current tile during the deposit pass
  __shared__ union {
    Acc j[TILE_VALS];
    Real f[FIELD_VALS];
  } lds;
  Acc *tile = lds.j;
  Real *ftile = lds.f;
  __shared__ int red[6 * (BLOCK / 64)];
  const GridConst &g = A.g;
  int s;
  int64_t c0;
  constexpr int PPT = push_ppt<Real>();
  if (!locate_chunk<SPARSE, PPT>(A.sp, s, c0, A.perm != nullptr, A.serial, A.block_base))
    return;  // uniform over the block
  const int ppt = SPARSE ? A.sp.ppt[s] : PPT;
  // a lane's ppt particles are consecutive (vector loads), and neighbouring
  // lanes 4 particles apart for ppt 4 and 2 (two waves interleave): a wave's
  // lanes then share each cell's field reads as broadcasts and spread the
  // deposit's same-address atomics alike (lanes 2 apart in FP64: 4.15 ->
  // 4.09 ms per step; 8 apart in FP32: 2.22 -> 2.33).  ppt 1 (below 3
  // particles per cell) keeps neighbouring lanes on neighbouring particles:
  // those lie in different cells anyway, and spreading them slowed the
  // sparsest species by 15 %
  const int lsh = (ppt == 2) ? 1 : 0;
  const int wv = (int)(threadIdx.x >> 6), ln = (int)(threadIdx.x & 63);
  const int slot = ((wv >> lsh) << (6 + lsh)) + (ln << lsh) + (wv & ((1 << lsh) - 1));
  const int64_t first = c0 + (int64_t)slot * ppt;
  const int cnt = (int)max((int64_t)0, min((int64_t)ppt, A.sp.n[s] - first));
  const int64_t p0 = A.sp.off[s] + first;

  int32_t cl[PPT];
  OffT<Real> qd[3][PPT];
  Real uu[3][PPT], ww[PPT], ph[PPT];
  if (A.perm) {  // first step after a sort: read through the permutation; the ids
                 // move to the sorted set here as well
    int32_t idv[PPT];
    int64_t js[PPT];
#pragma unroll
    for (int r = 0; r < PPT; ++r)
      js[r] = (r < cnt) ? A.sp.off[s] + (int64_t)A.perm[p0 + r] : A.sp.off[s];
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      const bool ok = r < cnt;
      cl[r] = ok ? A.src.cell[js[r]] : (int32_t)DEAD_BIT;
#pragma unroll
      for (int a = 0; a < DIM; ++a) qd[a][r] = ok ? A.src.offs[a][js[r]] : (OffT<Real>)0;
#pragma unroll
      for (int a = 0; a < 3; ++a) uu[a][r] = ok ? A.src.u[a][js[r]] : (Real)0;
      ww[r] = ok ? A.src.w[js[r]] : (Real)0;
      ph[r] = (ok && GEOM != 0) ? A.src.phi[js[r]] : (Real)0;
      idv[r] = ok ? A.src.id[js[r]] : 0;
    }
    store_n<PPT>(A.p.id + p0, cnt, idv);
  } else {
    load_n<PPT>(A.p.cell + p0, cnt, cl, (int32_t)DEAD_BIT);
#pragma unroll
    for (int a = 0; a < DIM; ++a) load_n<PPT>(A.p.offs[a] + p0, cnt, qd[a], (OffT<Real>)0);
#pragma unroll
    for (int a = 0; a < 3; ++a) load_n<PPT>(A.p.u[a] + p0, cnt, uu[a], (Real)0);
    load_n<PPT>(A.p.w + p0, cnt, ww, (Real)0);
    if (GEOM != 0) load_n<PPT>(A.p.phi + p0, cnt, ph, (Real)0);
  }
  if (A.write_prev) {
    store_n<PPT>(A.prev_cell + p0, cnt, cl);
#pragma unroll
    for (int a = 0; a < DIM; ++a) store_n<PPT>(A.prev_offs[a] + p0, cnt, qd[a]);
  }

  // bounding box of the chunk's current cells; a periodic dimension whose
  // cells span more than half the box is unwrapped (cells below N/2 shifted
  // by +N) so that a chunk straddling the boundary stays compact
  int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
  int ic[PPT][3];
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    cell_decode(g, cl[r], ic[r]);
    if (cl[r] & DEAD_BIT) continue;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = min(lo[d], ic[r][d]);
      hi[d] = max(hi[d], ic[r][d]);
    }
  }
  block_minmax3(lo, hi, red);
  if (lo[0] > hi[0]) {  // no live particle in the chunk (uniform)
    if (A.perm) {       // still move the frozen particles into the sorted set
      store_n<PPT>(A.p.cell + p0, cnt, cl);
#pragma unroll
      for (int a = 0; a < DIM; ++a) store_n<PPT>(A.p.offs[a] + p0, cnt, qd[a]);
#pragma unroll
      for (int a = 0; a < 3; ++a) store_n<PPT>(A.p.u[a] + p0, cnt, uu[a]);
      store_n<PPT>(A.p.w + p0, cnt, ww);
      if (GEOM != 0) store_n<PPT>(A.p.phi + p0, cnt, ph);
    }
    return;
  }
  int shift[3] = {0, 0, 0};
  if (GEOM == 0) {
    bool any = false;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      shift[d] = (hi[d] - lo[d] > (g.n[d] >> 1)) ? 1 : 0;
      any = any || shift[d];
    }
    if (any) {  // uniform: recompute the box on the shifted cells
      __syncthreads();
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lo[d] = INT32_MAX;
        hi[d] = INT32_MIN;
      }
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        if (cl[r] & DEAD_BIT) continue;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int v = ic[r][d] + ((shift[d] && ic[r][d] < (g.n[d] >> 1)) ? g.n[d] : 0);
          lo[d] = min(lo[d], v);
          hi[d] = max(hi[d], v);
        }
      }
      block_minmax3(lo, hi, red);
    }
  }
  // tile placement, for the field copy (stencils reach cell - 1 ... cell + 1)
  // and the current (cell - 1 ... cell + 2): the whole box when it fits, else
  // the largest cube (square in 2D) centred on the chunk's mean cell;
  // particles whose stencil leaves a tile read or deposit in global memory
  int t0[3] = {0, 0, 0}, ts[3] = {1, 1, 1}, f0[3] = {0, 0, 0}, fs[3] = {1, 1, 1};
  int64_t T = 1, TF = 1;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    ts[d] = hi[d] - lo[d] + 4;
    fs[d] = hi[d] - lo[d] + 3;
    T *= ts[d];
    TF *= fs[d];
  }
  const bool fit_j = 3 * T <= TILE_VALS;
  const bool fit_f = 6 * TF <= FIELD_VALS;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    t0[d] = lo[d] - 1;
    f0[d] = lo[d] - 1;
  }
  if (!fit_j || !fit_f) {  // uniform
    __syncthreads();
    int sum[3] = {0, 0, 0}, nl[3] = {0, 0, 0};
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      if (cl[r] & DEAD_BIT) continue;
      nl[0] += 1;
#pragma unroll
      for (int d = 0; d < DIM; ++d)
        sum[d] += ic[r][d] + ((shift[d] && ic[r][d] < (g.n[d] >> 1)) ? g.n[d] : 0);
    }
    block_sum3(sum, red);
    __syncthreads();
    block_sum3(nl, red);
    constexpr int SIDE = tile_side(TILE_VALS / 3, DIM);    // 3 SIDE^DIM <= TILE_VALS
    constexpr int SIDEF = tile_side(FIELD_VALS / 6, DIM);  // 6 SIDEF^DIM <= FIELD_VALS
    if (!fit_j) T = 1;
    if (!fit_f) TF = 1;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int ctr = (sum[d] + nl[0] / 2) / nl[0];
      if (!fit_j) {
        ts[d] = SIDE;
        t0[d] = ctr - SIDE / 2 - 1;
        T *= ts[d];
      }
      if (!fit_f) {
        fs[d] = SIDEF;
        f0[d] = ctr - SIDEF / 2;
        TF *= fs[d];
      }
    }
  }

  // copy the fields of the box (plus the stencil halo), or of the cube, into
  // LDS (periodic images on Cartesian grids; on curvilinear grids points
  // outside the padded lattice, which no particle stencil reaches, are left
  // zero)
  FieldTile<Real> ft;
  ft.F = ftile;
  ft.T = (int)TF;
  ft.sy = fs[0];
  ft.sz = fs[0] * fs[1];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    ft.o[d] = f0[d];
    ft.ts[d] = fs[d];
  }
  {
    const int npts = (int)g.npts;
    constexpr int WA = DIM - 1;  // walked axis (z in 3D, y in 2D)
    const int wstride = (DIM == 3) ? g.np[0] * g.np[1] : g.np[0];
    bool inside = true;  // uniform: the tile lies inside the padded lattice
#pragma unroll
    for (int d = 0; d < DIM; ++d) inside = inside && f0[d] >= -NG && f0[d] + fs[d] <= g.n[d] + NG;
    if (inside) {  // the ghost layers hold the periodic images (or the caller's values)
      tile_for_each_affine<16, Real>(
          6, DIM == 3 ? 2 : 1, fs[0], fs[1], fs[2], npts, wstride,
          [&](int ix, int iy) {
            return pad_index(g, f0[0] + ix, f0[1] + ((DIM == 3) ? iy : 0), f0[2], DIM);
          },
          [&](int gi, int) { return A.EB[gi]; }, [&](int, int x, Real v) { ftile[x] = v; });
    } else {
    // a point's padded index is its plane part (x, and y in 3D) plus the
    // walked axis times its stride; periodic images on Cartesian grids,
    // points outside the padded lattice (curvilinear) read as zero
    tile_for_each<16, Real>(
        6, DIM == 3 ? 2 : 1, fs[0], fs[1], fs[2],
        [&](int ix, int iy) {
          int gx = f0[0] + ix, gy = f0[1] + iy;
          bool ok = true;
          if (GEOM == 0) {
            gx = wrap_periodic(gx, g.n[0]);
            if (DIM == 3) gy = wrap_periodic(gy, g.n[1]);
          } else {
            ok = gx >= -NG && gx < g.n[0] + NG;
            if (DIM == 3) ok = ok && gy >= -NG && gy < g.n[1] + NG;
          }
          return PlanePt{(gx + NG) + ((DIM == 3) ? g.np[0] * (gy + NG) : 0), ok};
        },
        [&](const PlanePt &pp, int, int comp, int w) {
          int gw = f0[WA] + w;
          bool ok = pp.ok;
          if (GEOM == 0)
            gw = wrap_periodic(gw, g.n[WA]);
          else
            ok = ok && gw >= -NG && gw < g.n[WA] + NG;
          return ok ? A.EB[comp * npts + pp.off + wstride * (gw + NG)] : (Real)0;
        },
        [&](const PlanePt &, int x, int, int, Real v) { ftile[x] = v; });
    }
    __syncthreads();
  }


  const bool use_tile = A.deposit != 0;
  if (A.stats && A.deposit && threadIdx.x == 0) atomicAdd(A.stats, 1);

  // pass 1: interpolate, rotate, push and move every particle of the thread
  // (steps 3-7), keeping the old position for the deposit; two instances:
  // every stencil inside the field copy, or tested one by one against it
  int32_t co[PPT];
  OffT<Real> qo[3][PPT];
  int mp[PPT];
  Real d3[PPT];
  float bmax = 0.0f;
  bool nonfinite = false;  // a non-finite four-velocity (reported, not trapped)
  const Real qdt = (Real)A.sp.qdt[s];
  auto push_pass = [&](auto check) {
    constexpr bool CHK = decltype(check)::value;
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      co[r] = cl[r];
      mp[r] = 0;
      d3[r] = (Real)0;
#pragma unroll
      for (int a = 0; a < DIM; ++a) qo[a][r] = qd[a][r];
      if (r >= cnt || (cl[r] & DEAD_BIT)) continue;
      OffT<Real> q[3] = {qd[0][r], DIM > 1 ? qd[1][r] : (OffT<Real>)0,
                         DIM > 2 ? qd[2][r] : (OffT<Real>)0};
      Real u[3] = {uu[0][r], uu[1][r], uu[2][r]};
      float span = 0.0f;
      Real dx3;
      if (GEOM == 0) {
        cl[r] = cart_push<DIM, Real, CHK, PUSHERS>(A, ft, shift, s, cl[r], q, u, mp[r], dx3,
                                                   span);
      } else {
        Real p = ph[r];
        cl[r] = axi_push<GEOM, Real, CHK, PUSHERS>(A, ft, s, cl[r], q, u, p, mp[r], dx3, span);
        ph[r] = p;
      }
      d3[r] = dx3;
#pragma unroll
      for (int a = 0; a < DIM; ++a) qd[a][r] = q[a];
#pragma unroll
      for (int a = 0; a < 3; ++a) uu[a][r] = u[a];
      nonfinite = nonfinite || !(fabs(u[0]) + fabs(u[1]) + fabs(u[2]) < (Real)INFINITY);
      bmax = fmaxf(bmax, fabsf((float)(qdt * ww[r])) * fmaxf(span, fabsf((float)dx3)));
    }
  };
  if (fit_f)  // uniform
    push_pass(std::false_type{});
  else
    push_pass(std::true_type{});
  if (nonfinite && A.err) atomicOr(A.err, PIC_DEVERR_NONFINITE);

  store_n<PPT>(A.p.cell + p0, cnt, cl);
#pragma unroll
  for (int a = 0; a < DIM; ++a) store_n<PPT>(A.p.offs[a] + p0, cnt, qd[a]);
#pragma unroll
  for (int a = 0; a < 3; ++a) store_n<PPT>(A.p.u[a] + p0, cnt, uu[a]);
  if (A.perm) store_n<PPT>(A.p.w + p0, cnt, ww);  // the weights move with the sort
  if (GEOM != 0) store_n<PPT>(A.p.phi + p0, cnt, ph);
  if (!use_tile) return;  // uniform

  // the field copy is done with: the LDS buffer becomes the current tile
  __syncthreads();
  for (int x = threadIdx.x; x < 3 * (int)T; x += BLOCK) tile[x] = (Acc)0;

  // Fixed-point scale 2^esc of the FP32 tile from the block's largest
  // contribution bound: one particle adds at most B = |q w dt/m| max(span,
  // |dx3|) to any tile value (its segment fluxes along a dimension sum to
  // its displacement there, span the largest; shape weights are at most 1;
  // the out-of-plane current of 2D grids carries dx3).  With B 2^esc < 2^49
  // one contribution stays below the 2^51 of the rounding and the (at most
  // 1024) particles of the block below 2^60, and small displacements (cold plasma)
  // keep the full 48-bit resolution relative to the largest of the block.
  int esc = 0;
  if (sizeof(Acc) == 8 && sizeof(Real) == 4) {
    const float B = block_max_nonneg(bmax, red);  // also orders the tile zeroing
    if (B > 0.0f && B <= 3.0e38f) esc = 48 - ilogbf(B);
  } else {
    __syncthreads();  // tile zeroed
  }
  TileT<Real> tile_t;
  DepTarget<Real> glob_t;
  tile_t.J = tile;
  tile_t.cs = (int)T;
  tile_t.sy = ts[0];
  tile_t.sz = ts[0] * ts[1];
  tile_t.o[0] = t0[0];
  tile_t.o[1] = t0[1];
  tile_t.o[2] = t0[2];
  glob_t.J = A.J;
  glob_t.cs = (int)g.npts;
  glob_t.sy = g.np[0];
  glob_t.sz = g.np[0] * g.np[1];
  glob_t.o[0] = -NG;
  glob_t.o[1] = -NG;
  glob_t.o[2] = (DIM == 3) ? -NG : 0;

  // pass 2: deposit (step 8)
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    if (r >= cnt || (co[r] & DEAD_BIT)) continue;
    OffT<Real> a0[3] = {qo[0][r], DIM > 1 ? qo[1][r] : (OffT<Real>)0,
                        DIM > 2 ? qo[2][r] : (OffT<Real>)0};
    OffT<Real> a1[3] = {qd[0][r], DIM > 1 ? qd[1][r] : (OffT<Real>)0,
                        DIM > 2 ? qd[2][r] : (OffT<Real>)0};
    deposit_particle<GEOM, DIM, Real>(A, s, co[r], a0, a1, mp[r], ww[r], d3[r], tile_t, glob_t,
                                      ts, shift, esc);
  }

  if (use_tile) {
    __syncthreads();
    const int np0 = g.np[0], np01 = g.np[0] * g.np[1], npts = (int)g.npts;
    constexpr int WA = DIM - 1;  // walked axis
    const int wstride = (DIM == 3) ? np01 : np0;
    bool inside = true;  // uniform: the tile lies inside the padded lattice
#pragma unroll
    for (int d = 0; d < DIM; ++d) inside = inside && t0[d] >= -NG && t0[d] + ts[d] <= g.n[d] + NG;
    if (inside) {  // ghost values are folded into the active cells after the step
      tile_for_each_affine<8, Acc>(
          3, DIM == 3 ? 2 : 1, ts[0], ts[1], ts[2], npts, wstride,
          [&](int ix, int iy) {
            return pad_index(g, t0[0] + ix, t0[1] + ((DIM == 3) ? iy : 0), t0[2], DIM);
          },
          [&](int, int x) { return tile[x]; },
          [&](int gi, int, Acc acc) {
            if (acc != (Acc)0) atomic_add_r(A.J + gi, (Real)ldexp((double)acc, -esc));
          });
    } else {
    // periodic grids add straight into the image of each tile point
    tile_for_each<8, Acc>(
        3, DIM == 3 ? 2 : 1, ts[0], ts[1], ts[2],
        [&](int ix, int iy) {
          int gx = t0[0] + ix, gy = t0[1] + iy;
          if (GEOM == 0) {
            gx = wrap_periodic(gx, g.n[0]);
            if (DIM == 3) gy = wrap_periodic(gy, g.n[1]);
          }
          return PlanePt{(gx + NG) + ((DIM == 3) ? np0 * (gy + NG) : 0), true};
        },
        [&](const PlanePt &, int x, int, int) { return tile[x]; },
        [&](const PlanePt &pp, int, int comp, int w, Acc acc) {
          if (acc == (Acc)0) return;
          const Real v = (Real)ldexp((double)acc, -esc);
          int gw = t0[WA] + w;
          if (GEOM == 0) gw = wrap_periodic(gw, g.n[WA]);
          atomic_add_r(A.J + comp * npts + pp.off + wstride * (gw + NG), v);
        });
    }
  }
}

template <class Real, bool PUSHERS, bool SPARSE>
hipError_t launch_push_instance(const StepArgs<Real> &a, dim3 grid, dim3 block, hipStream_t s) {
  if (a.g.geom == 0) {
    if (a.g.dim == 2)
      hipLaunchKernelGGL((k_push<0, 2, Real, PUSHERS, SPARSE>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_push<0, 3, Real, PUSHERS, SPARSE>), grid, block, 0, s, a);
  } else if (a.g.geom == 1) {
    hipLaunchKernelGGL((k_push<1, 2, Real, PUSHERS, SPARSE>), grid, block, 0, s, a);
  } else {
    hipLaunchKernelGGL((k_push<2, 2, Real, PUSHERS, SPARSE>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

// serial: the debug launch with one block in flight (one launch per block,
// in the plain block order), for comparisons that rule out interference
// between blocks
template <class Real>
hipError_t launch_push_deposit(const StepArgs<Real> &a, hipStream_t s, bool serial) {
  const int64_t nblk = a.sp.blk0[a.sp.nspec];
  if (nblk == 0) return hipSuccess;
  bool pushers = false, sparse = false;
  for (int t = 0; t < a.sp.nspec; ++t) {
    pushers = pushers || a.sp.pusher[t] != 0;
    sparse = sparse || a.sp.ppt[t] != push_ppt<Real>();
  }
  auto launch = [&](const StepArgs<Real> &x, dim3 grid) {
    const dim3 block(BLOCK);
    // the other pushers take the general layout too (three instances, not four)
    if (pushers) return launch_push_instance<Real, true, true>(x, grid, block, s);
    return sparse ? launch_push_instance<Real, false, true>(x, grid, block, s)
                  : launch_push_instance<Real, false, false>(x, grid, block, s);
  };
  if (!serial) return launch(a, dim3((unsigned)nblk));
  StepArgs<Real> x = a;
  x.serial = 1;
  for (int64_t b = 0; b < nblk; ++b) {
    x.block_base = b;
    const hipError_t e = launch(x, dim3(1));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_push_deposit<float>(const StepArgs<float> &, hipStream_t, bool);
template hipError_t launch_push_deposit<double>(const StepArgs<double> &, hipStream_t, bool);

}  // namespace picstep
