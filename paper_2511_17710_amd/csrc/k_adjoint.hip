// k_adjoint.hip -- reverse-mode derivative of one particle step (Cartesian
// grids), written by hand: the forward step of the particle is recomputed in
// registers from its stored state, then the adjoints are propagated backwards
// through the zig-zag deposit (a gather of dL/dJ), the move, the Boris push
// and the interpolation (a scatter into dL/dE, dL/dB).  Discrete branches
// (cell crossings, the relay clamp, the half-cell stagger choice) take the
// derivative of the branch the forward step took.
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

// copy ncomp components of a padded global array over the box [o, o + s) of
// (unwrapped) cells into LDS, component-major, x fastest; Cartesian grids
// take the periodic image of points outside the padded lattice
template <int DIM, class Real>
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
          const int gx = wrap_periodic(o[0] + ix, g.n[0]);
          const int gy = (DIM == 3) ? wrap_periodic(o[1] + iy, g.n[1]) : 0;
          return PlanePt{(gx + NG) + ((DIM == 3) ? g.np[0] * (gy + NG) : 0), true};
        },
        [&](const PlanePt &pp, int, int comp, int w) {
          return src[comp * npts + pp.off + wstride * (wrap_periodic(o[WA] + w, g.n[WA]) + NG)];
        },
        [&](const PlanePt &, int x, int, int, Real v) { dst[x] = v; });
  }
}

// One particle per thread, BLOCK particles per block in XCD-aware order.  The
// scatter into dL/dE, dL/dB (the adjoint of the interpolation) goes to an LDS
// tile over the block's cells, accumulated like the forward current (64-bit
// fixed point in FP32 builds, scaled by the block's largest |dL/dF|) and
// flushed with one global atomic per nonzero value; particles whose stencil
// leaves the tile scatter with global atomics.
// Waves per SIMD the register allocation must allow: the FP32 instances run
// faster at 4 (a few spills) than uncapped at 3 (0.457 -> 0.41 ms per step on
// the 64^3 workload); the FP64 ones stay uncapped.
template <class Real>
constexpr int adj_waves() {
  return sizeof(Real) == 4 ? 4 : 1;
}

template <int DIM, class Real>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(adj_waves<Real>(), 8)))
void k_adjoint_cart(AdjArgs<Real> A) {
  using PS = Pos<Real>;
  using Acc = typename TileAcc<Real>::type;
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
  const int64_t local = (blk - A.sp.blk0[s]) * BLOCK + threadIdx.x;
  const bool inrange = local < A.sp.n[s];
  const int64_t p = A.sp.off[s] + (inrange ? local : 0);
  const int32_t cc = inrange ? A.p.cell[p] : (int32_t)DEAD_BIT;
  // a frozen (dead) particle maps to itself: its adjoints pass through
  const bool live = !(cc & DEAD_BIT);
  int i[3];
  cell_decode(g, cc, i);

  // ---------------- the block's box and its LDS tile (stencils reach i-1 .. i+1)
  int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
  if (live) {
#pragma unroll
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = i[d];
  }
  block_minmax3(lo, hi, red);
  if (lo[0] > hi[0]) return;  // no live particle in the block (uniform)
  int shift[3] = {0, 0, 0}, ib[3] = {i[0], i[1], i[2]};
  bool any = false;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    shift[d] = (hi[d] - lo[d] > (g.n[d] >> 1)) ? 1 : 0;
    any = any || shift[d];
    if (shift[d] && ib[d] < (g.n[d] >> 1)) ib[d] += g.n[d];
  }
  if (any) {  // a block straddling a periodic boundary: box of the unwrapped cells
    __syncthreads();
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = live ? ib[d] : INT32_MAX;
      hi[d] = live ? ib[d] : INT32_MIN;
    }
    block_minmax3(lo, hi, red);
  }
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
    int sum[3] = {0, 0, 0}, nl[3] = {live ? 1 : 0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) sum[d] = live ? ib[d] : 0;
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
    stage_box<DIM, Real>(g, A.EB, 6, t0, ts, lds.f);
    if (A.lamJ) stage_box<DIM, Real>(g, A.lamJ, 3, j0, js, lds.f + 6 * T);
    __syncthreads();
  }
  const int dsh[3] = {ib[0] - i[0], ib[1] - i[1], ib[2] - i[2]};  // unwrapped - stored

  Real Fbar[6] = {0, 0, 0, 0, 0, 0};
  Stencil1<Real> st[3];
  float bmax = 0.0f;
  if (live) {
  OffT<Real> q[3];
  Real d[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    q[a] = A.p.offs[a][p];
    d[a] = (Real)PS::weight(q[a]);
  }
  const Real u0[3] = {A.p.u[0][p], A.p.u[1][p], A.p.u[2][p]};
  const Real w = A.p.w[p];
  const Real k = (Real)A.sp.k[s];
  const Real dtr = (Real)A.dt;

  // ---------------- forward recompute (step 3: interpolation, keeping corners)
#pragma unroll
  for (int a = 0; a < DIM; ++a) st[a] = stencil1(i[a], d[a]);
  Real F[6];
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
  if (stage)
    interp6_tile<DIM, Real>(ft, dsh, st, F);
  else
    interp6<DIM, Real>(A.EB, g, st, F);
  Real E[3], B[3], sc[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    sc[a] = (a < DIM) ? (Real)g.dx[a] : (Real)1;
    E[a] = F[a] * sc[a];
    B[a] = F[3 + a] * sc[a];
  }
  // step 5: Boris, keeping intermediates
  Real um[3], t[3], s3[3], up[3], un[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) um[a] = u0[a] + k * E[a];
  // same operations as the forward kernel, so the recomputed step is identical
  const Real igm = rsqrt_r((Real)1 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
#pragma unroll
  for (int a = 0; a < 3; ++a) t[a] = k * B[a] * igm;
  const Real tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  const Real sf = (Real)2 * rcp_r((Real)1 + tt);
#pragma unroll
  for (int a = 0; a < 3; ++a) s3[a] = t[a] * sf;
  up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
  up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
  up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
  un[0] = um[0] + (up[1] * s3[2] - up[2] * s3[1]) + k * E[0];
  un[1] = um[1] + (up[2] * s3[0] - up[0] * s3[2]) + k * E[1];
  un[2] = um[2] + (up[0] * s3[1] - up[1] * s3[0]) + k * E[2];
  // steps 6-7: move
  const Real ig = rsqrt_r((Real)1 + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
  int m[3] = {0, 0, 0};
  double za[3] = {0, 0, 0}, zb[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const Real dx = cart_disp(g, a, dtr, un[a], ig);  // as in the forward kernel
    OffT<Real> qn;
    m[a] = PS::move(q[a], (double)dx, qn);
    za[a] = PS::exact(q[a]);
    zb[a] = PS::exact(qn) + (double)m[a];
  }

  // ---------------- reverse
  Real ab[3] = {0, 0, 0};   // adjoint of the old offsets
  Real dxb[3] = {0, 0, 0};  // adjoint of the in-plane displacements
  Real dx3b = 0;            // adjoint of the out-of-plane displacement (2D)
  // adjoint of the new offsets passes to the old offset and the displacement
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const Real l = A.lam_d[a][p];
    ab[a] += l;
    dxb[a] += l;
  }
  // step 8 reversed: gather dL/dJ through the zig-zag segments
  if (A.lamJ) {
    const Real C = (Real)A.sp.qdt[s] * w;
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
    const Real dx3 = (DIM == 2) ? dtr * un[2] * ig : (Real)0;
    Real Fb[2][3] = {{0, 0, 0}, {0, 0, 0}}, Wb[2][3] = {{0, 0, 0}, {0, 0, 0}};
    // dL/dJ from the LDS copy (box frame) or from global memory
    const Real *L = stage ? lds.f + 6 * T : A.lamJ;
    const int cs = stage ? TJ : (int)g.npts;
    const int sy = stage ? js[0] : g.np[0];
    const int sz = stage ? js[0] * js[1] : g.np[0] * g.np[1];
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
      const int I = i[0] + (sg ? m[0] : 0), Jc = i[1] + (sg ? m[1] : 0);
      const int K = (DIM == 3) ? i[2] + (sg ? m[2] : 0) : 0;
      const int base = stage ? (I + dsh[0] - j0[0]) + sy * (Jc + dsh[1] - j0[1]) +
                                   ((DIM == 3) ? sz * (K + dsh[2] - j0[2]) : 0)
                             : pad_index(g, I, Jc, K, DIM);
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
        const Real Fz = Fs[sg][2], Wz = Ws[sg][2];
        // component c with transverse dims (a, b): value = C F_c (w_a w_b + sgn F_a F_b / 12)
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) {
          const int da = (comp == 0) ? 1 : 0;
          const int db = (comp == 2) ? 1 : 2;
          const int sa = (da == 0) ? 1 : sy;
          const int sb = (db == 1) ? sy : sz;
          const Real *Lc = L + comp * cs + base;
          const Real l00 = Lc[0], l10 = Lc[sa], l01 = Lc[sb], l11 = Lc[sa + sb];
          const Real Fc = (comp == 0) ? Fx : (comp == 1 ? Fy : Fz);
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
        (void)Fz;
        (void)Wz;
      }
    }
    // relay: F1 = xr - a, F2 = b - xr, W1 = (a + xr)/2, W2 = (xr + b)/2 - m
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      Real xrb = Fb[0][a] - Fb[1][a] + (Real)0.5 * (Wb[0][a] + Wb[1][a]);
      Real abar = -Fb[0][a] + (Real)0.5 * Wb[0][a];
      Real bbar = Fb[1][a] + (Real)0.5 * Wb[1][a];
      if (mid_free[a]) {  // xr = (a + b)/2
        abar += (Real)0.5 * xrb;
        bbar += (Real)0.5 * xrb;
      }
      // b = a + dx
      ab[a] += abar + bbar;
      dxb[a] += bbar;
    }
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
  // step 5 reversed (Boris)
  Real Eb[3], Bb[3], umb[3], upb[3], sb[3], tb[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Eb[a] = k * unb[a];  // u+ = u+' + k E
    umb[a] = unb[a];     // u+' = um + up x s
  }
  // up x s: upb += s x unb, sb = unb x up
  upb[0] = s3[1] * unb[2] - s3[2] * unb[1];
  upb[1] = s3[2] * unb[0] - s3[0] * unb[2];
  upb[2] = s3[0] * unb[1] - s3[1] * unb[0];
  sb[0] = unb[1] * up[2] - unb[2] * up[1];
  sb[1] = unb[2] * up[0] - unb[0] * up[2];
  sb[2] = unb[0] * up[1] - unb[1] * up[0];
  // up = um + um x t: umb += upb + t x upb, tb = upb x um
#pragma unroll
  for (int a = 0; a < 3; ++a) umb[a] += upb[a];
  umb[0] += t[1] * upb[2] - t[2] * upb[1];
  umb[1] += t[2] * upb[0] - t[0] * upb[2];
  umb[2] += t[0] * upb[1] - t[1] * upb[0];
  tb[0] = upb[1] * um[2] - upb[2] * um[1];
  tb[1] = upb[2] * um[0] - upb[0] * um[2];
  tb[2] = upb[0] * um[1] - upb[1] * um[0];
  // s = t sf, sf = 2 / (1 + t.t)
  const Real ts = t[0] * sb[0] + t[1] * sb[1] + t[2] * sb[2];
  const Real c4 = (Real)4 / (((Real)1 + tt) * ((Real)1 + tt));
#pragma unroll
  for (int a = 0; a < 3; ++a) tb[a] += sf * sb[a] - c4 * t[a] * ts;
  // t = k B / gm
  Real gmb = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Bb[a] = k * igm * tb[a];
    gmb -= t[a] * tb[a] * igm;
  }
  // gm = sqrt(1 + um.um); um = u + k E
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    umb[a] += gmb * um[a] * igm;
    Eb[a] += k * umb[a];
  }
  // tetrad reversed; the offset derivative of the interpolation
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Fbar[a] = Eb[a] * sc[a];
    Fbar[3 + a] = Bb[a] * sc[a];
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const int sx = kStag[c][0], sy2 = kStag[c][1], sz2 = kStag[c][2];
    const int bx = sx ? st[0].bh : st[0].b0;
    const int by = sy2 ? st[1].bh : st[1].b0;
    const int bz = (DIM == 3) ? (sz2 ? st[2].bh : st[2].b0) : 0;
    const Real fx = sx ? st[0].fh : st[0].f0;
    const Real fy = sy2 ? st[1].fh : st[1].f0;
    const Real fz = (DIM == 3) ? (sz2 ? st[2].fh : st[2].f0) : (Real)0;
    Real cv[8];
    if (stage)
      corners<DIM, Real>(lds.f + c * T, (bx + dsh[0] - t0[0]) + ft.sy * (by + dsh[1] - t0[1]) +
                                            ((DIM == 3) ? ft.sz * (bz + dsh[2] - t0[2]) : 0),
                         ft.sy, ft.sz, cv);
    else
      corners<DIM, Real>(A.EB + c * (int)g.npts, pad_index(g, bx, by, bz, DIM), g.np[0],
                         g.np[0] * g.np[1], cv);
    const Real gx = (Real)1 - fx, gy = (Real)1 - fy, gz = (Real)1 - fz;
    const Real fb = Fbar[c];
    bmax = fmaxf(bmax, fabsf((float)fb));
    if (DIM == 2) {
      ab[0] += fb * (gy * (cv[1] - cv[0]) + fy * (cv[3] - cv[2]));
      ab[1] += fb * (gx * (cv[2] - cv[0]) + fx * (cv[3] - cv[1]));
    } else {
      ab[0] += fb * (gz * (gy * (cv[1] - cv[0]) + fy * (cv[3] - cv[2])) +
                     fz * (gy * (cv[5] - cv[4]) + fy * (cv[7] - cv[6])));
      ab[1] += fb * (gz * (gx * (cv[2] - cv[0]) + fx * (cv[3] - cv[1])) +
                     fz * (gx * (cv[6] - cv[4]) + fx * (cv[7] - cv[5])));
      ab[2] += fb * (gy * (gx * (cv[4] - cv[0]) + fx * (cv[5] - cv[1])) +
                     fy * (gx * (cv[6] - cv[2]) + fx * (cv[7] - cv[3])));
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) A.lam_u[a][p] = umb[a];
#pragma unroll
  for (int a = 0; a < DIM; ++a) A.lam_d[a][p] = ab[a];
  }  // live

  // ---------------- scatter of dL/dF into the tile (or global memory)
  // Fixed-point scale 2^esc (FP32): one particle adds at most max|dL/dF| to a
  // tile value (interpolation weights are at most 1), so with B 2^esc < 2^49
  // the BLOCK particles of the block stay below 2^57.
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
  if (live) {
    bool in = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) in = in && (ib[d] - 1 >= t0[d]) && (ib[d] + 1 < t0[d] + ts[d]);
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
        const Real fb = tile_coef(Fbar[c], esc);
        const int base = c * T + (bx + dsh[0] - t0[0]) + sy * (by + dsh[1] - t0[1]) +
                         ((DIM == 3) ? sz * (bz + dsh[2] - t0[2]) : 0);
#pragma unroll
        for (int e = 0; e < (1 << DIM); ++e) {
          const int o = (e & 1) + ((e >> 1) & 1) * sy + ((DIM == 3) ? ((e >> 2) & 1) * sz : 0);
          atomic_add_r(tile + base + o, fb * wt[e]);
        }
      } else {
        const Real fb = Fbar[c];
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
  tile_for_each<8, Acc>(
      6, DIM == 3 ? 2 : 1, ts[0], ts[1], ts[2],
      [&](int ix, int iy) {
        const int gx = wrap_periodic(t0[0] + ix, g.n[0]);
        const int gy = (DIM == 3) ? wrap_periodic(t0[1] + iy, g.n[1]) : 0;
        return PlanePt{(gx + NG) + ((DIM == 3) ? np0 * (gy + NG) : 0), true};
      },
      [&](const PlanePt &, int x, int, int) { return tile[x]; },
      [&](const PlanePt &pp, int, int comp, int w, Acc acc) {
        if (acc == (Acc)0) return;
        const Real v = (Real)ldexp((double)acc, -esc);
        const int gw = wrap_periodic(t0[WA] + w, g.n[WA]);
        atomic_add_r(A.dEB + comp * npts + pp.off + wstride * (gw + NG), v);
      });
}

template <class Real>
hipError_t launch_adjoint_step(const AdjArgs<Real> &a, hipStream_t s) {
  const int64_t nblk = a.sp.blk0[a.sp.nspec];
  if (nblk == 0) return hipSuccess;
  if (a.g.geom != 0) return hipErrorNotSupported;
  dim3 grid((unsigned)nblk), block(BLOCK);
  if (a.g.dim == 2)
    hipLaunchKernelGGL((k_adjoint_cart<2, Real>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((k_adjoint_cart<3, Real>), grid, block, 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_adjoint_step<float>(const AdjArgs<float> &, hipStream_t);
template hipError_t launch_adjoint_step<double>(const AdjArgs<double> &, hipStream_t);

}  // namespace picstep
