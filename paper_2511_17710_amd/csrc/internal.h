// internal.h -- shared host/device definitions of libpicstep (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "picstep.h"

namespace picstep {

constexpr int NG = 2;                  // ghost cells per side (Sec. 3.1)
constexpr int MAXSP = 8;               // species per context
constexpr int32_t DEAD_BIT = 0x40000000;
constexpr int BLOCK = 256;             // threads per block of the particle kernels
constexpr int PUSH_PPT = 4;            // fused step kernel: most particles per thread
// reverse-step kernel: particles per thread (FP32 1: its registers are full
// with one; FP64 2)
template <class Real>
constexpr int adj_ppt() {
  return sizeof(Real) == 4 ? 1 : 2;
}
constexpr int adj_chunk(size_t elem_bytes) { return BLOCK * (elem_bytes == 4 ? 1 : 2); }

// Grid constants passed by value to kernels.
struct GridConst {
  int geom, dim;
  int n[3];
  int np[3];
  int64_t npts;
  double dx[3];                 // Cartesian cell sizes (1 for unused dims)
  double inv_dx[3];             // 1 / dx
  float dxf[3], inv_dxf[3];     // the same rounded to FP32 on the host (FP32 kernels
                                // read them from scalar registers, no conversion per use)
  double rmin, dr, dth;         // spherical: r = rmin + x1 dr, theta = x2 dth
  double Rmin, dR, dT, r0, vt;  // quasi-spherical: r = r0 + exp(Rmin + x1 dR), T = x2 dT
  int fp64_cells;               // FP32 curvilinear: cells near theta=0,pi and r_min done in FP64
  int shift2, shift3;           // cell packing
  int32_t mask1, mask2, mask3;
  int brick[3];                 // sort order: cells brick by brick (4^3 in 3D, 8^2 in 2D)
  int brick_shift[3];           // log2(brick)
  int nbrick[3];
};

// In-cell offset storage: the FP32 build keeps offsets as 32-bit unsigned
// fixed point (offset = q * 2^-32, uniform resolution over [0,1)), the FP64
// build as double.
template <class Real>
struct OffStore;
template <>
struct OffStore<float> {
  using T = uint32_t;
};
template <>
struct OffStore<double> {
  using T = double;
};
template <class Real>
using OffT = typename OffStore<Real>::T;

template <class Real>
struct PSet {  // SoA of one particle set (device pointers)
  int32_t *cell;
  OffT<Real> *offs[3];
  Real *u[3];
  Real *w;
  Real *phi;
  int32_t *id;  // loaded index within the species, carried through every sort
};

struct SpeciesTable {
  int nspec;
  int64_t off[MAXSP];      // element offset of the species range
  int64_t n[MAXSP];        // loaded particles
  int64_t blk0[MAXSP + 1]; // prefix of block counts over species
  int ppt[MAXSP];          // fused step kernel: particles per thread (1, 2 or 4)
  double k[MAXSP];         // q dt / (2 m rho0)
  float kf[MAXSP];         // k rounded to FP32 on the host
  double qdt[MAXSP];       // q / dt
  int pusher[MAXSP];       // 0 Boris, 1 Vay, +2 guiding-centre hybrid
  double gca_e_ovr[MAXSP]; // hybrid: guiding centre while |E| < e_ovr |B| ...
  double gca_larmor[MAXSP];  // ... and the nominal gyroradius is below this length
};

template <class Real>
struct StepArgs {
  GridConst g;
  SpeciesTable sp;
  PSet<Real> p;
  int32_t *prev_cell;      // written when write_prev
  OffT<Real> *prev_offs[3];
  const Real *EB;
  Real *J;
  double dt;
  float dtf;               // dt rounded to FP32 on the host
  int write_prev;
  int deposit;             // 0: move only (adjoint recompute)
  int32_t *stats;          // [0]: blocks, [1]: blocks that deposited with global atomics
  int32_t *err;            // sticky device error word (PIC_DEVERR_* bits)
  // a sort's pending reorder (perm == nullptr: none): particle i of a species
  // is read from src at the species-local index perm[i], and the step writes
  // the sorted, advanced particles into p
  const int32_t *perm;
  PSet<Real> src;
  // debug launch with one block in flight: this launch is block block_base
  // of the whole grid (serial != 0; then blocks take the plain order)
  int64_t block_base;
  int serial;
};

// reverse step: recompute the forward step from the stored state and
// propagate adjoints (lamJ only on the last step)
template <class Real>
struct AdjArgs {
  GridConst g;
  SpeciesTable sp;
  PSet<Real> p;            // state before the step (read only)
  const Real *EB;
  const Real *lamJ;        // may be null
  Real *lam_u[3];          // in: adjoint of u after the step; out: before
  Real *lam_d[3];          // likewise for offsets
  Real *lam_phi;           // axisymmetric
  Real *dEB;               // accumulated field adjoint
  double dt;
};

// ---- launchers (defined in the .hip files) ----
template <class Real>
hipError_t launch_push_deposit(const StepArgs<Real> &a, hipStream_t s, bool serial = false);
template <class Real>
hipError_t launch_adjoint_step(const AdjArgs<Real> &a, hipStream_t s);
template <class Real>
hipError_t launch_fill_ghosts(const GridConst &g, Real *A, int ncomp, hipStream_t s);
template <class Real>
hipError_t launch_fold_ghosts(const GridConst &g, Real *A, int ncomp, hipStream_t s);
template <class Real>
hipError_t launch_zero(Real *A, int64_t n, hipStream_t s);
// field solver (k_fields.hip)
template <class Real>
hipError_t launch_faraday(const GridConst &g, Real *EB, double f, hipStream_t s);
template <class Real>
hipError_t launch_ampere(const GridConst &g, Real *EB, const Real *J, double dt, double coupling,
                         hipStream_t s);
template <class Real>
hipError_t launch_filter(const GridConst &g, const Real *in, Real *out, hipStream_t s);

// stable sort of one species range by cell key; writes perm (new i <- old perm[i])
struct SortScratch {
  uint32_t *keys[2];
  int32_t *vals[2];
  int32_t *hist;      // tile histograms, tile-major: max_tiles x 256
  int32_t *bsum;      // column sums of tile chunks: SCAN_CHUNKS x 256
  int64_t max_tiles;
};
// keys_out (optional): where the sorted keys are left
hipError_t launch_sort_species(const GridConst &g, const int32_t *cell, int64_t n,
                               const SortScratch &S, int32_t *perm_out, int keybits,
                               hipStream_t s, const uint32_t **keys_out = nullptr);
// brick starts of a sorted key sequence: bstart[b] = first index of brick b,
// bstart[nb] = first dead particle, bstart[nb + 1] = n
hipError_t launch_brick_bounds(const uint32_t *keys, int64_t n, int nb, int localbits,
                               uint32_t deadkey, int32_t *bstart, hipStream_t s);

// brick-neighbour sort of one species (k_bsort.hip): the species is in the
// order of its previous sort, whose brick starts are bold, and no particle
// has since crossed more than one brick in any dimension
struct BrickSortArgs {
  GridConst g;
  int nb;                // bricks
  int localbits;         // bits of the cell inside a brick (64 cells)
  uint32_t deadkey;
  int64_t n;             // particles of the species
  const int32_t *cell;   // species range, previous order
  const int32_t *bold;   // nb + 2: previous brick starts (entry nb: the dead), [nb + 1] = n
  int32_t *bnew;         // nb + 2: the new brick starts
  int32_t *cnt;          // (nb + 1) x (3^dim + 1): counts per destination, then its start
  int32_t *tot;          // nb: particles per new brick
  int32_t *dpre;         // nb + 1: dead particles of each old bin, then the exclusive prefix
  uint32_t *tkey;        // n: keys in brick-grouped order
  int32_t *tval;         // n: their previous indices
  int32_t *perm;         // n: new i <- previous perm[i]
  int32_t *flag;         // raised when a particle moved beyond the neighbours
  int32_t *err;          // sticky device error word
};
// writes the permutation; move: also moves every particle record from src
// into dst (species offset off)
template <class Real>
hipError_t launch_brick_sort(const BrickSortArgs &a, const PSet<Real> &src, const PSet<Real> &dst,
                             int64_t off, int has_phi, bool move, hipStream_t s);
template <class Real>
hipError_t launch_gather(const PSet<Real> &src, const PSet<Real> &dst, int dim, int has_phi,
                         int64_t off, int64_t n, const int32_t *perm, hipStream_t s);
template <class Real>
hipError_t launch_scatter_back(const Real *src, Real *dst, int64_t off, int64_t n,
                               const int32_t *perm, hipStream_t s);

constexpr int SORT_TILE = 4096;  // keys per block in the radix passes
constexpr int SCAN_CHUNKS = 64;  // most tile chunks of the histogram scan

}  // namespace picstep
