// Shared host/device definitions of the MDLG HIP library (kernels + host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mdlg {

constexpr int kBlock = 256;          // threads per block for every kernel
constexpr int kWaves = kBlock / 64;  // wave64
constexpr int kScanTile = 1024;      // cells per block of the cell-start scan
constexpr int kTileCopies = 8;       // copies of the scan-tile totals (one per XCD of the adding block)
constexpr int kScanItems = kScanTile / kBlock;
constexpr int kPartChunkMax = 512;   // particles per block of the per-particle kernels
constexpr int kCountChunkMax = 2048; // particles per block of the counting pass (at most)
constexpr int kMaxStripSites = 16;   // lattice sites per block of the binning kernel
constexpr int kMaxQ = 225;           // largest velocity window handled (V <= 7 in 2D, V <= 2 in 3D)
constexpr int kMaxShifts = 32;       // displaced / moving lattices binned beside the main one

// LDS budgets of the force kernel
constexpr int kMaxHalo2 = 1536;      // halo cells per brick (2D)
constexpr int kMaxHalo3 = 2560;      // halo cells per brick (3D)
constexpr int kBrickLdsBytes = 60 * 1024;  // dynamic LDS budget of a brick kernel
constexpr int kMaxRows = 64;         // brick rows (BY * BZ)

// Byte layout of a brick kernel's dynamic LDS: the staged coordinates (cap +
// pad of `coord` bytes, first, so that a list entry addresses them with one
// shift), the adjoint velocities (`lam` bytes per staged particle), the halo
// tables (LDS start and global start of every halo cell) and the halo cell of
// every staged slot (16 bits), each part on a 16-byte boundary.
struct BrickLdsLayout {
  size_t lam, hs, scell, end;
};
__host__ __device__ inline size_t lds_up16(size_t x) { return (x + 15) & ~size_t(15); }
__host__ __device__ inline BrickLdsLayout brick_lds_layout(int cap, int pad, size_t coord, size_t lam,
                                                           int lmaxh) {
  BrickLdsLayout o;
  o.lam = lds_up16((size_t)(cap + pad) * coord);
  o.hs = o.lam + lds_up16((size_t)cap * lam);
  o.scell = o.hs + lds_up16((size_t)(2 * lmaxh + 1) * sizeof(int));
  o.end = o.scell + lds_up16((size_t)cap * sizeof(unsigned short));
  return o;
}

// Displacement bound of the pair lists: every force launch that drifts the
// particles folds the largest squared half-step speed of each wave into one of
// kDispSlots words (float bits, atomic maximum; one 128-byte line per word
// so that the waves' updates spread over the memory channels), one row of
// words per MD step since the lists were built.
constexpr int kDispSlots = 64;
constexpr int kDispStride = 32;      // words between two slots of a row
constexpr int kDispRow = kDispSlots * kDispStride;

// device error word bits
constexpr unsigned kErrMargin = 1u;     // particle left its cell by more than the rebuild margin
constexpr unsigned kErrNonFinite = 2u;  // non-finite position or velocity
constexpr unsigned kErrJump = 4u;       // moved more than one cell between rebuilds / bad input
constexpr unsigned kErrImage = 8u;      // image counter or unwrapped cell out of range
constexpr unsigned kErrOverflow = 16u;  // more particles in one cell than a slot can index
constexpr unsigned kErrRecord = 64u;    // a pair-list target record names no particle (internal)

// pair lists: halo-local indices of 16 bits, four per 64-bit word; at most
// 63 words per list (the builder orders a brick's targets by word count in 64
// bins); the staging map packs a halo cell's coordinates in 8 bits per axis
constexpr int kMaxPairSlots = 252;
constexpr int kMaxListHalo = 255;    // halo cells per axis a packed coordinate can hold

// force-kernel modes (what the velocity buffer holds on entry)
enum StepMode : int {
  kModeStep = 0,    // v(t - dt/2): complete the kick, kick again, drift
  kModeStart = 1,   // v(t): kick, drift
  kModeFinish = 2,  // v(t - dt/2): complete the kick only, store v(t)
  kModeProbe = 3    // v(t): forces only (for readout of accelerations)
};

struct Replica {
  int Mc[3];     // MD cells per axis
  unsigned dmul[2];  // exact division by Mc[0] and Mc[1] (div_magic)
  int dsh[2];
  int M[3];      // lattice sites per axis
  int cell_off;  // first global MD cell
  int part_off;  // first global particle
  int site_off;  // first global lattice site
  int n;         // particles
  int brick_off; // first force brick
  int nbricks;   // force bricks
  int chunk_off; // first particle chunk
  int nchunks;   // particle chunks
};

// Exact quotient n / d for 0 <= n < 2^31 and a divisor d >= 2 given as the
// multiplier m = ceil(2^(31 + s0) / d) and shift s = s0 - 1, s0 = ceil(log2 d):
// n m / 2^(31 + s0) exceeds n / d by less than n / 2^(31 + s0) < 1 / d, too
// little to reach the next integer, so the floor is exact.
__host__ __device__ inline void div_magic_of(int d, unsigned* m, int* s) {
  int s0 = 0;
  while ((1ll << s0) < d) ++s0;
  const unsigned long long num = 1ull << (31 + s0);
  *m = (unsigned)((num + (unsigned long long)d - 1) / (unsigned long long)d);
  *s = s0 - 1;
}
__device__ __forceinline__ int div_magic(int n, unsigned m, int s) {
  return (int)(__umulhi((unsigned)n, m) >> s);
}

// Global physical and layout parameters (identical for all replicas).
struct Phys {
  float s;          // MD cell side
  float inv_s;
  int F;            // fixed-point bits per MD cell in the force kernel (unit u = s / 2^F)
  float fscale;     // 2^F / s
  int rcq;          // (r_cut + margin) / u, rounded up
  float rc2_u;      // (r_cut / u)^2
  int mq;           // rebuild margin / u, rounded up, plus a few units
  int rlq;          // pair-list radius (r_cut + 2 margin) / u, rounded up
  float rl2_u;      // (pair-list radius / u)^2, widened against rounding
  int sh16;         // list builder: 14-bit coordinate = (fixed + 2 cells) >> sh16
  int rl16;         // list builder: accept a candidate when |d|^2 < rl16 in 14-bit units
  int nl_wide;      // list builder: test 32 candidates per step (long rows) instead of 16
  int kmax;         // pair-list slots per particle (multiple of 4; 0 = no lists)
  float skin;       // largest displacement allowed since the lists were built
  float vcap2;      // squared speed cap of one drift in the lists' displacement bound
  float dslack;     // rounding of one drift of an offset (half an ulp of s + margin)
  int lmaxh;        // halo cells of the largest brick (dynamic LDS table)
  int lcap;         // staged particles per LDS chunk
  float sig2_u;     // (sigma / u)^2
  float eps24m_u;   // 24 eps / (m u)
  float dt;
  float half_dt;
  float lo;         // -margin
  float hi;         // s + margin
  float mass;
  int ns;           // stencil half-width in cells
  int log2k;        // MD cells per lattice cell = 1 << log2k
  int vmax;
  int Q;
  int nm;           // per-site moments
  int BX, BY, BZ;   // brick extent
  int bthreads;     // threads per block of the force and pair-list kernels (64, 128, 256)
  int forces_off;
  int n_rep;
  int n_total;
  int n_cells;
  int n_sites;
  double s_d;       // MD cell side in double (displacement sums)
  double rc_d;      // r_cut (host bookkeeping)
  double u_d;       // fixed-point unit s / 2^F (host bookkeeping)
};

}  // namespace mdlg
