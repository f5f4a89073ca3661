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
constexpr int kCountChunkMax = 4096; // particles per block of the counting pass (at most)
constexpr int kMaxStripSites = 16;   // lattice sites per block of the binning kernel
constexpr int kMaxQ = 225;           // largest velocity window handled (V <= 7 in 2D, V <= 2 in 3D)
constexpr int kMaxShifts = 32;       // displaced / moving lattices binned beside the main one

// LDS budgets of the force kernel
constexpr int kMaxHalo2 = 1536;      // halo cells per brick (2D)
constexpr int kMaxHalo3 = 2560;      // halo cells per brick (3D)
constexpr int kBrickLdsBytes = 60 * 1024;  // dynamic LDS budget of a brick kernel
constexpr int kMaxRows = 64;         // brick rows (BY * BZ)

// device error word bits
constexpr unsigned kErrMargin = 1u;     // particle left its cell by more than the rebuild margin
constexpr unsigned kErrNonFinite = 2u;  // non-finite position or velocity
constexpr unsigned kErrJump = 4u;       // moved more than one cell between rebuilds / bad input
constexpr unsigned kErrImage = 8u;      // image counter or unwrapped cell out of range
constexpr unsigned kErrOverflow = 16u;  // more particles in one cell than a slot can index
constexpr unsigned kErrSkin = 32u;      // moved farther than the margin since the pair lists were built
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
  int M[3];      // lattice sites per axis
  int cell_off;  // first global MD cell
  int part_off;  // first global particle
  int site_off;  // first global lattice site
  int n;         // particles
  int brick_off; // first force brick
  int nbricks;   // force bricks
};

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
  float disp2;      // largest squared displacement since the lists were built
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
