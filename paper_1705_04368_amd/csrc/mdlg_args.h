// Kernel argument blocks of the MDLG HIP library, shared by the kernels and
// the host-side launch sequence.
#pragma once

#include "mdlg_device.h"

namespace mdlg {

struct IngestArgs {
  Phys P;
  const Replica* reps;
  const int4* chunks;  // {replica, g0, g1, -}
  const float* pos_abs;
  const float* vel_in;
  float* pos;
  float* vel;
  int* img;
  int* id;
  int* cell;
  unsigned* err;
};

struct SortArgs {
  Phys P;
  const Replica* reps;
  const int4* chunks;
  const int4* cchunks;    // the counting pass's chunks (larger)
  const int* cell_start;
  const float* pos;
  const float* vel;
  const int* img;
  const int* id;
  const int* cell;
  int2* keyslot;
  int* count;
  int* tile_sum;
  float* pos_out;
  float* vel_out;
  int* img_out;
  int* id_out;
  int* cell_out;
  const int* prev_u;      // snapshot (sorted order), permuted with the state
  const float* prev_off;
  int* prev_u_out;
  float* prev_off_out;
  unsigned* mcnt;         // [n_cells][mwords] arrivals per cell: total, then a byte per direction
  unsigned* mcnt_clear;   // the other parity's counters, cleared by the scatter
  unsigned* err;
  int mwords;             // words of arrival counters per cell: 3 (2D), 8 (3D)
  int first;              // 1: input in arbitrary order (ingest, import): slots from
                          // atomics, then k_cellsort orders every cell by id
  int ntiles;
  int nchunks;
  int ncchunks;
  int xcd_remap;
};

// First rebuild after ingest or import: the scattered state (src) is copied
// back into the state arrays (dst) with every cell ordered by particle id.
struct CellsortArgs {
  const Replica* reps;
  const int4* chunks;
  const int* cell_start;
  const float* pos_src;
  const float* vel_src;
  const int* img_src;
  const int* id_src;
  const int* cell_src;
  const int* prev_u_src;
  const float* prev_off_src;
  float* pos;
  float* vel;
  int* img;
  int* id;
  int* cell;
  int* prev_u;
  float* prev_off;
};

// Thermostat: velocities of every replica scaled by its factor.
struct RescaleArgs {
  const int4* chunks;
  const float* lambda;
  float* vel;
};

struct ScanArgs {
  int* count;
  int* cell_start;
  int* tile_sum;
  int n;
  int ntiles;
};

struct ForceArgs {
  Phys P;
  const Replica* reps;
  const int4* bricks;  // {replica, bx, by, bz}
  const int* cell_start;
  const float* pos_in;
  float* pos_out;
  float* vel;
  float* acc_out;      // optional
  float* vel_full_out; // optional: the full-step velocities v(t) of this launch's kick
  unsigned* err;
  int mode;
  int nbricks;
  int xcd_remap;
  // pair lists (null nl: every brick walks its cell rows)
  const int2* smap;    // [nbricks][lcap] halo particles the lists may name, in LDS order:
                       // {particle, LDS slot << 16 | halo cell (8 bits per axis in 2D, 5 in 3D)}
  const int4* binfo;   // [nbricks] {halo slots, targets, lists valid, map entries}
  const unsigned long long* nl;  // [kmax / 4][n_total] four 16-bit halo indices per word
  const int2* trec;    // [nbricks][lcap] targets in processing order {particle, slot | words << 16}
  // displacement bound since the lists were built: stale_in set means the
  // lists may miss a pair and every brick walks its cells (counted in
  // fallbacks).  Unless no later launch uses the lists (disp_out null), this
  // launch folds its drift into row disp_out and sets stale_out when the
  // bound over the ndisp completed drifts (the running sum psum[ndisp - 1]
  // plus row ndisp - 1 of disp_in), plus this drift at the speed cap, passes
  // P.skin, or when a speed passes the cap.
  const unsigned* stale_in;
  const unsigned* disp_in;
  int ndisp;
  unsigned* disp_out;
  unsigned* stale_out;
  double* psum;        // running sums of the bound: psum[ndisp] written here, psum[ndisp - 1] read
  unsigned long long* fallbacks;
};

struct NlistArgs {
  Phys P;
  const Replica* reps;
  const int4* bricks;
  const int* cell_start;
  const float* pos;
  int2* smap;
  int4* binfo;
  unsigned long long* nl;
  int2* trec;
  unsigned* disp_clear;  // rows of the displacement bound cleared for the new lists
  int ndisp_clear;
  unsigned* stale_clear;  // their staleness flags, cleared too
  int nbricks;
  int xcd_remap;
};

// FP64 kinetic partials of every particle chunk (sum of m v and of m v^2 / 2
// over the chunk's full-step velocities, in particle order).
struct KinPartArgs {
  const int4* chunks;
  const float* vel;
  double* kpart;   // [nchunks][D + 1]
  double mass;
};
void launch_kinpart(int D, int nchunks, const KinPartArgs& a, hipStream_t s);

struct KinArgs {
  const Replica* reps;
  const double* kpart;  // per-chunk partials (k_kinpart)
  double* kin;     // [n_rep][D + 1]
  float* lambda;   // [n_rep]
  int n_rep;
  int D;
  int thermostat;
  double kT;
  double mass;
};

struct BinArgs {
  Phys P;
  const Replica* reps;
  const int4* strips;  // {replica, sx0, sy, sz}
  const int* cell_start;
  const float* pos;
  const int* img;
  const int* id;
  const int* cell;
  int* prev_u;           // snapshot in the sorted order of the state
  float* prev_off;
  unsigned* A;
  long long* mom;
  double* dpart;       // [nstrips][2D]
  unsigned* err;
  int snapshot_only;
  int BSX;             // sites per strip row
  int BSY;             // site rows per strip
  unsigned* nstep;     // optional: this step's n_i(x,t) [sites][Q], overwritten
  long long* shift_k;  // optional: lattice-time counter of the shifted lattices, advanced here
};

struct ShiftArgs {
  Phys P;
  const Replica* reps;
  const int4* chunks;          // {replica, g0, g1, -}
  const float* pos;            // sorted state at t
  const int* img;
  const int* cell;
  const int* prev_u;           // snapshot at t - Delta t (sorted order)
  const float* prev_off;
  const double* shifts;        // [n_shifts][2][D]: offset a, drift b (lattice units)
  const long long* shift_k;    // lattice time index k of t
  unsigned long long* acc;     // [n_shifts][Q + 1 + D + D(D+1)/2]
  double dx;                   // lattice spacing
  int n_shifts;
  int nchunks;
};

struct XiArgs {
  const Replica* reps;
  const unsigned* ncur;        // n_i(x, t + dt_L) [sites][Q]
  const unsigned* nprev;       // n_i(x, t) [sites][Q]
  long long* xi_site;          // [sites][Q] running sum over t of Xi_i(x, t)
  int* xi_last;                // [sites][Q] Xi_i(x, t) of this step
  unsigned long long* sums;    // [5][Q] sums of Xi, Xi^2, Xi n, n, n^2 (two's complement)
  long long* part;             // [nblocks][5][Q] per-block sums of this step
  int n_sites;
  int sites_per_block;
  int nblocks;
  int n_rep;
  int Q;
  int vmax;
};

struct FsumArgs {
  const unsigned* A;
  const long long* mom;
  unsigned long long* fcount;  // [Q]
  long long* momsum;           // [nm]
  int n_sites;
  int Q;
  int nm;
  int sites_per_block;
};

struct FfinalArgs {
  const unsigned long long* fcount;
  const double* dpart;
  double* f;       // [Q]
  double* disp;    // [2D]
  double denom;    // lattice steps * sites
  int Q;
  int nstrips;
  int nd;          // 2D
};

struct SiteAvgArgs {
  const unsigned* A;
  const long long* mom;
  double* f_site;    // [count][Q] or null
  double* mom_site;  // [count][nm] or null
  long long first;   // first site
  long long count;   // sites in this chunk
  int Q;
  int nm;
  double inv_T;
};

struct XportArgs {
  Phys P;
  const Replica* reps;
  const int4* chunks;
  float* pos;        // sorted state
  float* vel;
  int* img;
  int* id;
  int* cell;
  const float* acc;  // sorted accelerations (export, optional)
  int* x_u;          // id-ordered staging
  float* x_off;
  float* x_vel;
  float* x_acc;      // optional
  int* prev_u;       // snapshot, sorted order
  float* prev_off;
  int* x_pu;         // snapshot, id order (import: null = none)
  float* x_poff;
  unsigned* err;
};

struct AdjArgs {
  Phys P;
  const Replica* reps;
  const int4* bricks;
  const int* cell_start;
  const float* pos;        // positions x_s (sorted order, cells fixed for the window)
  const float* lam_v_in;   // adjoint velocity before this step
  float* lam_v_out;        // adjoint velocity after this step
  float* lam_x;            // adjoint position, updated in place
  double* gpart;           // this reverse step's per-brick partials of (dL/deps, dL/dsigma)
  float c;                 // weight of the two half kicks that use a(x_s): h or h/2
  int drift;               // 1: apply lam_v += h lam_x (not at the first position)
  float e1_over_sigma;     // 24 eps / (m u sigma)
  float e2;                // 24 eps / (m u^2)
  double eps;
  int nbricks;
  unsigned* err;
  // pair lists of the window (null nl: every brick walks its cell rows)
  const int2* smap;    // [nbricks][lcap_list] staged halo of the list builder
  const int4* binfo;
  const int2* trec;    // [nbricks][lcap_list] targets {particle, LDS slot | words << 16}
  const unsigned long long* nl;
  int lcap_list;
  // set when the window's drifts may have made the lists stale: the bricks
  // then walk their cells
  const unsigned* stale;
};

struct AdjLossArgs {
  const float* off0;       // offsets at the start of the window
  const float* offW;       // offsets at its end
  float* lam_x;
  float* lam_v;
  double* lpart;           // per-block partial losses
  int n;
  int loss;                // 0: per-axis MSD, 1: mean x displacement
  int nblocks;
};

struct AdjFinalArgs {
  const double* lpart;
  const double* gpart;
  double* out;             // loss, dL/deps, dL/dsigma
  int nl;
  int nb;                  // partial pairs in gpart (reverse steps x bricks)
};

struct AdjIoArgs {
  const int* id;
  float* sorted;
  float* by_id;
  int n;
  int to_sorted;
};

// Events of the next launch of a timed kernel: when set, the launcher hands
// them to hipExtLaunchKernelGGL, which records them immediately before and
// after the kernel, and clears them.
struct LaunchEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
extern thread_local LaunchEvents g_launch_events;

void launch_fill_u32(unsigned* p, unsigned v, long long n, hipStream_t s);
void launch_clock_wait(long long ticks, hipStream_t s, hipEvent_t start, hipEvent_t stop);
size_t brick_lds_bytes(const Phys& P, int D, bool adj);
void launch_adjoint(int D, const AdjArgs& a, hipStream_t s);
// a reverse step and an independent force step in one launch (both on the
// layout's block size; the force part takes no XCD remapping)
struct AdjForceArgs {
  AdjArgs adj;
  ForceArgs force;
};
void launch_adjoint_force(int D, const AdjForceArgs& a, hipStream_t s);
void launch_adj_loss(int D, const AdjLossArgs& a, hipStream_t s);
void launch_adj_final(const AdjFinalArgs& a, hipStream_t s);
void launch_adj_io(int D, const AdjIoArgs& a, hipStream_t s);
void launch_copy_f32(const float* src, float* dst, long long n, hipStream_t s);
void launch_fill_f32(float* p, float v, long long n, hipStream_t s);
void launch_ingest(int D, int nchunks, const IngestArgs& a, hipStream_t s);
void launch_count(int D, int nchunks, const SortArgs& a, hipStream_t s);
void launch_scan(const ScanArgs& a, hipStream_t s);
void launch_scatter(int D, int nchunks, const SortArgs& a, hipStream_t s);
void launch_cellsort(int D, int nchunks, const CellsortArgs& a, hipStream_t s);
void launch_rescale(int D, int nchunks, const RescaleArgs& a, hipStream_t s);
void launch_force(int D, const ForceArgs& a, hipStream_t s);
void launch_nlist(int D, const NlistArgs& a, hipStream_t s);
void launch_kin(const KinArgs& a, hipStream_t s);
void launch_bin(int D, int nstrips, const BinArgs& a, hipStream_t s);
void launch_xi(int D, const XiArgs& a, hipStream_t s);
void launch_shift(int D, const ShiftArgs& a, hipStream_t s);
void launch_fsum(const FsumArgs& a, hipStream_t s);
void launch_ffinal(const FfinalArgs& a, hipStream_t s);
void launch_site_avg(const SiteAvgArgs& a, hipStream_t s);
void launch_export(int D, int nchunks, const XportArgs& a, hipStream_t s);
void launch_import(int D, int nchunks, const XportArgs& a, hipStream_t s);

}  // namespace mdlg
