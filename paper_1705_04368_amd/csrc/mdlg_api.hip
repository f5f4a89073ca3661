// Host side of the MDLG C ABI (include/mdlg.h): configuration checks, the
// workspace layout, the launch sequence of an MD step and of a lattice step,
// HIP-graph replay of lattice steps, readout and state I/O.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "mdlg.h"
#include "mdlg_args.h"

using namespace mdlg;

namespace {

thread_local std::string g_create_error = "no error";

// The workspace of mdlg_create_static: one array per GPU the library runs on,
// held until the process ends.  Host code never passes `scratch` itself to a
// kernel (in host code it names a host-side stand-in): it takes the device
// address from hipGetSymbolAddress once per device and uses that.
constexpr size_t kStaticWorkspaceBytes = MDLG_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) char scratch[kStaticWorkspaceBytes];

struct StaticSlot {
  void* ptr = nullptr;  // device address of `scratch` on this device
  bool in_use = false;  // a handle created by mdlg_create_static is alive
};
std::mutex g_static_mu;
std::map<int, StaticSlot> g_static;

constexpr int kPartChunk = kPartChunkMax;  // particles per block of the per-particle kernels
// largest mean MD-cell occupancy (at the densest replica) of a layout: the
// counting pass ranks a particle among at most kBlock earlier particles of
// its cell that precede its chunk, and a cell twice as full as the mean
// still fits that window
constexpr int kMaxCellMean = kBlock / 2;
// lattice steps of up to kGraphMaxSteps MD steps replay as one graph; longer
// ones as graphs of about kGraphBlockSteps MD steps (whole rebuild intervals)
constexpr int kGraphMaxSteps = 400;
constexpr int kGraphBlockSteps = 200;
constexpr int kStepGraph = 1 << 30;      // graph kind of a block of plain MD steps
constexpr int kAdjointGraph = (1 << 30) + 1;  // graph kind of an adjoint window

struct Layout {
  mdlg_layout pub;
  int D = 0;
  int k = 1;
  int log2k = 0;
  int ns = 1;
  int Q = 1;
  int nm = 0;
  int BX = 1, BY = 1, BZ = 1;
  int bthreads = 256;
  int BSX = 1;
  int BSY = 1;
  long long n_total = 0, n_cells = 0, n_sites = 0;
  int nbricks = 0, nchunks = 0, ncchunks = 0, nstrips = 0, ntiles = 0;
  std::vector<Replica> reps;
  std::vector<int4> bricks, chunks, cchunks, strips;
  double s = 0, margin = 0, margin_max = 0;
  double vfast = 0;  // design speed of the rebuild margin (8 (kT/m)^(1/2))
  double skin = 0;     // pair-list skin: lists of radius r_cut + 2 skin
  int sort_every = 1;
  int halo_cells = 0;  // halo cells of the largest force brick
  int lcap = 0;        // staged particles per LDS chunk of a force brick
  int lcap_adj = 0;    // the same for the adjoint (stages the adjoint velocity too)
  double per_cell = 0; // mean particles per MD cell
  int kmax = 0;        // pair-list slots per particle (0 = cell walk every step)
  bool xi = false;     // collision-operator statistics buffers
  int n_shifts = 0;    // displaced / moving lattices
  int adj_ckpts = 0;   // checkpoints the workspace holds (0 = no adjoint)
  int kmax_adj = 0;    // pair-list slots of the adjoint window (radius r_cut + 2 margin_max; 0 = none)
  int adj_seg = 0;     // segment positions the workspace holds
  int adj_window = 0;  // longest adjoint window (MD steps)
};

// Workspace carve-out, in the order buffers are laid out.
struct Carve {
  size_t off = 0;
  template <typename T>
  T* take(char* base, size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

int ilog2_exact(int k) {
  int l = 0;
  while ((1 << l) < k) ++l;
  return (1 << l) == k ? l : -1;
}

bool set_err(std::string* msg, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
bool set_err(std::string* msg, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (msg) *msg = buf;
  return false;
}

// Validate cfg and derive the layout.  Host only.
bool build_layout(const mdlg_config* c, Layout* L, std::string* msg) {
  if (!c) return set_err(msg, "config is NULL");
  if (c->dim != 2 && c->dim != 3) return set_err(msg, "dim must be 2 or 3 (got %d)", c->dim);
  const int D = c->dim;
  if (c->n_replicas < 1) return set_err(msg, "n_replicas must be >= 1");
  if (!c->n_particles || !c->lattice) return set_err(msg, "n_particles and lattice are required");
  if (!(c->lattice_dx > 0) || !std::isfinite(c->lattice_dx)) return set_err(msg, "lattice_dx must be > 0");
  if (!(c->epsilon > 0) || !(c->sigma > 0) || !(c->mass > 0) || !(c->r_cut > 0))
    return set_err(msg, "epsilon, sigma, mass and r_cut must be > 0");
  if (!(c->dt > 0) || !std::isfinite(c->dt)) return set_err(msg, "dt must be > 0");
  if (c->md_steps_per_lattice_step < 1) return set_err(msg, "md_steps_per_lattice_step must be >= 1");
  if (c->vmax < 0 || c->vmax > 7) return set_err(msg, "vmax must be in 0..7");
  if (c->thermostat_every < 0) return set_err(msg, "thermostat_every must be >= 0");
  if (c->thermostat_every > 0 && !(c->kT > 0)) return set_err(msg, "thermostat needs kT > 0");
  if (c->kT < 0 || !std::isfinite(c->kT)) return set_err(msg, "kT must be >= 0");
  if (c->sort_every < 0) return set_err(msg, "sort_every must be >= 0");
  if (c->brick_x < 0 || c->brick_y < 0 || c->brick_z < 0) return set_err(msg, "brick extents must be >= 0");
  if (c->block_threads != 0 && c->block_threads != 64 && c->block_threads != 128 &&
      c->block_threads != 256)
    return set_err(msg, "block_threads must be 0, 64, 128 or 256 (got %d)", c->block_threads);
  if (c->adjoint_window < 0) return set_err(msg, "adjoint_window must be >= 0");
  if (c->n_shifts < 0 || c->n_shifts > kMaxShifts)
    return set_err(msg, "n_shifts must be in 0..%d", kMaxShifts);
  if (c->n_shifts > 0) {
    if (!c->shifts) return set_err(msg, "shifts is NULL");
    for (int i = 0; i < c->n_shifts * 2 * c->dim; ++i)
      if (!std::isfinite(c->shifts[i]) || std::fabs(c->shifts[i]) > 1e6)
        return set_err(msg, "shift values must be finite and below 1e6 lattice spacings");
  }
  if (c->adjoint_window > 0 && (c->adjoint_every < 1 || c->adjoint_every > c->adjoint_window))
    return set_err(msg, "adjoint_every must be in 1..adjoint_window");
  L->D = D;
  int Q = 1;
  for (int a = 0; a < D; ++a) Q *= 2 * c->vmax + 1;
  if (Q > kMaxQ) return set_err(msg, "velocity window too large: Q = %d > %d", Q, kMaxQ);
  L->Q = Q;
  L->nm = 2 + D + D * (D + 1) / 2;
  long long n_total = 0;
  int min_m = 1 << 30;
  double vol = 0, rho_max = 0;
  for (int r = 0; r < c->n_replicas; ++r) {
    if (c->n_particles[r] < 1) return set_err(msg, "replica %d has no particles", r);
    n_total += c->n_particles[r];
    long long ns = 1;
    double v = 1;
    for (int a = 0; a < D; ++a) {
      const int m = c->lattice[r * D + a];
      if (m < 1) return set_err(msg, "replica %d: lattice sites per axis must be >= 1", r);
      if (m * c->lattice_dx <= 2 * c->r_cut)
        return set_err(msg, "replica %d: box side %g must exceed 2 r_cut = %g", r,
                       m * c->lattice_dx, 2 * c->r_cut);
      min_m = std::min(min_m, m);
      ns *= m;
      v *= m * c->lattice_dx;
    }
    (void)ns;
    vol += v;
    rho_max = std::max(rho_max, c->n_particles[r] / v);
  }
  if (n_total > (1ll << 30)) return set_err(msg, "too many particles (%lld)", n_total);
  const double rho = n_total / vol;
  // MD cell split k: the cell side s = dx / k
  int k = c->md_cell_split;
  auto margin_of = [&](int kk, int* ns_out) {
    const double s = c->lattice_dx / kk;
    const int ns = (int)std::ceil(c->r_cut / s - 1e-12);
    if (ns_out) *ns_out = ns;
    return (ns * s - c->r_cut) / 2;
  };
  const bool want_list = !c->no_pair_list && !c->forces_off;
  if (k == 0 && want_list) {
    // with pair lists the MD step stages the brick halo and walks the lists;
    // the cell walk runs only at rebuilds.  Measured best on 4 sigma
    // lattices: the smallest cells that keep a one-cell stencil (r_cut +
    // sigma) in 2D, and a two-cell stencil ((r_cut + sigma) / 2) in 3D, where
    // a one-cell stencil would walk ~1000 candidates per particle at each
    // rebuild; coarser lattices split further (up to 8 cells per side)
    const double smin = (D == 2) ? (c->r_cut + c->sigma) : 0.5 * (c->r_cut + c->sigma);
    int kk = 1;
    while (kk < 8 && c->lattice_dx / (2 * kk) >= smin) kk *= 2;
    int ns_k;
    const double m = margin_of(kk, &ns_k);
    if (m >= 0.5 * c->sigma && min_m * kk >= 2 * ns_k + 1) k = kk;
  }
  if (k == 0) {
    // fewest candidates per target: the force kernel visits the cells that
    // overlap a cube of side 2 (r_cut + margin) around each target, i.e.
    // about (2 (r_cut + m) + s)^D rho candidates in (2 (r_cut + m) / s + 1)^(D-1)
    // contiguous rows; a row costs about eight candidates of loop overhead.
    // Splits whose rebuild margin is below sigma / 2 are skipped (the cell
    // list would be rebuilt every few steps).
    double best = 1e300;
    for (int kk = 1; kk <= 8; kk *= 2) {
      int ns;
      const double m = margin_of(kk, &ns);
      if (m < 0.5 * c->sigma) continue;
      if (min_m * kk < 2 * ns + 1) continue;
      const double s = c->lattice_dx / kk;
      const double reach = 2 * (c->r_cut + m);
      const double cost = std::pow(reach + s, D) * rho + 8.0 * std::pow(reach / s + 1, D - 1);
      if (cost < best) {
        best = cost;
        k = kk;
      }
    }
    if (k == 0) k = 1;
  }
  const int lk = ilog2_exact(k);
  if (lk < 0 || k > 8) return set_err(msg, "md_cell_split must be a power of two in 1..8 (got %d)", k);
  if (D == 3 && k * k > 64) return set_err(msg, "md_cell_split too large for 3D");
  L->k = k;
  L->log2k = lk;
  // the float32 cell side is the one definition of the MD cell (kernels
  // canonicalise offsets with it); the box side is Mc * s
  L->s = (double)(float)(c->lattice_dx / k);
  L->ns = (int)std::ceil(c->r_cut / L->s - 1e-12);
  if (L->ns > 7)
    return set_err(msg, "MD cells of side %g are too small for r_cut %g (stencil half-width %d > 7)",
                   L->s, c->r_cut, L->ns);
  // the counting sort ranks within a bounded window of each cell's particles
  const double occ = rho_max * std::pow(L->s, D);
  if (occ > kMaxCellMean)
    return set_err(msg,
                   "MD cells of side %g hold %.0f particles on average (densest replica), more than "
                   "the %d the counting sort supports: raise md_cell_split",
                   L->s, occ, kMaxCellMean);
  // largest excursion outside the cell that the stencil still covers
  const double m_max = (L->ns * L->s - c->r_cut) / 2;
  if (min_m * k < 2 * L->ns + 1)
    return set_err(msg, "too few MD cells per axis (%d) for the stencil half-width %d", min_m * k, L->ns);
  // rebuild interval and the margin it needs: eight standard deviations of
  // the Maxwell speed per axis times the interval.  The margin is a design
  // figure: the cell walk stays exact up to the stencil's reach m_max, and
  // only a particle beyond that is an error
  const double vfast = c->kT > 0 ? 8.0 * std::sqrt(c->kT / c->mass) : 0.0;

  // with pair lists the margin also widens every list (radius r_cut + 2 m),
  // so the automatic interval aims at m <= 0.16 r_cut instead of the largest
  // margin the stencil allows
  int R = c->sort_every;
  if (R == 0) {
    if (m_max <= 0 || !(vfast > 0)) {
      R = 1;
    } else {
      const double m_aim = want_list ? std::min(m_max, 0.16 * c->r_cut) : m_max;
      R = (int)std::floor(m_aim / (vfast * c->dt));
      R = std::max(want_list ? 2 : 1, std::min(R, c->md_steps_per_lattice_step));
      // as few rebuilds per lattice step as that allows, evenly spaced
      const int steps = c->md_steps_per_lattice_step;
      const int nreb = (steps + R - 1) / R;
      R = (steps + nreb - 1) / nreb;
      if (R * vfast * c->dt > m_max) R = std::max(1, (int)std::floor(m_max / (vfast * c->dt)));
    }
  }
  if (R > 1 && m_max <= 0)
    return set_err(msg, "sort_every > 1 needs a positive margin (stencil reach %g vs r_cut %g)",
                   L->ns * L->s, c->r_cut);
  L->sort_every = R;
  L->margin_max = m_max;
  L->vfast = vfast;
  L->margin = (vfast > 0) ? std::min(m_max, R * vfast * c->dt) : m_max;
  if (L->margin < 0) L->margin = 0;
  // the pair lists' skin: R drifts at a speed that the fastest of the
  // n_total particles passes only rarely (a Maxwell tail of about e^-5 per
  // step: v^2 = (kT/m) (2 ln n + 10) in 2D, + 14 in 3D for the extra degree
  // of freedom), at most the margin.  The force kernel bounds the actual
  // drifts since the build; past the skin the bricks walk their cells (exact
  // within the stencil's reach) until the next rebuild.
  L->skin = L->margin;
  if (vfast > 0) {
    const double vs = std::min(8.0, std::sqrt(2.0 * std::log((double)std::max(2ll, n_total)) +
                                              (D == 3 ? 14.0 : 10.0))) *
                      std::sqrt(c->kT / c->mass);
    L->skin = std::min(L->margin, R * vs * c->dt);
  }
  // a particle then sits less than one cell outside its own (the pair-list
  // builder's coordinate range relies on it)
  if (L->margin >= L->s) return set_err(msg, "rebuild margin %g reaches the cell side %g", L->margin, L->s);
  // force bricks
  int BX = c->brick_x, BY = c->brick_y, BZ = c->brick_z;
  const double per_cell = rho * std::pow(L->s, D);
  // threads per force block (the autotuner also tries 64 and 128)
  int NT = c->block_threads;
  if (NT == 0) NT = 256;
  L->bthreads = NT;
  if (D == 2) {
    // targets per block: about one per thread in bricks of four rows with
    // pair lists, half a thread's worth in two rows for the cell walk
    // (measured best on the 2D workloads)
    const double cells = (want_list ? 1.0 * NT : 0.5 * NT) / std::max(per_cell, 0.05);
    if (BY == 0) BY = want_list ? (cells >= 32 ? 4 : (cells >= 16 ? 2 : 1)) : (cells >= 32 ? 2 : 1);
    if (BX == 0) BX = std::max(4, std::min(128, (int)std::lround(cells / BY)));
    BZ = 1;
  } else if (want_list) {
    // about 3/4 target per thread in a compact brick, which keeps the halo
    // (staged in LDS) small enough for several blocks per CU
    const double cells = 0.75 * NT / std::max(per_cell, 0.05);
    if (BZ == 0) BZ = cells >= 27 ? 3 : (cells >= 8 ? 2 : 1);
    const int side = std::max(1, (int)std::lround(std::sqrt(cells / BZ)));
    if (BX == 0) BX = std::min(16, side);
    if (BY == 0) BY = std::min(16, std::max(1, (int)std::lround(cells / (BZ * BX))));
  } else {
    if (BX == 0 || BY == 0) {
      const double cells = 256.0 / std::max(per_cell, 0.05);
      int bx = 1;
      while (bx * bx * 2 <= cells && bx < 16) bx *= 2;
      if (BX == 0) BX = bx;
      if (BY == 0) BY = std::max(1, (int)std::lround(cells / BX));
      BY = std::min(BY, 16);
    }
    if (BZ == 0) BZ = 1;
  }
  const int nsz = (D == 3) ? L->ns : 0;
  const int maxh = (D == 2) ? kMaxHalo2 : kMaxHalo3;
  auto halo_of = [&](int bx, int by, int bz) {
    return (long long)(bx + 2 * L->ns) * (by + 2 * L->ns) * (bz + 2 * nsz);
  };
  // automatic extents shrink until the halo fits the LDS cell table
  while (c->brick_x == 0 && BX > 1 && halo_of(BX, BY, BZ) > maxh) BX = (BX + 1) / 2;
  while (c->brick_y == 0 && BY > 1 && halo_of(BX, BY, BZ) > maxh) BY = (BY + 1) / 2;
  const long long halo = halo_of(BX, BY, BZ);
  L->halo_cells = (int)halo;
  L->per_cell = per_cell;
  {
    // dynamic LDS of the brick kernels: the halo cell table of the largest
    // brick and room for about 1.5x the expected halo particles (a fuller
    // halo is staged in several chunks); the adjoint also stages d floats each
    // (the force and list kernels size it at 1.25x + 64 so that more blocks
    // fit a CU: the count of a halo of hundreds of cells rarely strays more
    // than a few percent from its mean, and a brick that overflows takes the
    // chunked cell walk)
    const double expect = halo * per_cell;
    // (the halo tables, and 16-byte alignment of each part of the layout)
    const size_t head = ((size_t)(2 * halo + 1) * sizeof(int) + 15) / 16 * 16 + 64;
    // a staged particle: its coordinates and its halo cell (16 bits)
    const size_t coord = (D == 2 ? sizeof(int2) : sizeof(int4)) + sizeof(unsigned short);
    auto fit = [&](double grow, long long extra, size_t per) {
      long long cap = (long long)std::ceil(grow * expect) + extra;
      cap = (cap + 63) / 64 * 64;
      const long long f = (long long)((kBrickLdsBytes - head) / per) / 64 * 64;
      return (int)std::max<long long>(64, std::min(cap, f));
    };
    L->lcap = fit(1.25, 64, coord);
    L->lcap_adj = fit(1.5, 128, coord + D * sizeof(float));
  }
  if (halo > maxh) return set_err(msg, "brick %dx%dx%d with stencil %d needs %lld halo cells > %d",
                                  BX, BY, BZ, L->ns, halo, maxh);
  if ((long long)BY * BZ > kMaxRows) return set_err(msg, "brick has more than %d rows", kMaxRows);
  // the staging map of the pair lists packs a halo cell in 8 bits per axis
  // in 2D and in 5 in 3D
  const int hlim = (D == 2) ? 256 : 32;
  if (BX + 2 * L->ns > hlim || BY + 2 * L->ns > hlim || BZ + 2 * nsz > hlim)
    return set_err(msg, "brick %dx%dx%d with stencil %d has a halo wider than %d cells", BX, BY, BZ,
                   L->ns, hlim);
  L->BX = BX;
  L->BY = BY;
  L->BZ = BZ;
  // pair lists: radius r_cut + 2 skin; slots for 1.5x the neighbours
  // expected at the densest replica's mean density plus 20 (a brick with a
  // fuller list walks its cells instead)
  L->kmax = 0;
  // (list entries are 16-bit staging indices: lcap < 2^16)
  if (want_list && R >= 2 && L->lcap < 65536 && BX + 2 * L->ns <= kMaxListHalo &&
      BY + 2 * L->ns <= kMaxListHalo && BZ + 2 * nsz <= kMaxListHalo) {
    const double rl = c->r_cut + 2 * L->skin;
    const double vol_l = (D == 2) ? M_PI * rl * rl : 4.0 / 3.0 * M_PI * rl * rl * rl;
    const int want = (int)std::ceil(1.5 * vol_l * rho_max) + 20;
    L->kmax = std::min(kMaxPairSlots, (want + 3) / 4 * 4);
  }
  // binning strips: BSX sites along x (LDS budget 60 kB) times BSY site rows,
  // about 512 particles per block (two per thread), at most 64 MD-cell rows
  L->BSX = std::max(1, std::min(kMaxStripSites, 60000 / ((L->Q + L->nm) * 4)));
  {
    const int rows_per = (D == 2) ? L->k : L->k * L->k;
    const double per_site = rho * std::pow(c->lattice_dx, D);
    int bsy = (int)std::lround(512.0 / std::max(1.0, L->BSX * per_site));
    bsy = std::min(bsy, 64 / rows_per);
    bsy = std::min(bsy, 60000 / (L->BSX * (L->Q + L->nm) * 4));
    L->BSY = std::max(1, bsy);
  }
  // tables
  L->reps.clear();
  L->bricks.clear();
  L->chunks.clear();
  L->cchunks.clear();
  L->strips.clear();
  // the counting pass takes larger chunks on large systems (about 1024
  // blocks): its per-block chain of dependent memory operations then serves
  // more particles
  int cchunk = (int)std::min<long long>(kCountChunkMax, (n_total / 1024 + kBlock - 1) / kBlock * kBlock);
  cchunk = std::max(cchunk, kPartChunk);
  long long cell_off = 0, part_off = 0, site_off = 0;
  for (int r = 0; r < c->n_replicas; ++r) {
    Replica rep{};
    long long ncell = 1, nsite = 1;
    for (int a = 0; a < 3; ++a) {
      rep.M[a] = a < D ? c->lattice[r * D + a] : 1;
      rep.Mc[a] = a < D ? rep.M[a] * k : 1;
      ncell *= rep.Mc[a];
      nsite *= rep.M[a];
    }
    if (cell_off + ncell > (1ll << 30)) return set_err(msg, "too many MD cells");
    // (a replica has at least three MD cells per axis, checked above)
    for (int a = 0; a < 2; ++a) div_magic_of(std::max(2, rep.Mc[a]), &rep.dmul[a], &rep.dsh[a]);
    rep.cell_off = (int)cell_off;
    rep.part_off = (int)part_off;
    rep.site_off = (int)site_off;
    rep.n = c->n_particles[r];
    rep.brick_off = (int)L->bricks.size();
    const int nbx = (rep.Mc[0] + BX - 1) / BX, nby = (rep.Mc[1] + BY - 1) / BY;
    const int nbz = (D == 3) ? (rep.Mc[2] + BZ - 1) / BZ : 1;
    for (int bz = 0; bz < nbz; ++bz)
      for (int by = 0; by < nby; ++by)
        for (int bx = 0; bx < nbx; ++bx) L->bricks.push_back(make_int4(r, bx, by, bz));
    rep.nbricks = (int)L->bricks.size() - rep.brick_off;
    rep.chunk_off = (int)L->chunks.size();
    for (long long g = part_off; g < part_off + rep.n; g += kPartChunk)
      L->chunks.push_back(make_int4(r, (int)g, (int)std::min(part_off + rep.n, g + kPartChunk), 0));
    rep.nchunks = (int)L->chunks.size() - rep.chunk_off;
    for (long long g = part_off; g < part_off + rep.n; g += cchunk)
      L->cchunks.push_back(make_int4(r, (int)g, (int)std::min(part_off + rep.n, g + cchunk), 0));
    const int nsz_rows = (D == 3) ? rep.M[2] : 1;
    for (int sz = 0; sz < nsz_rows; ++sz)
      for (int sy = 0; sy < rep.M[1]; sy += L->BSY)
        for (int sx = 0; sx < rep.M[0]; sx += L->BSX) L->strips.push_back(make_int4(r, sx, sy, sz));
    L->reps.push_back(rep);
    cell_off += ncell;
    part_off += rep.n;
    site_off += nsite;
  }
  L->xi = c->collision_stats != 0;
  L->n_shifts = c->n_shifts;
  if (c->adjoint_window > 0) {
    L->adj_ckpts = c->adjoint_window / c->adjoint_every + 1;
    L->adj_window = c->adjoint_window;
    L->adj_seg = c->adjoint_every + 1;
    // the window's force launches walk pair lists of radius r_cut + 2
    // margin_max, built once at its start (cells stay frozen for the window,
    // so no particle moves farther than margin_max from its build position)
    if (want_list && L->lcap < 65536 && L->margin_max > 0) {
      const double rl = c->r_cut + 2 * L->margin_max;
      const double vol_l = (D == 2) ? M_PI * rl * rl : 4.0 / 3.0 * M_PI * rl * rl * rl;
      const int want = (int)std::ceil(1.5 * vol_l * rho_max) + 20;
      L->kmax_adj = std::min(kMaxPairSlots, (want + 3) / 4 * 4);
    }
  }
  L->n_total = n_total;
  L->n_cells = cell_off;
  L->n_sites = site_off;
  L->nbricks = (int)L->bricks.size();
  L->nchunks = (int)L->chunks.size();
  L->ncchunks = (int)L->cchunks.size();
  L->nstrips = (int)L->strips.size();
  L->ntiles = (int)((L->n_cells + kScanTile - 1) / kScanTile);
  mdlg_layout& P = L->pub;
  P.md_cell_split = k;
  P.sort_every = R;
  P.stencil = L->ns;
  P.n_velocities = Q;
  P.n_moments = L->nm;
  P.brick[0] = BX;
  P.brick[1] = BY;
  P.brick[2] = BZ;
  P.n_total = n_total;
  P.n_sites = L->n_sites;
  P.n_cells = L->n_cells;
  P.n_bricks = L->nbricks;
  P.cell_side = L->s;
  P.margin = L->margin;
  P.reach = L->margin_max;
  P.skin = L->skin;
  P.pair_slots = L->kmax;
  P.block_threads = L->bthreads;
  return true;
}

}  // namespace

// ---------------------------------------------------------------- the handle

struct mdlg_system {
  mdlg_config cfg{};
  std::vector<int32_t> n_particles, lattice;
  Layout L;
  Phys P{};
  hipStream_t stream = nullptr;
  int D = 2;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // device buffers
  float* pos[2] = {nullptr, nullptr};
  float* vel[2] = {nullptr, nullptr};
  int* img[2] = {nullptr, nullptr};
  int* id[2] = {nullptr, nullptr};
  int* cell[2] = {nullptr, nullptr};
  int2* keyslot = nullptr;
  int* count = nullptr;
  int* cell_start = nullptr;
  int* tile_sum = nullptr;
  unsigned* mcnt[2] = {nullptr, nullptr};  // arrivals per cell and direction (parity mpar)
  int* prev_u[2] = {nullptr, nullptr};    // snapshot, sorted order (set parity)
  float* prev_off[2] = {nullptr, nullptr};
  unsigned* A = nullptr;
  long long* mom = nullptr;
  double* dpart = nullptr;
  double* kpart = nullptr;
  double* kin = nullptr;
  float* lambda = nullptr;
  unsigned* err = nullptr;
  Replica* reps = nullptr;
  int4* bricks = nullptr;
  int4* chunks = nullptr;
  int4* cchunks = nullptr;
  int4* strips = nullptr;
  unsigned long long* fcount = nullptr;
  long long* momsum = nullptr;
  double* fout = nullptr;
  double* dispout = nullptr;
  float* acc_sorted = nullptr;
  // displaced / moving lattices
  std::vector<double> shifts_host;
  double* shifts = nullptr;
  long long* shift_k = nullptr;
  unsigned long long* shift_acc = nullptr;
  // collision operator (eq. Xi)
  unsigned* nstep[2] = {nullptr, nullptr};
  long long* xi_site = nullptr;
  int* xi_last = nullptr;
  unsigned long long* xi_sums = nullptr;
  long long* xi_part = nullptr;
  int xi_par = 0;         // nstep[xi_par] receives the next lattice step
  bool xi_have = false;   // nstep[xi_par ^ 1] holds the previous lattice step
  long long xi_steps = 0;
  // pair lists
  int2* smap = nullptr;
  int4* binfo = nullptr;
  unsigned long long* nl = nullptr;
  unsigned* disp = nullptr;  // displacement bound rows [disp_rows][kDispRow]
  double* psum = nullptr;    // its running sums [disp_rows]
  unsigned long long* fallbacks = nullptr;  // force launches that walked cells for stale lists
  unsigned* stale = nullptr;  // [disp_rows] lists possibly stale after that many drifts
  int2* trec = nullptr;
  // adjoint window buffers (sorted order)
  float* adj_ckpt_pos = nullptr;
  float* adj_ckpt_vel = nullptr;
  float* adj_seg_pos = nullptr;
  float* adj_seg_pos2 = nullptr;  // second segment buffer (recomputation beside the sweep)
  float* adj_lx = nullptr;
  float* adj_lv[2] = {nullptr, nullptr};
  double* adj_gpart = nullptr;
  double* adj_lpart = nullptr;
  double* adj_out = nullptr;
  char* staging = nullptr;
  size_t staging_bytes = 0;
  // host-side state
  int pcur = 0, scur = 0;
  bool vel_full = true;
  int since_sort = 0;
  int adj_window_steps = 0;  // MD steps of the adjoint window in progress
  long long md_step = 0;
  long long n_lattice = 0;
  bool snapshot_valid = false;
  int mpar = 0;              // parity of the arrival counters the next rebuild uses
  bool first_sort = false;   // the state arrays hold an input in arbitrary order
  int xcd_remap = 1;
  int static_dev = -1;  // device whose static workspace this handle holds (-1: none)
  bool use_graph = true;
  hipStream_t cap_stream = nullptr;
  // host-side sequencing state a captured graph starts from and leaves
  struct SeqState {
    int pcur, scur, since_sort;
    bool vel_full;
    int mpar;
    int xi_par;
    bool xi_have;
    long long md_step, n_lattice, xi_steps;
  };
  struct GraphEntry {
    hipGraphExec_t exec;
    SeqState after;  // counters as advanced by one replay from the key's state
  };
  // key: (kind, pcur, scur, since_sort, vel_full, mpar, xi_par, xi_have, tag);
  // kind 0 = a whole lattice step, B > 0 = a block of B MD steps, -n = the
  // last n MD steps of a lattice step with its binning, kStepGraph = a block
  // of plain MD steps and kAdjointGraph = an adjoint window (their tags
  // carry the rest of what the work depends on)
  std::map<std::tuple<int, int, int, int, bool, int, int, bool, unsigned long long>, GraphEntry> graphs;
  // per-kernel event timing (measurement aid)
  bool timing = false;
  struct Timed {
    int cls;
    int launches;
    hipEvent_t a, b;
  };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> event_pool;
  double timed_ms[MDLG_K_NCLASS] = {};
  int64_t timed_n[MDLG_K_NCLASS] = {};
  std::string last_error = "no error";
};

namespace {

// Words of arrival counters per MD cell: the number of arrivals, then one
// byte for each of the 3^d - 1 directions a rebuild can move a particle in.
int arrival_words(int D) { return D == 2 ? 3 : 8; }

// Rows of the displacement bound: one per MD step of the longest stretch
// that uses one set of pair lists (a rebuild interval, or an adjoint window).
int disp_rows(const Layout& L) { return std::max(L.sort_every, L.adj_window) + 1; }

// Accumulators per displaced lattice: Q + 1 counts and d + d(d+1)/2 sums.
int shift_per(const Layout& L) { return L.Q + 1 + L.D + L.D * (L.D + 1) / 2; }

// Sites per block of the collision-operator kernel, and its block count.
constexpr int kXiSites = 64;
int xi_blocks(const Layout& L) { return (int)((L.n_sites + kXiSites - 1) / kXiSites); }

size_t carve(mdlg_system* S, char* base) {
  const Layout& L = S->L;
  const int D = L.D;
  const size_t N = (size_t)L.n_total;
  Carve c;
  for (int i = 0; i < 2; ++i) {
    S->pos[i] = c.take<float>(base, N * D);
    S->vel[i] = c.take<float>(base, N * D);
    S->img[i] = c.take<int>(base, N * D);
    S->id[i] = c.take<int>(base, N);
    S->cell[i] = c.take<int>(base, N);
  }
  S->keyslot = c.take<int2>(base, N);
  S->count = c.take<int>(base, (size_t)L.n_cells);
  S->cell_start = c.take<int>(base, (size_t)L.n_cells + 1);
  S->tile_sum = c.take<int>(base, (size_t)L.ntiles * kTileCopies);
  for (int i = 0; i < 2; ++i) S->mcnt[i] = c.take<unsigned>(base, (size_t)L.n_cells * arrival_words(L.D));
  for (int i = 0; i < 2; ++i) {
    S->prev_u[i] = c.take<int>(base, N * D);
    S->prev_off[i] = c.take<float>(base, N * D);
  }
  S->A = c.take<unsigned>(base, (size_t)L.n_sites * L.Q);
  S->mom = c.take<long long>(base, (size_t)L.n_sites * L.nm);
  S->dpart = c.take<double>(base, (size_t)L.nstrips * 2 * D);
  S->kpart = c.take<double>(base, (size_t)L.nchunks * (D + 1));
  S->kin = c.take<double>(base, L.reps.size() * (D + 1));
  S->lambda = c.take<float>(base, L.reps.size());
  S->err = c.take<unsigned>(base, 64);
  S->reps = c.take<Replica>(base, L.reps.size());
  S->bricks = c.take<int4>(base, L.bricks.size());
  S->chunks = c.take<int4>(base, L.chunks.size());
  S->cchunks = c.take<int4>(base, L.cchunks.size());
  S->strips = c.take<int4>(base, L.strips.size());
  S->fcount = c.take<unsigned long long>(base, kMaxQ);
  S->momsum = c.take<long long>(base, 16);
  S->fout = c.take<double>(base, kMaxQ);
  S->dispout = c.take<double>(base, 8);
  S->acc_sorted = c.take<float>(base, N * D);
  if (L.n_shifts > 0) {
    S->shifts = c.take<double>(base, (size_t)L.n_shifts * 2 * D);
    S->shift_k = c.take<long long>(base, 1);
    S->shift_acc = c.take<unsigned long long>(base, (size_t)L.n_shifts * shift_per(L) * kTileCopies);
  }
  if (L.xi) {
    const size_t sq = (size_t)L.n_sites * L.Q;
    S->nstep[0] = c.take<unsigned>(base, sq);
    S->nstep[1] = c.take<unsigned>(base, sq);
    S->xi_site = c.take<long long>(base, sq);
    S->xi_last = c.take<int>(base, sq);
    S->xi_sums = c.take<unsigned long long>(base, (size_t)5 * L.Q);
    S->xi_part = c.take<long long>(base, (size_t)xi_blocks(L) * 5 * L.Q);
  }
  if (L.kmax > 0 || L.kmax_adj > 0) {
    S->smap = c.take<int2>(base, (size_t)L.nbricks * L.lcap);
    S->binfo = c.take<int4>(base, (size_t)L.nbricks);
    S->nl = c.take<unsigned long long>(base, (size_t)(std::max(L.kmax, L.kmax_adj) / 4) * N);
    S->disp = c.take<unsigned>(base, (size_t)disp_rows(L) * kDispRow);
    S->psum = c.take<double>(base, (size_t)disp_rows(L));
    S->fallbacks = c.take<unsigned long long>(base, 1);
    S->stale = c.take<unsigned>(base, (size_t)disp_rows(L));
    S->trec = c.take<int2>(base, (size_t)L.nbricks * L.lcap);
  }
  if (L.adj_ckpts > 0) {
    S->adj_ckpt_pos = c.take<float>(base, N * D * L.adj_ckpts);
    S->adj_ckpt_vel = c.take<float>(base, N * D * L.adj_ckpts);
    S->adj_seg_pos = c.take<float>(base, N * D * L.adj_seg);
    S->adj_seg_pos2 = c.take<float>(base, N * D * L.adj_seg);
    S->adj_lx = c.take<float>(base, N * D);
    S->adj_lv[0] = c.take<float>(base, N * D);
    S->adj_lv[1] = c.take<float>(base, N * D);
    // per-brick parameter partials of every reverse step of the longest window
    S->adj_gpart = c.take<double>(base, (size_t)(L.adj_window + 1) * L.nbricks * 2);
    S->adj_lpart = c.take<double>(base, 1024);
    S->adj_out = c.take<double>(base, 4);
  }
  S->staging_bytes = std::max<size_t>(N * D * 4 * 6, size_t(4) << 20);
  S->staging = c.take<char>(base, S->staging_bytes);
  return c.off + 256;
}

// Pair-list parameters of P for lists of radius r_cut + 2 margin with kmax
// slots (u, F and the brick extents already set).
static void set_list_params(Phys& P, const mdlg_config* c, const Layout& L, double margin, int kmax) {
  const double u = P.u_d;
  const double rl = c->r_cut + 2 * margin;
  P.rlq = (int)std::ceil(rl / u) + 1;
  P.rl2_u = (float)((rl / u) * (rl / u) * (1 + 1e-5));
  // The list builder compares coarser copies of the coordinates: the halo of
  // the widest brick, widened by two cells on either side (a particle sits
  // less than one cell outside its own), in 14-bit units, so that a squared
  // distance over three axes cannot overflow 31 bits.  Each axis of a
  // difference is off by less than one unit, so its length by less than
  // sqrt(D) units: the threshold widened by that keeps every pair within
  // the list radius (a few pairs just beyond it enter the list too).
  const int hx16 = std::max(std::max(L.BX, L.BY), L.D == 3 ? L.BZ : 1) + 2 * L.ns + 4;
  int lg16 = 0;
  while ((1 << lg16) < hx16) ++lg16;
  P.sh16 = std::max(0, P.F - (14 - lg16));
  const double r16 = rl / (u * std::ldexp(1.0, P.sh16)) + std::sqrt((double)L.D);
  P.rl16 = (int)std::ceil(r16 * r16) + 1;
  // candidates of the row through the target: its reach plus one cell
  const double row = (2 * rl + L.s) * std::pow(L.s, L.D - 1) * L.per_cell / std::pow(L.s, L.D);
  P.nl_wide = row >= 48 ? 1 : 0;
  P.kmax = kmax;
  P.skin = (float)margin;
  // speed cap of one drift: the margin's design speed
  const double vcap = L.vfast > 0 ? L.vfast : margin / c->dt;
  P.vcap2 = (float)(vcap * vcap);
  // half an ulp of the largest offset magnitude s + margin: the rounding of
  // one drift of an offset
  int ex = 0;
  std::frexp((double)L.s + margin, &ex);  // s + margin in [2^(ex-1), 2^ex)
  P.dslack = (float)std::ldexp(1.0, ex - 1 - 24);
}

Phys make_phys(const mdlg_config* c, const Layout& L) {
  Phys P{};
  P.s = (float)L.s;
  P.inv_s = (float)(1.0 / L.s);
  // fixed-point frame of the force kernel: coordinates reach at most the
  // widest halo extent plus the cutoff reach, which must stay below 2^31
  // units; at most 26 bits per cell keep pair separations exact in float
  // after the integer difference (|dX| < (2 ns + 1) 2^F < 2^30)
  const int nsz = (L.D == 3) ? L.ns : 0;
  const int hmax = std::max(std::max(L.BX + 2 * L.ns, L.BY + 2 * L.ns), L.BZ + 2 * nsz) + L.ns + 2;
  int lg = 0;
  while ((1 << lg) < hmax) ++lg;
  P.F = std::min(26, 31 - lg);
  const double u = L.s / std::ldexp(1.0, P.F);
  P.fscale = (float)(std::ldexp(1.0, P.F) / L.s);
  // the cell walk prunes with the stencil's full reach, the largest
  // excursion outside its cell that the staged halo still covers, not with
  // the rebuild margin (the design excursion that sets the interval): a
  // particle that outruns the margin between rebuilds is then still exact
  P.rcq = (int)std::ceil((c->r_cut + L.margin_max) / u) + 1;
  P.mq = (int)std::ceil(L.margin_max / u) + 4;
  P.rc_d = c->r_cut;
  P.u_d = u;
  set_list_params(P, c, L, L.skin, L.kmax);
  // dynamic LDS of the brick kernels: the halo cell table of the largest
  // brick and room for about 1.5x the expected halo particles (a fuller halo
  // is staged in several chunks); the adjoint also stages d floats each
  P.lmaxh = L.halo_cells;
  P.lcap = L.lcap;
  P.rc2_u = (float)((c->r_cut / u) * (c->r_cut / u));
  P.sig2_u = (float)((c->sigma / u) * (c->sigma / u));
  P.eps24m_u = (float)(24.0 * c->epsilon / (c->mass * u));
  P.dt = (float)c->dt;
  P.half_dt = (float)(0.5 * c->dt);
  P.lo = (float)(-L.margin_max);
  P.hi = (float)(L.s + L.margin_max);
  P.mass = (float)c->mass;
  P.ns = L.ns;
  P.log2k = L.log2k;
  P.vmax = c->vmax;
  P.Q = L.Q;
  P.nm = L.nm;
  P.BX = L.BX;
  P.BY = L.BY;
  P.BZ = L.BZ;
  P.bthreads = L.bthreads;
  P.forces_off = c->forces_off ? 1 : 0;
  P.n_rep = (int)L.reps.size();
  P.n_total = (int)L.n_total;
  P.n_cells = (int)L.n_cells;
  P.n_sites = (int)L.n_sites;
  P.s_d = L.s;
  return P;
}

mdlg_status hip_fail(mdlg_system* S, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (S) S->last_error = m; else g_create_error = m;
  return MDLG_E_DEVICE;
}

#define HIPCHK(S, expr)                                  \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return hip_fail(S, e_, #expr); \
  } while (0)

mdlg_status check_launch(mdlg_system* S, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(S, e, what);
  return MDLG_OK;
}

// ----- launch sequence

hipEvent_t pool_event(mdlg_system* S) {
  if (!S->event_pool.empty()) {
    hipEvent_t e = S->event_pool.back();
    S->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// With timing on, every launch of a timed class gets its own event pair,
// which hipExtLaunchKernelGGL records around the kernel itself (the time of
// the kernel alone, not of the gaps between launches).  A launcher that ends
// up launching nothing leaves its events unused; they are returned.
void drain_timing(mdlg_system* S);

// pending pairs are read back once this many are in flight (a lattice step of
// many MD steps launches hundreds of thousands of kernels)
constexpr size_t kMaxTimedPending = 16384;

struct TimedLaunch {
  mdlg_system* S;
  bool on = false;
  TimedLaunch(mdlg_system* sys, int cls) : S(sys) {
    if (!S->timing) return;
    if (S->timed.size() >= kMaxTimedPending) drain_timing(S);
    hipEvent_t a = pool_event(S), b = pool_event(S);
    if (!a || !b) return;
    g_launch_events = LaunchEvents{a, b};
    S->timed.push_back({cls, 1, a, b});
    on = true;
  }
  ~TimedLaunch() {
    if (!on || !g_launch_events.start) return;
    g_launch_events = LaunchEvents{};
    const mdlg_system::Timed t = S->timed.back();
    S->timed.pop_back();
    S->event_pool.push_back(t.a);
    S->event_pool.push_back(t.b);
  }
};

void drain_timing(mdlg_system* S) {
  for (auto& t : S->timed) {
    float ms = 0.f;
    if (hipEventSynchronize(t.b) == hipSuccess && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      S->timed_ms[t.cls] += ms;
      S->timed_n[t.cls] += t.launches;
    }
    S->event_pool.push_back(t.a);
    S->event_pool.push_back(t.b);
  }
  S->timed.clear();
}

SortArgs sort_args(mdlg_system* S) {
  SortArgs a{};
  a.P = S->P;
  a.reps = S->reps;
  a.chunks = S->chunks;
  a.cchunks = S->cchunks;
  a.cell_start = S->cell_start;
  a.pos = S->pos[S->pcur];
  a.vel = S->vel[S->scur];
  a.img = S->img[S->scur];
  a.id = S->id[S->scur];
  a.cell = S->cell[S->scur];
  a.keyslot = S->keyslot;
  a.count = S->count;
  a.tile_sum = S->tile_sum;
  a.pos_out = S->pos[S->pcur ^ 1];
  a.vel_out = S->vel[S->scur ^ 1];
  a.img_out = S->img[S->scur ^ 1];
  a.id_out = S->id[S->scur ^ 1];
  a.cell_out = S->cell[S->scur ^ 1];
  a.prev_u = S->prev_u[S->scur];
  a.prev_off = S->prev_off[S->scur];
  a.prev_u_out = S->prev_u[S->scur ^ 1];
  a.prev_off_out = S->prev_off[S->scur ^ 1];
  a.mcnt = S->mcnt[S->mpar];
  a.mcnt_clear = S->mcnt[S->mpar ^ 1];
  a.mwords = arrival_words(S->D);
  a.first = S->first_sort ? 1 : 0;
  a.err = S->err;
  a.ntiles = S->L.ntiles;
  a.nchunks = S->L.nchunks;
  a.ncchunks = S->L.ncchunks;
  a.xcd_remap = S->xcd_remap;
  return a;
}

// Pair lists of the current positions (all inside their cells) with the list
// parameters of P.
void enqueue_nlist(mdlg_system* S, const Phys& P) {
  NlistArgs nl{};
  nl.P = P;
  nl.reps = S->reps;
  nl.bricks = S->bricks;
  nl.cell_start = S->cell_start;
  nl.pos = S->pos[S->pcur];
  nl.smap = S->smap;
  nl.binfo = S->binfo;
  nl.nl = S->nl;
  nl.trec = S->trec;
  nl.disp_clear = S->disp;
  nl.ndisp_clear = disp_rows(S->L);
  nl.stale_clear = S->stale;
  nl.nbricks = S->L.nbricks;
  nl.xcd_remap = S->xcd_remap;
  TimedLaunch t(S, MDLG_K_NLIST);
  launch_nlist(S->D, nl, S->stream);
}

void enqueue_sort(mdlg_system* S) {
  SortArgs a = sort_args(S);
  {
    TimedLaunch t(S, MDLG_K_COUNT);
    launch_count(S->D, S->L.ncchunks, a, S->stream);
  }
  ScanArgs sc{};
  sc.count = S->count;
  sc.cell_start = S->cell_start;
  sc.tile_sum = S->tile_sum;
  sc.n = (int)S->L.n_cells;
  sc.ntiles = S->L.ntiles;
  {
    TimedLaunch t(S, MDLG_K_SCAN);
    launch_scan(sc, S->stream);
  }
  {
    TimedLaunch t(S, MDLG_K_SCATTER);
    launch_scatter(S->D, S->L.nchunks, a, S->stream);
  }
  S->mpar ^= 1;
  if (S->first_sort) {
    // an input in arbitrary order: order every cell by id, back into the
    // arrays the scatter read
    CellsortArgs cs{};
    cs.reps = S->reps;
    cs.chunks = S->chunks;
    cs.cell_start = S->cell_start;
    cs.pos_src = a.pos_out;
    cs.vel_src = a.vel_out;
    cs.img_src = a.img_out;
    cs.id_src = a.id_out;
    cs.cell_src = a.cell_out;
    cs.prev_u_src = a.prev_u_out;
    cs.prev_off_src = a.prev_off_out;
    cs.pos = S->pos[S->pcur];
    cs.vel = S->vel[S->scur];
    cs.img = S->img[S->scur];
    cs.id = S->id[S->scur];
    cs.cell = S->cell[S->scur];
    cs.prev_u = S->prev_u[S->scur];
    cs.prev_off = S->prev_off[S->scur];
    launch_cellsort(S->D, S->L.nchunks, cs, S->stream);
    S->first_sort = false;
  } else {
    S->pcur ^= 1;
    S->scur ^= 1;
  }
  S->since_sort = 0;
  if (S->L.kmax > 0) enqueue_nlist(S, S->P);
}

void enqueue_force(mdlg_system* S, int mode, bool sort_follows, float* acc_out) {
  ForceArgs a{};
  a.P = S->P;
  if (sort_follows) {
    // the rebuild that follows canonicalises any move of up to one cell
    a.P.lo = -S->P.s;
    a.P.hi = 2.f * S->P.s;
  }
  a.reps = S->reps;
  a.bricks = S->bricks;
  a.cell_start = S->cell_start;
  a.pos_in = S->pos[S->pcur];
  a.pos_out = S->pos[S->pcur ^ 1];
  a.vel = S->vel[S->scur];
  a.acc_out = acc_out;
  a.err = S->err;
  a.mode = mode;
  a.nbricks = S->L.nbricks;
  a.xcd_remap = S->xcd_remap;
  if (S->L.kmax > 0) {
    a.smap = S->smap;
    a.binfo = S->binfo;
    a.nl = S->nl;
    a.trec = S->trec;
    // the drifts since the lists were built are checked; this one is
    // recorded unless the rebuild that follows makes new lists
    a.stale_in = S->stale + S->since_sort;
    a.disp_in = S->disp;
    a.psum = S->psum;
    a.ndisp = S->since_sort;
    const bool drift = (mode == kModeStep || mode == kModeStart);
    if (drift && !sort_follows) {
      a.disp_out = S->disp + (size_t)S->since_sort * kDispRow;
      a.stale_out = S->stale + S->since_sort + 1;
    }
    a.fallbacks = S->fallbacks;
  }
  {
    TimedLaunch t(S, MDLG_K_FORCE);
    launch_force(S->D, a, S->stream);
  }
  if (mode == kModeStep || mode == kModeStart) S->pcur ^= 1;
}

// Kinetics of the full-step velocities in the state (per replica, FP64):
// per-chunk partials, then their sum per replica; with thermostat, the
// rescale to kT as well.
void enqueue_kin(mdlg_system* S, bool thermostat) {
  KinPartArgs kp{};
  kp.chunks = S->chunks;
  kp.vel = S->vel[S->scur];
  kp.kpart = S->kpart;
  kp.mass = S->cfg.mass;
  launch_kinpart(S->D, S->L.nchunks, kp, S->stream);
  KinArgs k{};
  k.reps = S->reps;
  k.kpart = S->kpart;
  k.kin = S->kin;
  k.lambda = S->lambda;
  k.n_rep = (int)S->L.reps.size();
  k.D = S->D;
  k.thermostat = thermostat ? 1 : 0;
  k.kT = S->cfg.kT;
  k.mass = S->cfg.mass;
  launch_kin(k, S->stream);
  if (thermostat) {
    // the velocities at the current time, rescaled now
    RescaleArgs r{};
    r.chunks = S->chunks;
    r.lambda = S->lambda;
    r.vel = S->vel[S->scur];
    launch_rescale(S->D, S->L.nchunks, r, S->stream);
  }
}

// One velocity-Verlet step; force_sort requests a rebuild right after it.
void enqueue_md_step(mdlg_system* S, bool force_sort) {
  const int mode = S->vel_full ? kModeStart : kModeStep;
  const bool sort_next = force_sort || (S->since_sort + 1 >= S->L.sort_every);
  enqueue_force(S, mode, sort_next, nullptr);
  S->vel_full = false;
  S->since_sort += 1;
  S->md_step += 1;
  if (sort_next) enqueue_sort(S);
}

void enqueue_bin(mdlg_system* S, bool snapshot_only) {
  BinArgs b{};
  b.P = S->P;
  b.reps = S->reps;
  b.strips = S->strips;
  b.cell_start = S->cell_start;
  b.pos = S->pos[S->pcur];
  b.img = S->img[S->scur];
  b.id = S->id[S->scur];
  b.cell = S->cell[S->scur];
  b.prev_u = S->prev_u[S->scur];
  b.prev_off = S->prev_off[S->scur];
  b.A = S->A;
  b.mom = S->mom;
  b.dpart = S->dpart;
  b.err = S->err;
  b.snapshot_only = snapshot_only ? 1 : 0;
  b.BSX = S->L.BSX;
  b.BSY = S->L.BSY;
  b.nstep = (S->L.xi && !snapshot_only) ? S->nstep[S->xi_par] : nullptr;
  b.shift_k = (S->L.n_shifts > 0 && !snapshot_only) ? S->shift_k : nullptr;
  {
    TimedLaunch t(S, MDLG_K_BIN);
    launch_bin(S->D, S->L.nstrips, b, S->stream);
  }
}

void enqueue_snapshot(mdlg_system* S) {
  if (S->since_sort != 0) enqueue_sort(S);
  enqueue_bin(S, true);
  S->snapshot_valid = true;
  S->xi_have = false;  // a new chain of lattice steps starts here
}

// Xi of the previous lattice step from its arrivals and this step's.
void enqueue_xi(mdlg_system* S) {
  XiArgs x{};
  x.reps = S->reps;
  x.ncur = S->nstep[S->xi_par];
  x.nprev = S->nstep[S->xi_par ^ 1];
  x.xi_site = S->xi_site;
  x.xi_last = S->xi_last;
  x.sums = S->xi_sums;
  x.part = S->xi_part;
  x.n_sites = (int)S->L.n_sites;
  x.sites_per_block = kXiSites;
  x.nblocks = xi_blocks(S->L);
  x.n_rep = (int)S->L.reps.size();
  x.Q = S->L.Q;
  x.vmax = S->cfg.vmax;
  TimedLaunch t(S, MDLG_K_XI);
  launch_xi(S->D, x, S->stream);
}

// The last `steps` MD steps of a lattice step (the last one followed by a
// cell-list rebuild), then the lattice step's binning.
void enqueue_lattice_tail(mdlg_system* S, int steps) {
  for (int s = 1; s <= steps; ++s) enqueue_md_step(S, s == steps);
  if (S->L.n_shifts > 0) {
    // before the binning, which moves the snapshot forward
    ShiftArgs h{};
    h.P = S->P;
    h.reps = S->reps;
    h.chunks = S->chunks;
    h.pos = S->pos[S->pcur];
    h.img = S->img[S->scur];
    h.cell = S->cell[S->scur];
    h.prev_u = S->prev_u[S->scur];
    h.prev_off = S->prev_off[S->scur];
    h.shifts = S->shifts;
    h.shift_k = S->shift_k;
    h.acc = S->shift_acc;
    h.dx = S->cfg.lattice_dx;
    h.n_shifts = S->L.n_shifts;
    h.nchunks = S->L.nchunks;
    TimedLaunch t(S, MDLG_K_SHIFT);
    launch_shift(S->D, h, S->stream);
  }
  enqueue_bin(S, false);
  if (S->L.xi) {
    if (S->xi_have) {
      enqueue_xi(S);
      S->xi_steps += 1;
    }
    S->xi_par ^= 1;
    S->xi_have = true;
  }
  S->n_lattice += 1;
}

void enqueue_lattice_step(mdlg_system* S) { enqueue_lattice_tail(S, S->cfg.md_steps_per_lattice_step); }

mdlg_status read_err(mdlg_system* S) {
  unsigned e = 0;
  HIPCHK(S, hipMemcpyAsync(&e, S->err, sizeof e, hipMemcpyDeviceToHost, S->stream));
  HIPCHK(S, hipStreamSynchronize(S->stream));
  if (e) {
    std::string m = "device error word 0x" + std::to_string(e) + ":";
    if (e & kErrMargin)
      m += " a particle left its cell between rebuilds by more than the stencil's reach (stencil s - r_cut) / 2 (lower sort_every or dt);";
    if (e & kErrRecord) m += " internal: a pair-list target record named no particle;";
    if (e & kErrNonFinite) m += " non-finite coordinates;";
    if (e & kErrJump) m += " a particle moved more than one cell between rebuilds or started outside the box;";
    if (e & kErrImage) m += " image counter out of range;";
    if (e & kErrOverflow) m += " cell occupancy overflow;";
    S->last_error = m;
    return MDLG_E_UNSTABLE;
  }
  return MDLG_OK;
}

void zero_accumulators(mdlg_system* S) {
  const Layout& L = S->L;
  launch_fill_u32(S->A, 0u, (long long)L.n_sites * L.Q, S->stream);
  launch_fill_u32(reinterpret_cast<unsigned*>(S->mom), 0u, (long long)L.n_sites * L.nm * 2, S->stream);
  launch_fill_u32(reinterpret_cast<unsigned*>(S->dpart), 0u, (long long)L.nstrips * 2 * L.D * 2,
                  S->stream);
  if (L.n_shifts > 0) {
    launch_fill_u32(reinterpret_cast<unsigned*>(S->shift_acc), 0u,
                    (long long)L.n_shifts * shift_per(L) * 2 * kTileCopies, S->stream);
    // lattice time of the next arrival: 1 (the snapshot is time 0)
    launch_fill_u32(reinterpret_cast<unsigned*>(S->shift_k), 1u, 1, S->stream);
    launch_fill_u32(reinterpret_cast<unsigned*>(S->shift_k) + 1, 0u, 1, S->stream);
  }
  if (L.xi) {
    launch_fill_u32(reinterpret_cast<unsigned*>(S->xi_site), 0u, (long long)L.n_sites * L.Q * 2,
                    S->stream);
    launch_fill_u32(reinterpret_cast<unsigned*>(S->xi_last), 0u, (long long)L.n_sites * L.Q,
                    S->stream);
    launch_fill_u32(reinterpret_cast<unsigned*>(S->xi_sums), 0u, (long long)5 * L.Q * 2, S->stream);
    S->xi_steps = 0;
  }
  S->n_lattice = 0;
}

// ----- checkpoints

// the blob format, raised whenever a saved region changes its layout (3: the
// staging-map entries carry their LDS slot)
constexpr char kCkptMagic[8] = {'M', 'D', 'L', 'G', 'C', 'K', 'P', '3'};

struct CkptHeader {
  char magic[8];
  uint64_t fingerprint;
  uint64_t bytes;  // whole blob
  int32_t pcur, scur, since_sort, vel_full, mpar, xi_par, xi_have, snapshot_valid, has_lists, pad;
  int64_t md_step, n_lattice, xi_steps;
};

void fnv(uint64_t& h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
}

// Everything a trajectory depends on: the configuration (current LJ
// parameters included) and the layout derived from it.
uint64_t fingerprint(const mdlg_system* S) {
  uint64_t h = 1469598103934665603ull;
  const mdlg_config& c = S->cfg;
  const Layout& L = S->L;
  const int32_t ints[] = {c.dim, c.n_replicas, c.forces_off, c.md_steps_per_lattice_step, c.vmax,
                          c.thermostat_every, L.k, L.sort_every, L.BX, L.BY, L.BZ, L.bthreads,
                          L.kmax, L.lcap, L.Q, L.nm, L.nbricks, L.nstrips, L.xi ? 1 : 0,
                          L.n_shifts};
  fnv(h, ints, sizeof ints);
  const double dbl[] = {c.lattice_dx, c.epsilon, c.sigma, c.mass, c.r_cut, c.dt, c.kT};
  fnv(h, dbl, sizeof dbl);
  fnv(h, S->n_particles.data(), S->n_particles.size() * sizeof(int32_t));
  fnv(h, S->lattice.data(), S->lattice.size() * sizeof(int32_t));
  fnv(h, S->shifts_host.data(), S->shifts_host.size() * sizeof(double));
  return h;
}

struct Region {
  void* dev;
  size_t bytes;
};

// The device buffers of a checkpoint, in blob order.  The pair lists are
// included only between rebuilds; at a rebuild they are rebuilt from the
// restored positions, which reproduces them exactly.
std::vector<Region> ckpt_regions(mdlg_system* S, bool lists) {
  const Layout& L = S->L;
  const int D = L.D;
  const size_t N = (size_t)L.n_total;
  std::vector<Region> r = {
      {S->pos[S->pcur], N * D * sizeof(float)},
      {S->vel[S->scur], N * D * sizeof(float)},
      {S->img[S->scur], N * D * sizeof(int)},
      {S->id[S->scur], N * sizeof(int)},
      {S->cell[S->scur], N * sizeof(int)},
      {S->prev_u[S->scur], N * D * sizeof(int)},
      {S->prev_off[S->scur], N * D * sizeof(float)},
      {S->cell_start, ((size_t)L.n_cells + 1) * sizeof(int)},
      {S->A, (size_t)L.n_sites * L.Q * sizeof(unsigned)},
      {S->mom, (size_t)L.n_sites * L.nm * sizeof(long long)},
      {S->dpart, (size_t)L.nstrips * 2 * D * sizeof(double)},
      {S->kin, L.reps.size() * (D + 1) * sizeof(double)},
  };
  if (L.n_shifts > 0) {
    r.push_back({S->shift_k, sizeof(long long)});
    r.push_back({S->shift_acc, (size_t)L.n_shifts * shift_per(L) * kTileCopies * sizeof(unsigned long long)});
  }
  if (L.xi) {
    const size_t sq = (size_t)L.n_sites * L.Q;
    r.push_back({S->nstep[0], sq * sizeof(unsigned)});
    r.push_back({S->nstep[1], sq * sizeof(unsigned)});
    r.push_back({S->xi_site, sq * sizeof(long long)});
    r.push_back({S->xi_last, sq * sizeof(int)});
    r.push_back({S->xi_sums, (size_t)5 * L.Q * sizeof(unsigned long long)});
  }
  if (lists) {
    r.push_back({S->smap, (size_t)L.nbricks * L.lcap * sizeof(int2)});
    r.push_back({S->binfo, (size_t)L.nbricks * sizeof(int4)});
    r.push_back({S->nl, (size_t)(L.kmax / 4) * N * sizeof(unsigned long long)});
    r.push_back({S->disp, (size_t)disp_rows(L) * kDispRow * sizeof(unsigned)});
    r.push_back({S->stale, (size_t)disp_rows(L) * sizeof(unsigned)});
    r.push_back({S->psum, (size_t)disp_rows(L) * sizeof(double)});
    r.push_back({S->trec, (size_t)L.nbricks * L.lcap * sizeof(int2)});
  }
  return r;
}

bool ckpt_lists(const mdlg_system* S) { return S->L.kmax > 0 && S->since_sort > 0; }

size_t ckpt_bytes(mdlg_system* S) {
  size_t b = sizeof(CkptHeader);
  for (const Region& r : ckpt_regions(S, ckpt_lists(S))) b += r.bytes;
  return b;
}

}  // namespace

// ---------------------------------------------------------------- C ABI

extern "C" {

mdlg_status mdlg_describe(const mdlg_config* cfg, mdlg_layout* out) {
  Layout L;
  std::string msg;
  if (!build_layout(cfg, &L, &msg)) {
    g_create_error = msg;
    return MDLG_E_INVALID;
  }
  if (out) *out = L.pub;
  return MDLG_OK;
}

mdlg_status mdlg_workspace_bytes(const mdlg_config* cfg, size_t* bytes) {
  if (!bytes) {
    g_create_error = "bytes is NULL";
    return MDLG_E_INVALID;
  }
  mdlg_system tmp;
  std::string msg;
  if (!build_layout(cfg, &tmp.L, &msg)) {
    g_create_error = msg;
    return MDLG_E_INVALID;
  }
  *bytes = carve(&tmp, nullptr);
  return MDLG_OK;
}

mdlg_status mdlg_create(const mdlg_config* cfg, void* workspace_dev, size_t workspace_bytes,
                        void* hip_stream, const float* pos_dev, const float* vel_dev,
                        mdlg_system** out) {
  if (!out) {
    g_create_error = "out is NULL";
    return MDLG_E_INVALID;
  }
  *out = nullptr;
  if (!workspace_dev || !pos_dev || !vel_dev) {
    g_create_error = "workspace, positions and velocities are required";
    return MDLG_E_INVALID;
  }
  if (reinterpret_cast<uintptr_t>(workspace_dev) & 255) {
    g_create_error = "workspace must be 256-byte aligned";
    return MDLG_E_INVALID;
  }
  mdlg_system* S = new mdlg_system();
  std::string msg;
  if (!build_layout(cfg, &S->L, &msg)) {
    g_create_error = msg;
    delete S;
    return MDLG_E_INVALID;
  }
  S->cfg = *cfg;
  S->D = cfg->dim;
  S->n_particles.assign(cfg->n_particles, cfg->n_particles + cfg->n_replicas);
  S->lattice.assign(cfg->lattice, cfg->lattice + (size_t)cfg->n_replicas * cfg->dim);
  S->cfg.n_particles = S->n_particles.data();
  S->cfg.lattice = S->lattice.data();
  const size_t need = carve(S, nullptr);
  if (workspace_bytes < need) {
    g_create_error = "workspace too small: need " + std::to_string(need) + " bytes";
    delete S;
    return MDLG_E_NOMEM;
  }
  S->ws = static_cast<char*>(workspace_dev);
  S->ws_bytes = workspace_bytes;
  carve(S, S->ws);
  S->P = make_phys(cfg, S->L);
  S->stream = static_cast<hipStream_t>(hip_stream);
  if (const char* g = getenv("MDLG_NO_GRAPH")) S->use_graph = !(g[0] == '1');
  if (const char* x = getenv("MDLG_NO_XCD_REMAP")) S->xcd_remap = !(x[0] == '1');
  auto fail = [&](mdlg_status st) {
    g_create_error = S->last_error;
    delete S;
    return st;
  };
#define CREATE_HIP(expr)                                              \
  do {                                                                \
    hipError_t e_ = (expr);                                           \
    if (e_ != hipSuccess) return fail(hip_fail(S, e_, #expr));        \
  } while (0)
  const Layout& L = S->L;
  CREATE_HIP(hipMemcpyAsync(S->reps, L.reps.data(), L.reps.size() * sizeof(Replica),
                            hipMemcpyHostToDevice, S->stream));
  CREATE_HIP(hipMemcpyAsync(S->bricks, L.bricks.data(), L.bricks.size() * sizeof(int4),
                            hipMemcpyHostToDevice, S->stream));
  CREATE_HIP(hipMemcpyAsync(S->chunks, L.chunks.data(), L.chunks.size() * sizeof(int4),
                            hipMemcpyHostToDevice, S->stream));
  CREATE_HIP(hipMemcpyAsync(S->cchunks, L.cchunks.data(), L.cchunks.size() * sizeof(int4),
                            hipMemcpyHostToDevice, S->stream));
  CREATE_HIP(hipMemcpyAsync(S->strips, L.strips.data(), L.strips.size() * sizeof(int4),
                            hipMemcpyHostToDevice, S->stream));
  if (L.n_shifts > 0) {
    S->shifts_host.assign(cfg->shifts, cfg->shifts + (size_t)L.n_shifts * 2 * L.D);
    S->cfg.shifts = S->shifts_host.data();
    CREATE_HIP(hipMemcpyAsync(S->shifts, S->shifts_host.data(),
                              S->shifts_host.size() * sizeof(double), hipMemcpyHostToDevice,
                              S->stream));
  }
  launch_fill_u32(reinterpret_cast<unsigned*>(S->count), 0u, L.n_cells, S->stream);
  launch_fill_u32(reinterpret_cast<unsigned*>(S->tile_sum), 0u, (long long)L.ntiles * kTileCopies, S->stream);
  for (int i = 0; i < 2; ++i)
    launch_fill_u32(S->mcnt[i], 0u, L.n_cells * arrival_words(L.D), S->stream);
  launch_fill_u32(S->err, 0u, 64, S->stream);
  launch_fill_f32(S->lambda, 1.f, (long long)L.reps.size(), S->stream);
  if (S->fallbacks) launch_fill_u32(reinterpret_cast<unsigned*>(S->fallbacks), 0u, 2, S->stream);
  zero_accumulators(S);
  // ingest into set 0, then the first counting sort
  IngestArgs ia{};
  ia.P = S->P;
  ia.reps = S->reps;
  ia.chunks = S->chunks;
  ia.pos_abs = pos_dev;
  ia.vel_in = vel_dev;
  ia.pos = S->pos[0];
  ia.vel = S->vel[0];
  ia.img = S->img[0];
  ia.id = S->id[0];
  ia.cell = S->cell[0];
  ia.err = S->err;
  launch_ingest(S->D, L.nchunks, ia, S->stream);
  S->pcur = 0;
  S->scur = 0;
  S->first_sort = true;
  enqueue_sort(S);
  enqueue_bin(S, true);
  S->snapshot_valid = true;
  S->vel_full = true;
  if (check_launch(S, "mdlg_create kernels") != MDLG_OK) return fail(MDLG_E_DEVICE);
  CREATE_HIP(hipStreamSynchronize(S->stream));
  mdlg_status st = read_err(S);
  if (st != MDLG_OK) return fail(st);
  *out = S;
  return MDLG_OK;
}

mdlg_status mdlg_create_static(const mdlg_config* cfg, void* hip_stream, const float* pos_dev,
                               const float* vel_dev, mdlg_system** out) {
  if (!out) {
    g_create_error = "out is NULL";
    return MDLG_E_INVALID;
  }
  *out = nullptr;
  size_t need = 0;
  mdlg_status st = mdlg_workspace_bytes(cfg, &need);
  if (st != MDLG_OK) return st;
  if (need > kStaticWorkspaceBytes) {
    g_create_error = "configuration needs a workspace of " + std::to_string(need) +
                     " bytes; the static workspace holds " + std::to_string(kStaticWorkspaceBytes) +
                     " (use mdlg_create with a workspace of that size)";
    return MDLG_E_NOMEM;
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticSlot& slot = g_static[dev];
  if (slot.in_use) {
    g_create_error = "the static workspace of device " + std::to_string(dev) +
                     " is held by another handle (mdlg_destroy it first)";
    return MDLG_E_STATE;
  }
  if (!slot.ptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
    slot.ptr = p;
  }
  // mdlg_create clears every buffer that must start at zero (the array holds
  // whatever the last handle left)
  st = mdlg_create(cfg, slot.ptr, kStaticWorkspaceBytes, hip_stream, pos_dev, vel_dev, out);
  if (st != MDLG_OK) return st;
  slot.in_use = true;
  (*out)->static_dev = dev;
  return MDLG_OK;
}

extern "C++" {

static mdlg_system::SeqState seq_state(const mdlg_system* S) {
  return {S->pcur, S->scur, S->since_sort, S->vel_full, S->mpar, S->xi_par, S->xi_have,
          S->md_step, S->n_lattice, S->xi_steps};
}

static void set_seq_state(mdlg_system* S, const mdlg_system::SeqState& q) {
  S->pcur = q.pcur;
  S->scur = q.scur;
  S->since_sort = q.since_sort;
  S->vel_full = q.vel_full;
  S->mpar = q.mpar;
  S->xi_par = q.xi_par;
  S->xi_have = q.xi_have;
  S->md_step = q.md_step;
  S->n_lattice = q.n_lattice;
  S->xi_steps = q.xi_steps;
}

// Launch the work `body` enqueues as a HIP graph: captured (on a capture
// stream, recording only) the first time it is asked for from this
// sequencing state, replayed on the user's stream every time.  The host
// state then advances as the body would have advanced it.
template <class F>
mdlg_status replay_graph(mdlg_system* S, int kind, F body, unsigned long long tag = 0) {
  auto key = std::make_tuple(kind, S->pcur, S->scur, S->since_sort, S->vel_full, S->mpar,
                             S->xi_par, S->xi_have, tag);
  auto it = S->graphs.find(key);
  const mdlg_system::SeqState before = seq_state(S);
  if (it == S->graphs.end()) {
    if (!S->cap_stream) HIPCHK(S, hipStreamCreateWithFlags(&S->cap_stream, hipStreamNonBlocking));
    hipStream_t user = S->stream;
    S->stream = S->cap_stream;
    HIPCHK(S, hipStreamBeginCapture(S->cap_stream, hipStreamCaptureModeThreadLocal));
    body();
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(S->cap_stream, &g);
    S->stream = user;
    mdlg_system::GraphEntry ent{};
    ent.after = seq_state(S);
    // the capture only recorded work: back to the state it started from
    set_seq_state(S, before);
    if (e != hipSuccess) return hip_fail(S, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&ent.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(S, e, "hipGraphInstantiate");
    // counters advance by the replay's increments from wherever they stand
    ent.after.md_step -= before.md_step;
    ent.after.n_lattice -= before.n_lattice;
    ent.after.xi_steps -= before.xi_steps;
    it = S->graphs.emplace(key, ent).first;
  }
  HIPCHK(S, hipGraphLaunch(it->second.exec, S->stream));
  mdlg_system::SeqState q = it->second.after;
  q.md_step += before.md_step;
  q.n_lattice += before.n_lattice;
  q.xi_steps += before.xi_steps;
  set_seq_state(S, q);
  return MDLG_OK;
}

}  // extern "C++"

// One block of plain MD steps, with the equilibration thermostat at every
// thermostat_every-th step.
static void enqueue_md_steps(mdlg_system* S, int64_t n) {
  const int te = S->cfg.thermostat_every;
  for (int64_t i = 0; i < n; ++i) {
    enqueue_md_step(S, false);
    if (te > 0 && S->md_step % te == 0) {
      enqueue_force(S, kModeFinish, false, nullptr);
      enqueue_kin(S, true);
      S->vel_full = true;
    }
  }
}

mdlg_status mdlg_step(mdlg_system* S, int64_t n) {
  if (!S) return MDLG_E_INVALID;
  if (n < 0) {
    S->last_error = "n_md_steps must be >= 0";
    return MDLG_E_INVALID;
  }
  if (!S->use_graph || S->timing) {
    enqueue_md_steps(S, n);
  } else {
    // graphs of up to kGraphBlockSteps steps, keyed by the block length and
    // the thermostat's phase
    const int te = S->cfg.thermostat_every;
    for (int64_t left = n; left > 0;) {
      const int m = (int)std::min<int64_t>(left, kGraphBlockSteps);
      const unsigned long long tag =
          ((unsigned long long)m << 32) | (unsigned long long)(te > 0 ? S->md_step % te : 0);
      mdlg_status st = replay_graph(S, kStepGraph, [S, m] { enqueue_md_steps(S, m); }, tag);
      if (st != MDLG_OK) return st;
      left -= m;
    }
  }
  if (n > 0) S->snapshot_valid = false;
  return check_launch(S, "mdlg_step");
}

mdlg_status mdlg_coarse_grain(mdlg_system* S, int64_t T) {
  if (!S) return MDLG_E_INVALID;
  if (T < 0) {
    S->last_error = "n_lattice_steps must be >= 0";
    return MDLG_E_INVALID;
  }
  if (T == 0) return MDLG_OK;
  if (!S->snapshot_valid) enqueue_snapshot(S);
  const int steps = S->cfg.md_steps_per_lattice_step;
  // lattice steps of many MD steps are replayed in blocks (a graph of a whole
  // lattice step would hold every launch of it): blocks of whole rebuild
  // intervals, then the rest of the lattice step with its binning
  const int R = std::max(1, S->L.sort_every);
  const int block = R * std::max(1, kGraphBlockSteps / R);
  for (int64_t t = 0; t < T; ++t) {
    if (!S->use_graph || S->timing) {
      enqueue_lattice_step(S);
      continue;
    }
    mdlg_status st;
    if (steps <= kGraphMaxSteps) {
      st = replay_graph(S, 0, [S] { enqueue_lattice_step(S); });
    } else {
      int left = steps;
      st = MDLG_OK;
      while (st == MDLG_OK && left > block) {
        st = replay_graph(S, block, [S, block] {
          for (int i = 0; i < block; ++i) enqueue_md_step(S, false);
        });
        left -= block;
      }
      if (st == MDLG_OK) st = replay_graph(S, -left, [S, left] { enqueue_lattice_tail(S, left); });
    }
    if (st != MDLG_OK) return st;
  }
  return check_launch(S, "mdlg_coarse_grain");
}

mdlg_status mdlg_get_f(mdlg_system* S, double* f, double* f_site, double* mom_site, uint64_t* counts,
                       int64_t* n_samples, int64_t* n_overflow, double* disp,
                       int64_t* n_lattice_steps) {
  if (!S) return MDLG_E_INVALID;
  const Layout& L = S->L;
  const int D = S->D;
  launch_fill_u32(reinterpret_cast<unsigned*>(S->fcount), 0u, kMaxQ * 2, S->stream);
  launch_fill_u32(reinterpret_cast<unsigned*>(S->momsum), 0u, 32, S->stream);
  FsumArgs fs{};
  fs.A = S->A;
  fs.mom = S->mom;
  fs.fcount = S->fcount;
  fs.momsum = S->momsum;
  fs.n_sites = (int)L.n_sites;
  fs.Q = L.Q;
  fs.nm = L.nm;
  fs.sites_per_block = 64;
  launch_fsum(fs, S->stream);
  FfinalArgs ff{};
  ff.fcount = S->fcount;
  ff.dpart = S->dpart;
  ff.f = S->fout;
  ff.disp = S->dispout;
  ff.denom = (double)S->n_lattice * (double)L.n_sites;
  ff.Q = L.Q;
  ff.nstrips = L.nstrips;
  ff.nd = 2 * D;
  launch_ffinal(ff, S->stream);
  mdlg_status st = check_launch(S, "mdlg_get_f kernels");
  if (st != MDLG_OK) return st;
  std::vector<double> fh(L.Q), dh(2 * D);
  std::vector<unsigned long long> ch(L.Q);
  std::vector<long long> mh(16);
  HIPCHK(S, hipMemcpyAsync(fh.data(), S->fout, L.Q * sizeof(double), hipMemcpyDeviceToHost, S->stream));
  HIPCHK(S, hipMemcpyAsync(ch.data(), S->fcount, L.Q * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           S->stream));
  HIPCHK(S, hipMemcpyAsync(mh.data(), S->momsum, 16 * sizeof(long long), hipMemcpyDeviceToHost, S->stream));
  HIPCHK(S, hipMemcpyAsync(dh.data(), S->dispout, 2 * D * sizeof(double), hipMemcpyDeviceToHost, S->stream));
  if (f_site || mom_site) {
    const double inv_T = S->n_lattice > 0 ? 1.0 / (double)S->n_lattice : 0.0;
    const size_t per_site = (size_t)std::max(L.Q, L.nm) * sizeof(double);
    const long long chunk = std::max<long long>(1, (long long)(S->staging_bytes / (2 * per_site)));
    double* sf = reinterpret_cast<double*>(S->staging);
    double* sm = sf + chunk * L.Q;
    for (long long s0 = 0; s0 < L.n_sites; s0 += chunk) {
      const long long cnt = std::min(chunk, L.n_sites - s0);
      SiteAvgArgs sa{};
      sa.A = S->A;
      sa.mom = S->mom;
      sa.f_site = f_site ? sf : nullptr;
      sa.mom_site = mom_site ? sm : nullptr;
      sa.first = s0;
      sa.count = cnt;
      sa.Q = L.Q;
      sa.nm = L.nm;
      sa.inv_T = inv_T;
      launch_site_avg(sa, S->stream);
      if (f_site)
        HIPCHK(S, hipMemcpyAsync(f_site + s0 * L.Q, sf, cnt * L.Q * sizeof(double), hipMemcpyDeviceToHost,
                                 S->stream));
      if (mom_site)
        HIPCHK(S, hipMemcpyAsync(mom_site + s0 * L.nm, sm, cnt * L.nm * sizeof(double),
                                 hipMemcpyDeviceToHost, S->stream));
      HIPCHK(S, hipStreamSynchronize(S->stream));
    }
  }
  st = read_err(S);  // synchronises
  if (f) std::memcpy(f, fh.data(), L.Q * sizeof(double));
  if (counts) std::memcpy(counts, ch.data(), L.Q * sizeof(uint64_t));
  if (disp) std::memcpy(disp, dh.data(), 2 * D * sizeof(double));
  if (n_samples) *n_samples = S->n_lattice * L.n_sites;
  if (n_overflow) *n_overflow = mh[1];
  if (n_lattice_steps) *n_lattice_steps = S->n_lattice;
  return st;
}

mdlg_status mdlg_get_kinetics(mdlg_system* S, double* out) {
  if (!S || !out) return MDLG_E_INVALID;
  // (a half-step state is completed first)
  if (!S->vel_full) enqueue_force(S, kModeFinish, false, nullptr);
  S->vel_full = true;
  enqueue_kin(S, false);
  mdlg_status st = check_launch(S, "mdlg_get_kinetics");
  if (st != MDLG_OK) return st;
  const size_t n = S->L.reps.size() * (S->D + 1);
  HIPCHK(S, hipMemcpyAsync(out, S->kin, n * sizeof(double), hipMemcpyDeviceToHost, S->stream));
  return read_err(S);
}

mdlg_status mdlg_get_shifts(mdlg_system* S, uint64_t* counts, int64_t* moments, int64_t* n_steps) {
  if (!S) return MDLG_E_INVALID;
  const Layout& L = S->L;
  if (L.n_shifts == 0) {
    S->last_error = "no shifted lattices were configured (n_shifts = 0)";
    return MDLG_E_STATE;
  }
  const int per = shift_per(L), nmo = per - L.Q - 1;
  // the kernel's per-XCD copies of the accumulators, summed here (modulo
  // 2^64: the moments are two's-complement)
  const size_t one = (size_t)L.n_shifts * per;
  std::vector<unsigned long long> hc(one * kTileCopies), h(one, 0ull);
  HIPCHK(S, hipMemcpyAsync(hc.data(), S->shift_acc, hc.size() * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, S->stream));
  mdlg_status st = read_err(S);
  for (int c = 0; c < kTileCopies; ++c)
    for (size_t i = 0; i < one; ++i) h[i] += hc[(size_t)c * one + i];
  for (int j = 0; j < L.n_shifts; ++j) {
    if (counts)
      for (int i = 0; i <= L.Q; ++i) counts[(size_t)j * (L.Q + 1) + i] = h[(size_t)j * per + i];
    if (moments)
      for (int i = 0; i < nmo; ++i)
        moments[(size_t)j * nmo + i] = (int64_t)h[(size_t)j * per + L.Q + 1 + i];
  }
  if (n_steps) *n_steps = S->n_lattice;
  return st;
}

mdlg_status mdlg_get_xi(mdlg_system* S, int64_t* sums, int64_t* xi_site, int32_t* xi_last,
                        int64_t* n_steps) {
  if (!S) return MDLG_E_INVALID;
  const Layout& L = S->L;
  if (!L.xi) {
    S->last_error = "collision_stats was not enabled in the configuration";
    return MDLG_E_STATE;
  }
  const size_t sq = (size_t)L.n_sites * L.Q;
  if (sums)
    HIPCHK(S, hipMemcpyAsync(sums, S->xi_sums, sizeof(int64_t) * 5 * L.Q, hipMemcpyDeviceToHost,
                             S->stream));
  if (xi_site)
    HIPCHK(S, hipMemcpyAsync(xi_site, S->xi_site, sizeof(int64_t) * sq, hipMemcpyDeviceToHost,
                             S->stream));
  if (xi_last)
    HIPCHK(S, hipMemcpyAsync(xi_last, S->xi_last, sizeof(int32_t) * sq, hipMemcpyDeviceToHost,
                             S->stream));
  if (n_steps) *n_steps = S->xi_steps;
  return read_err(S);
}

mdlg_status mdlg_reset_accumulators(mdlg_system* S) {
  if (!S) return MDLG_E_INVALID;
  zero_accumulators(S);
  S->snapshot_valid = false;
  return check_launch(S, "mdlg_reset_accumulators");
}

mdlg_status mdlg_get_state(mdlg_system* S, mdlg_particles* out) {
  if (!S || !out) return MDLG_E_INVALID;
  const Layout& L = S->L;
  const int D = S->D;
  const size_t nd = (size_t)L.n_total * D;
  enqueue_force(S, S->vel_full ? kModeProbe : kModeFinish, false, S->acc_sorted);
  S->vel_full = true;
  XportArgs x{};
  x.P = S->P;
  x.reps = S->reps;
  x.chunks = S->chunks;
  x.pos = S->pos[S->pcur];
  x.vel = S->vel[S->scur];
  x.img = S->img[S->scur];
  x.id = S->id[S->scur];
  x.cell = S->cell[S->scur];
  x.acc = S->acc_sorted;
  x.x_u = reinterpret_cast<int*>(S->staging);
  x.x_off = reinterpret_cast<float*>(S->staging) + nd;
  x.x_vel = reinterpret_cast<float*>(S->staging) + 2 * nd;
  x.x_acc = reinterpret_cast<float*>(S->staging) + 3 * nd;
  x.prev_u = S->prev_u[S->scur];
  x.prev_off = S->prev_off[S->scur];
  x.x_pu = reinterpret_cast<int*>(S->staging) + 4 * nd;
  x.x_poff = reinterpret_cast<float*>(S->staging) + 5 * nd;
  x.err = S->err;
  launch_export(D, L.nchunks, x, S->stream);
  mdlg_status st = check_launch(S, "mdlg_get_state");
  if (st != MDLG_OK) return st;
  if (out->ucell) HIPCHK(S, hipMemcpyAsync(out->ucell, x.x_u, nd * 4, hipMemcpyDeviceToHost, S->stream));
  if (out->off) HIPCHK(S, hipMemcpyAsync(out->off, x.x_off, nd * 4, hipMemcpyDeviceToHost, S->stream));
  if (out->vel) HIPCHK(S, hipMemcpyAsync(out->vel, x.x_vel, nd * 4, hipMemcpyDeviceToHost, S->stream));
  if (out->acc) HIPCHK(S, hipMemcpyAsync(out->acc, x.x_acc, nd * 4, hipMemcpyDeviceToHost, S->stream));
  if (out->prev_ucell)
    HIPCHK(S, hipMemcpyAsync(out->prev_ucell, x.x_pu, nd * 4, hipMemcpyDeviceToHost, S->stream));
  if (out->prev_off)
    HIPCHK(S, hipMemcpyAsync(out->prev_off, x.x_poff, nd * 4, hipMemcpyDeviceToHost, S->stream));
  return read_err(S);
}

mdlg_status mdlg_set_state(mdlg_system* S, const mdlg_particles* in) {
  if (!S || !in) return MDLG_E_INVALID;
  if (!in->ucell || !in->off || !in->vel) {
    S->last_error = "set_state needs ucell, off and vel";
    return MDLG_E_INVALID;
  }
  if ((in->prev_ucell == nullptr) != (in->prev_off == nullptr)) {
    S->last_error = "prev_ucell and prev_off go together";
    return MDLG_E_INVALID;
  }
  const Layout& L = S->L;
  const int D = S->D;
  const size_t nd = (size_t)L.n_total * D;
  const float s = S->P.s;
  for (size_t i = 0; i < nd; ++i) {
    if (!(in->off[i] >= 0.f && in->off[i] < s) || !std::isfinite(in->vel[i])) {
      S->last_error = "offset outside [0, s) or non-finite velocity at element " + std::to_string(i);
      return MDLG_E_INVALID;
    }
    if (in->prev_off && !(in->prev_off[i] >= 0.f && in->prev_off[i] < s)) {
      S->last_error = "prev offset outside [0, s) at element " + std::to_string(i);
      return MDLG_E_INVALID;
    }
  }
  // wait for queued work before overwriting the staging area
  HIPCHK(S, hipStreamSynchronize(S->stream));
  XportArgs x{};
  x.P = S->P;
  x.reps = S->reps;
  x.chunks = S->chunks;
  x.pos = S->pos[S->pcur];
  x.vel = S->vel[S->scur];
  x.img = S->img[S->scur];
  x.id = S->id[S->scur];
  x.cell = S->cell[S->scur];
  x.x_u = reinterpret_cast<int*>(S->staging);
  x.x_off = reinterpret_cast<float*>(S->staging) + nd;
  x.x_vel = reinterpret_cast<float*>(S->staging) + 2 * nd;
  x.prev_u = S->prev_u[S->scur];
  x.prev_off = S->prev_off[S->scur];
  if (in->prev_ucell) {
    x.x_pu = reinterpret_cast<int*>(S->staging) + 4 * nd;
    x.x_poff = reinterpret_cast<float*>(S->staging) + 5 * nd;
    HIPCHK(S, hipMemcpyAsync(x.x_pu, in->prev_ucell, nd * 4, hipMemcpyHostToDevice, S->stream));
    HIPCHK(S, hipMemcpyAsync(x.x_poff, in->prev_off, nd * 4, hipMemcpyHostToDevice, S->stream));
  }
  x.err = S->err;
  HIPCHK(S, hipMemcpyAsync(x.x_u, in->ucell, nd * 4, hipMemcpyHostToDevice, S->stream));
  HIPCHK(S, hipMemcpyAsync(x.x_off, in->off, nd * 4, hipMemcpyHostToDevice, S->stream));
  HIPCHK(S, hipMemcpyAsync(x.x_vel, in->vel, nd * 4, hipMemcpyHostToDevice, S->stream));
  launch_import(D, L.nchunks, x, S->stream);
  S->since_sort = 1;  // the imported arrays are in id order: rebuild
  S->first_sort = true;
  enqueue_sort(S);
  if (!in->prev_ucell) enqueue_bin(S, true);
  S->snapshot_valid = true;
  S->xi_have = false;
  S->vel_full = true;
  mdlg_status st = check_launch(S, "mdlg_set_state");
  if (st != MDLG_OK) return st;
  HIPCHK(S, hipStreamSynchronize(S->stream));
  return read_err(S);
}

// Phys of an adjoint window: the cell list stays frozen for the whole window,
// so particles may use the stencil's full reach (ns s - r_cut) / 2, which the
// cell walk's pruning and drift bounds already take.
static Phys window_phys(const mdlg_system* S) {
  Phys P = S->P;
  P.lcap = S->L.lcap_adj;
  P.kmax = 0;
  return P;
}

// The window's force launches with pair lists (radius r_cut + 2 margin_max,
// the stencil's reach): the force kernel's LDS capacity, and the list
// parameters for that margin.
static Phys window_list_phys(const mdlg_system* S) {
  Phys P = window_phys(S);
  P.lcap = S->L.lcap;
  set_list_params(P, &S->cfg, S->L, S->L.margin_max, S->L.kmax_adj);
  return P;
}

// kdisp: drifts made since the lists were built (checked, and this one
// recorded), or -1 for a recomputation of steps already checked.
static ForceArgs force_args_raw(mdlg_system* S, const Phys& P, int mode, const float* pos_in,
                                float* pos_out, float* vel, int kdisp, float* vel_full_out) {
  ForceArgs a{};
  a.P = P;
  a.vel_full_out = vel_full_out;
  if (P.kmax > 0) {
    // lists built at the start of the window by enqueue_nlist(S, P)
    a.smap = S->smap;
    a.binfo = S->binfo;
    a.nl = S->nl;
    a.trec = S->trec;
    if (kdisp >= 0) {
      a.stale_in = S->stale + kdisp;
      a.disp_in = S->disp;
      a.psum = S->psum;
      a.ndisp = kdisp;
      a.disp_out = S->disp + (size_t)kdisp * kDispRow;
      a.stale_out = S->stale + kdisp + 1;
      a.fallbacks = S->fallbacks;
    } else {
      // a recomputation inside the window: the flag at its end covers it
      a.stale_in = S->stale + S->adj_window_steps;
    }
  }
  a.reps = S->reps;
  a.bricks = S->bricks;
  a.cell_start = S->cell_start;
  a.pos_in = pos_in;
  a.pos_out = pos_out;
  a.vel = vel;
  a.err = S->err;
  a.mode = mode;
  a.nbricks = S->L.nbricks;
  a.xcd_remap = S->xcd_remap;
  return a;
}

static void launch_force_raw(mdlg_system* S, const Phys& P, int mode, const float* pos_in,
                             float* pos_out, float* vel, int kdisp, float* vel_full_out = nullptr) {
  const ForceArgs a = force_args_raw(S, P, mode, pos_in, pos_out, vel, kdisp, vel_full_out);
  TimedLaunch t(S, MDLG_K_FORCE);
  launch_force(S->D, a, S->stream);
}

// The adjoint velocity buffer that receives dL/dv0 in id order after the
// reverse sweep of a window of W steps: the sweep flips the two buffers once
// per reverse step (W + 1 of them, whatever the checkpoint interval), leaving
// lam_v in buffer (W + 1) & 1; the other one is free.
static int adjoint_grad_buffer(int W) { return ((W + 1) & 1) ^ 1; }

static int enqueue_adjoint(mdlg_system* S, int32_t W, int32_t k, int32_t loss, bool want_g);

mdlg_status mdlg_adjoint(mdlg_system* S, int32_t W, int32_t k, int32_t loss, const float* v0_dev,
                         double* out_loss, double* dL_deps, double* dL_dsigma, float* g_v0_dev) {
  if (!S) return MDLG_E_INVALID;
  const Layout& L = S->L;
  if (L.adj_ckpts == 0) {
    S->last_error = "the configuration reserved no adjoint buffers (adjoint_window = 0)";
    return MDLG_E_STATE;
  }
  if (W < 1 || k < 1 || W % k != 0 || W / k + 1 > L.adj_ckpts || k + 1 > L.adj_seg ||
      W > S->cfg.adjoint_window) {
    S->last_error = "adjoint window/checkpoint interval outside the reserved sizes";
    return MDLG_E_INVALID;
  }
  if (loss != MDLG_LOSS_MSD && loss != MDLG_LOSS_MEAN_X) {
    S->last_error = "unknown loss";
    return MDLG_E_INVALID;
  }
  // start of the window: canonical cells (frozen from here on), and the
  // caller's v0 (id order) if given
  if (S->since_sort != 0) enqueue_sort(S);
  if (v0_dev) {
    AdjIoArgs io{S->id[S->scur], S->vel[S->scur], const_cast<float*>(v0_dev), (int)L.n_total, 1};
    launch_adj_io(S->D, io, S->stream);
    S->vel_full = true;
  }
  const bool want_g = g_v0_dev != nullptr;
  int gbuf = 0;  // the adjoint buffer that receives dL/dv0 in id order
  if (!S->use_graph || S->timing) {
    gbuf = enqueue_adjoint(S, W, k, loss, want_g);
  } else {
    // one graph per window shape and loss (no caller pointer inside it)
    const unsigned long long tag = ((unsigned long long)W << 40) | ((unsigned long long)k << 20) |
                                   ((unsigned long long)loss << 1) | (want_g ? 1ull : 0ull);
    mdlg_status gs = replay_graph(S, kAdjointGraph, [&] { gbuf = enqueue_adjoint(S, W, k, loss, want_g); },
                                  tag);
    if (gs != MDLG_OK) return gs;
    // (the buffer index follows from W and k alone)
    gbuf = adjoint_grad_buffer(W);
  }
  if (want_g) launch_copy_f32(S->adj_lv[gbuf], g_v0_dev, L.n_total * S->D, S->stream);
  S->snapshot_valid = false;
  mdlg_status st = check_launch(S, "mdlg_adjoint");
  if (st != MDLG_OK) return st;
  double out[3] = {0, 0, 0};
  HIPCHK(S, hipMemcpyAsync(out, S->adj_out, sizeof out, hipMemcpyDeviceToHost, S->stream));
  st = read_err(S);
  if (out_loss) *out_loss = out[0];
  if (dL_deps) *dL_deps = out[1];
  if (dL_dsigma) *dL_dsigma = out[2];
  return st;
}


// The device work of mdlg_adjoint (arguments checked; the cells canonical and
// v0, if given, in place): the forward window with checkpoints, the loss,
// the reverse sweep segment by segment, the gradient reductions, dL/dv0 in id
// order into the other adjoint velocity buffer (want_g), and the rebuild at
// the end of the window.  Returns that buffer's index.
static int enqueue_adjoint(mdlg_system* S, int32_t W, int32_t k, int32_t loss, bool want_g) {
  const Layout& L = S->L;
  const int D = S->D;
  const long long nd = L.n_total * D;
  const Phys PW = window_phys(S);
  // the window's force launches (forward and recomputed) walk pair lists
  // built here on the frozen cells
  const Phys PF = L.kmax_adj > 0 ? window_list_phys(S) : PW;
  S->adj_window_steps = W;
  if (PF.kmax > 0) enqueue_nlist(S, PF);
  // Forward window.  x(0) goes to checkpoint 0 (the loss and the
  // recomputation of segment 0 read it there); each later checkpoint
  // position, and every position of the last segment, is written there by
  // the step that makes it (the last segment is not recomputed: the reverse
  // sweep reads its positions from the segment buffer, and x(W) from the
  // state).  The first step writes the full-step v(0) into checkpoint 0 (a
  // half-step state is completed by that step's kick, as a finishing launch
  // would), and later checkpoints copy the velocities.
  const int last0 = W - k;  // first position of the last segment
  float* x0 = S->adj_ckpt_pos;
  launch_copy_f32(S->pos[S->pcur], x0, nd, S->stream);
  const float* cur_pos = S->pos[S->pcur];
  for (int n = 1; n <= W; ++n) {
    float* pout;
    if (n == W) pout = S->pos[S->pcur ^ 1];
    else if (n >= last0) pout = S->adj_seg_pos + (size_t)(n - last0) * nd;
    else if (n % k == 0) pout = S->adj_ckpt_pos + (size_t)(n / k) * nd;
    else pout = S->pos[S->pcur ^ 1];
    const int mode = (n == 1 && S->vel_full) ? kModeStart : kModeStep;
    launch_force_raw(S, PF, mode, cur_pos, pout, S->vel[S->scur], n - 1,
                     n == 1 ? S->adj_ckpt_vel : nullptr);
    S->pcur ^= 1;
    cur_pos = pout;
    if (n % k == 0 && n < last0)
      launch_copy_f32(S->vel[S->scur], S->adj_ckpt_vel + (size_t)(n / k) * nd, nd, S->stream);
  }
  S->vel_full = false;
  // loss and dL/dx(W); lam_v(W) = 0
  const int nlb = (int)std::min<long long>(1024, (L.n_total + kBlock - 1) / kBlock);
  const float* xW = S->pos[S->pcur];
  AdjLossArgs la{x0, xW, S->adj_lx, S->adj_lv[0], S->adj_lpart, (int)L.n_total, loss, nlb};
  launch_adj_loss(D, la, S->stream);
  // Reverse sweep, segment by segment.  The segments before the last are
  // recomputed from their checkpoints (their velocities run in place in the
  // checkpoint, used only here), each during the sweep over the segment
  // after it: recomputation step i of segment seg - 1 goes in the same
  // launch as reverse step k + 1 - i of segment seg, so that the force
  // step, which depends on nothing the reverse steps write, costs no launch
  // of its own.  The last segment's positions are in segment buffer 0 (the
  // forward window wrote them); the recomputed segments alternate between
  // the two buffers, so that a segment is recomputed into the buffer the
  // sweep left one segment earlier.
  const float h = (float)S->cfg.dt;
  const double u = PW.u_d;
  const double e1 = 24.0 * S->cfg.epsilon / (S->cfg.mass * u);
  const int nseg = W / k;
  float* segbuf[2] = {S->adj_seg_pos, S->adj_seg_pos2};
  auto buf_of = [&](int seg) { return segbuf[(nseg - 1 - seg) & 1]; };
  int cur = 0;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const bool last = seg == nseg - 1;
    const float* seg0 = S->adj_ckpt_pos + (size_t)seg * nd;  // x at the segment's start
    float* buf = buf_of(seg);
    float* nbuf = seg > 0 ? buf_of(seg - 1) : nullptr;  // the previous segment's, being recomputed
    const float* nseg0 = seg > 0 ? S->adj_ckpt_pos + (size_t)(seg - 1) * nd : nullptr;
    for (int j = k; j >= (seg == 0 ? 0 : 1); --j) {
      const int sg = seg * k + j;
      AdjArgs a{};
      a.P = PW;
      a.reps = S->reps;
      a.bricks = S->bricks;
      a.cell_start = S->cell_start;
      a.pos = (last && j == k) ? xW : (j == 0 ? seg0 : buf + (size_t)j * nd);
      a.lam_v_in = S->adj_lv[cur];
      a.lam_v_out = S->adj_lv[cur ^ 1];
      a.lam_x = S->adj_lx;
      // (each reverse step writes its own row of partials: no read-modify-write)
      a.gpart = S->adj_gpart + (size_t)(W - sg) * L.nbricks * 2;
      a.c = (sg == W || sg == 0) ? 0.5f * h : h;
      a.drift = sg > 0 ? 1 : 0;
      a.e1_over_sigma = (float)(e1 / S->cfg.sigma);
      a.e2 = (float)(e1 / u);
      a.eps = S->cfg.epsilon;
      a.nbricks = L.nbricks;
      a.err = S->err;
      if (PF.kmax > 0) {
        a.smap = S->smap;
        a.binfo = S->binfo;
        a.trec = S->trec;
        a.nl = S->nl;
        a.lcap_list = PF.lcap;
        a.stale = S->stale + W;
      }
      if (seg > 0) {
        const int i = k + 1 - j;  // recomputation step of segment seg - 1
        AdjForceArgs af{};
        af.adj = a;
        af.force = force_args_raw(S, PF, (seg == 1 && i == 1) ? kModeStart : kModeStep,
                                  i == 1 ? nseg0 : nbuf + (size_t)(i - 1) * nd, nbuf + (size_t)i * nd,
                                  S->adj_ckpt_vel + (size_t)(seg - 1) * nd, -1, nullptr);
        af.force.xcd_remap = 0;
        TimedLaunch t(S, MDLG_K_ADJOINT_FORCE);
        launch_adjoint_force(D, af, S->stream);
      } else {
        TimedLaunch t(S, MDLG_K_ADJOINT);
        launch_adjoint(D, a, S->stream);
      }
      cur ^= 1;
    }
  }
  AdjFinalArgs fa{S->adj_lpart, S->adj_gpart, S->adj_out, nlb, (W + 1) * L.nbricks};
  launch_adj_final(fa, S->stream);
  if (want_g) {
    // dL/dv0 in id order into the buffer the sweep no longer needs
    AdjIoArgs io{S->id[S->scur], S->adj_lv[cur], S->adj_lv[cur ^ 1], (int)L.n_total, 0};
    launch_adj_io(D, io, S->stream);
  }
  // leave the system at the end of the window, cells rebuilt
  S->vel_full = false;
  S->since_sort = W;
  S->md_step += W;
  enqueue_sort(S);
  S->snapshot_valid = false;
  return cur ^ 1;
}

mdlg_status mdlg_get_list_fallbacks(mdlg_system* S, int64_t* launches) {
  if (!S || !launches) return MDLG_E_INVALID;
  unsigned long long v = 0;
  if (S->fallbacks) {
    HIPCHK(S, hipMemcpyAsync(&v, S->fallbacks, sizeof v, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(S, hipStreamSynchronize(S->stream));
  }
  *launches = (int64_t)v;
  return read_err(S);
}

mdlg_status mdlg_checkpoint_bytes(mdlg_system* S, size_t* bytes) {
  if (!S || !bytes) return MDLG_E_INVALID;
  *bytes = ckpt_bytes(S);
  return MDLG_OK;
}

mdlg_status mdlg_checkpoint_save(mdlg_system* S, void* blob, size_t bytes) {
  if (!S || !blob) return MDLG_E_INVALID;
  const size_t need = ckpt_bytes(S);
  if (bytes < need) {
    S->last_error = "checkpoint buffer too small: need " + std::to_string(need) + " bytes";
    return MDLG_E_NOMEM;
  }
  mdlg_status st = read_err(S);  // synchronises; a failed run is not saved
  if (st != MDLG_OK) return st;
  const bool lists = ckpt_lists(S);
  CkptHeader h{};
  std::memcpy(h.magic, kCkptMagic, sizeof h.magic);
  h.fingerprint = fingerprint(S);
  h.bytes = need;
  h.pcur = S->pcur;
  h.scur = S->scur;
  h.since_sort = S->since_sort;
  h.vel_full = S->vel_full ? 1 : 0;
  h.mpar = S->mpar;
  h.xi_par = S->xi_par;
  h.xi_have = S->xi_have ? 1 : 0;
  h.snapshot_valid = S->snapshot_valid ? 1 : 0;
  h.has_lists = lists ? 1 : 0;
  h.md_step = S->md_step;
  h.n_lattice = S->n_lattice;
  h.xi_steps = S->xi_steps;
  char* out = static_cast<char*>(blob);
  std::memcpy(out, &h, sizeof h);
  size_t off = sizeof h;
  for (const Region& r : ckpt_regions(S, lists)) {
    HIPCHK(S, hipMemcpyAsync(out + off, r.dev, r.bytes, hipMemcpyDeviceToHost, S->stream));
    off += r.bytes;
  }
  HIPCHK(S, hipStreamSynchronize(S->stream));
  return MDLG_OK;
}

mdlg_status mdlg_checkpoint_load(mdlg_system* S, const void* blob, size_t bytes) {
  if (!S || !blob) return MDLG_E_INVALID;
  CkptHeader h{};
  if (bytes < sizeof h) {
    S->last_error = "checkpoint blob too short";
    return MDLG_E_INVALID;
  }
  std::memcpy(&h, blob, sizeof h);
  if (std::memcmp(h.magic, kCkptMagic, sizeof h.magic) != 0) {
    S->last_error = "not an MDLG checkpoint";
    return MDLG_E_INVALID;
  }
  if (h.fingerprint != fingerprint(S)) {
    S->last_error = "checkpoint was taken with a different configuration";
    return MDLG_E_INVALID;
  }
  if (h.bytes != bytes || h.pcur < 0 || h.pcur > 1 || h.scur < 0 || h.scur > 1 || h.mpar < 0 ||
      h.mpar > 1 || h.xi_par < 0 || h.xi_par > 1 || h.since_sort < 0 ||
      h.since_sort >= std::max(1, S->L.sort_every) ||
      (h.has_lists != 0) != (S->L.kmax > 0 && h.since_sort > 0)) {
    S->last_error = "checkpoint header is inconsistent";
    return MDLG_E_INVALID;
  }
  // wait for queued work before overwriting the state
  HIPCHK(S, hipStreamSynchronize(S->stream));
  S->pcur = h.pcur;
  S->scur = h.scur;
  S->since_sort = h.since_sort;
  S->vel_full = h.vel_full != 0;
  S->mpar = h.mpar;
  S->xi_par = h.xi_par;
  S->xi_have = h.xi_have != 0;
  S->snapshot_valid = h.snapshot_valid != 0;
  S->md_step = h.md_step;
  S->n_lattice = h.n_lattice;
  S->xi_steps = h.xi_steps;
  S->first_sort = false;
  const char* in = static_cast<const char*>(blob);
  size_t off = sizeof h;
  for (const Region& r : ckpt_regions(S, h.has_lists != 0)) {
    HIPCHK(S, hipMemcpyAsync(r.dev, in + off, r.bytes, hipMemcpyHostToDevice, S->stream));
    off += r.bytes;
  }
  launch_fill_u32(S->err, 0u, 64, S->stream);
  // the arrival counters the next rebuild uses start at zero
  launch_fill_u32(S->mcnt[S->mpar], 0u, S->L.n_cells * arrival_words(S->D), S->stream);
  if (S->L.kmax > 0 && h.has_lists == 0) enqueue_nlist(S, S->P);
  mdlg_status st = check_launch(S, "mdlg_checkpoint_load");
  if (st != MDLG_OK) return st;
  HIPCHK(S, hipStreamSynchronize(S->stream));
  return read_err(S);
}

mdlg_status mdlg_set_potential(mdlg_system* S, double epsilon, double sigma) {
  if (!S) return MDLG_E_INVALID;
  if (!(epsilon > 0) || !(sigma > 0) || !std::isfinite(epsilon) || !std::isfinite(sigma)) {
    S->last_error = "epsilon and sigma must be > 0";
    return MDLG_E_INVALID;
  }
  S->cfg.epsilon = epsilon;
  S->cfg.sigma = sigma;
  S->P = make_phys(&S->cfg, S->L);
  // captured lattice steps carry the old parameters
  HIPCHK(S, hipStreamSynchronize(S->stream));
  for (auto& kv : S->graphs) (void)hipGraphExecDestroy(kv.second.exec);
  S->graphs.clear();
  return MDLG_OK;
}

mdlg_status mdlg_set_timing(mdlg_system* S, int enable) {
  if (!S) return MDLG_E_INVALID;
  HIPCHK(S, hipStreamSynchronize(S->stream));
  drain_timing(S);
  for (int i = 0; i < MDLG_K_NCLASS; ++i) {
    S->timed_ms[i] = 0.0;
    S->timed_n[i] = 0;
  }
  S->timing = enable != 0;
  return MDLG_OK;
}

mdlg_status mdlg_get_timing(mdlg_system* S, double* total_ms, int64_t* launches) {
  if (!S) return MDLG_E_INVALID;
  HIPCHK(S, hipStreamSynchronize(S->stream));
  drain_timing(S);
  for (int i = 0; i < MDLG_K_NCLASS; ++i) {
    if (total_ms) total_ms[i] = S->timed_ms[i];
    if (launches) launches[i] = S->timed_n[i];
  }
  return read_err(S);
}

mdlg_status mdlg_timing_offset(mdlg_system* S, int reps, double* offset_ms) {
  if (!S || !offset_ms || reps < 1 || reps > 1000) return MDLG_E_INVALID;
  int dev = 0, khz = 0;
  HIPCHK(S, hipGetDevice(&dev));
  HIPCHK(S, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) {
    S->last_error = "device reports no wall clock rate";
    return MDLG_E_DEVICE;
  }
  // a wait of about 20 microseconds on the device's wall clock
  const long long ticks = std::max(1LL, (long long)std::llround(0.02 * khz));
  const double span_ms = (double)ticks / (double)khz;
  HIPCHK(S, hipStreamSynchronize(S->stream));
  drain_timing(S);
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  for (int r = 0; r < reps; ++r) {
    hipEvent_t a = pool_event(S), b = pool_event(S);
    if (!a || !b) {
      if (a) S->event_pool.push_back(a);
      if (b) S->event_pool.push_back(b);
      break;
    }
    ev.emplace_back(a, b);
    launch_clock_wait(ticks, S->stream, a, b);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
  std::vector<double> d;
  for (auto& p : ev) {
    float ms = 0.f;
    if (e == hipSuccess && hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess)
      d.push_back((double)ms - span_ms);
    S->event_pool.push_back(p.first);
    S->event_pool.push_back(p.second);
  }
  if (e != hipSuccess) return hip_fail(S, e, "clock wait");
  if (d.empty()) {
    S->last_error = "no event pair could be timed";
    return MDLG_E_DEVICE;
  }
  std::sort(d.begin(), d.end());
  *offset_ms = d[d.size() / 2];
  return MDLG_OK;
}

mdlg_status mdlg_timing_head_start(mdlg_system* S, double microseconds) {
  if (!S || !(microseconds >= 0.0) || microseconds > 1e6) return MDLG_E_INVALID;
  int dev = 0, khz = 0;
  HIPCHK(S, hipGetDevice(&dev));
  HIPCHK(S, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) {
    S->last_error = "device reports no wall clock rate";
    return MDLG_E_DEVICE;
  }
  launch_clock_wait((long long)std::llround(microseconds * 1e-3 * khz), S->stream, nullptr, nullptr);
  return check_launch(S, "clock wait");
}

mdlg_status mdlg_sync(mdlg_system* S) {
  if (!S) return MDLG_E_INVALID;
  return read_err(S);
}

const char* mdlg_last_error(const mdlg_system* S) {
  return S ? S->last_error.c_str() : g_create_error.c_str();
}

void mdlg_destroy(mdlg_system* S) {
  if (!S) return;
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  for (auto& kv : S->graphs) (void)hipGraphExecDestroy(kv.second.exec);
  drain_timing(S);
  for (hipEvent_t e : S->event_pool) (void)hipEventDestroy(e);
  if (S->cap_stream) (void)hipStreamDestroy(S->cap_stream);
  if (S->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static[S->static_dev].in_use = false;
  }
  delete S;
}

}  // extern "C"
