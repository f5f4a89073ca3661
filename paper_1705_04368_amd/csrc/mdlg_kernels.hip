// HIP kernels of the MDLG hot path for gfx950 (wave64).
//
// Particle state lives in HBM as structure-of-arrays sorted by MD cell:
//   pos  float[N][D]  offset of the particle inside its MD cell (side s)
//   vel  float[N][D]  velocity (half-step or full-step, see StepMode)
//   img  int  [N][D]  periodic image counters
//   id   int  [N]     particle id (index in the input)
//   cell int  [N]     global MD-cell index at the last rebuild
// MD cells of side s = dx / k tile every replica's box; cell_start[c] is the
// first particle of cell c after the last counting sort.  Between rebuilds a
// particle may leave its cell by at most the rebuild margin, which the force
// stencil covers.
//
// Kernels:
//   k_ingest   absolute positions -> (cell, offset), unsorted
//   k_count    canonicalise (cell, offset, image) and count particles per cell
//   k_scan     exclusive scan of the counts into cell_start
//   k_scatter  permutation of the state into cell order (slots fixed by the
//              old order: deterministic)
//   k_cellsort first rebuild of an input in arbitrary order: cells by id
//   k_rescale  thermostat rescale of the velocities
//   k_nlist_narrow / k_nlist_wide    pair lists of radius r_cut + 2 skin
//              per brick at each rebuild (14-bit candidate tests), with the
//              staging map and target order the force kernel follows
//   k_force    LJ forces with the neighbour cells of a brick staged in LDS
//              (pair lists, or the cell walk), fused with the velocity-Verlet
//              half kicks and the drift
//   k_shift    binning on displaced and moving lattices
//   k_bin      MDLG binning (eq. MDni): lattice velocity from the unwrapped
//              lattice cells at t and at the previous snapshot, LDS histogram
//              per site strip with wave-aggregated atomics, flush to HBM
//   k_xi / k_xi_reduce               collision operator (eq. Xi)
//   k_adjoint / k_adj_loss / k_adj_final / k_adj_io   reverse velocity Verlet
//   k_fsum / k_ffinal / k_site_avg   f_i^eq readout (eq. fieq)
//   k_kin      FP64 momentum / kinetic energy per replica, thermostat factor
//   k_export / k_import              state in id order
//   k_clock_wait                     a wait of known length on the device's
//              wall clock (timing aid: the event pairs' own excess, and a
//              head start for an event-timed pass)
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "mdlg_args.h"

namespace mdlg {

// ---------------------------------------------------------------- helpers

template <int D>
__device__ __forceinline__ void ldv(const float* __restrict__ p, int g, float (&v)[D]) {
  if constexpr (D == 2) {
    const float2 t = reinterpret_cast<const float2*>(p)[g];
    v[0] = t.x;
    v[1] = t.y;
  } else {
    const float* q = p + 3 * (size_t)g;
    v[0] = q[0];
    v[1] = q[1];
    v[2] = q[2];
  }
}

template <int D>
__device__ __forceinline__ void stv(float* __restrict__ p, int g, const float (&v)[D]) {
  if constexpr (D == 2) {
    reinterpret_cast<float2*>(p)[g] = make_float2(v[0], v[1]);
  } else {
    float* q = p + 3 * (size_t)g;
    q[0] = v[0];
    q[1] = v[1];
    q[2] = v[2];
  }
}

template <int D>
__device__ __forceinline__ void ldi(const int* __restrict__ p, int g, int (&v)[D]) {
  if constexpr (D == 2) {
    const int2 t = reinterpret_cast<const int2*>(p)[g];
    v[0] = t.x;
    v[1] = t.y;
  } else {
    const int* q = p + 3 * (size_t)g;
    v[0] = q[0];
    v[1] = q[1];
    v[2] = q[2];
  }
}

template <int D>
__device__ __forceinline__ void sti(int* __restrict__ p, int g, const int (&v)[D]) {
  if constexpr (D == 2) {
    reinterpret_cast<int2*>(p)[g] = make_int2(v[0], v[1]);
  } else {
    int* q = p + 3 * (size_t)g;
    q[0] = v[0];
    q[1] = v[1];
    q[2] = v[2];
  }
}

__device__ __forceinline__ int wrap_cell(int c, int m) {
  return c < 0 ? c + m : (c >= m ? c - m : c);
}

__device__ __forceinline__ int floor_div(int a, int b) {
  int q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

template <int D>
__device__ __forceinline__ void cell_coords(int local, const Replica& R, int (&c)[D]) {
  const int q = div_magic(local, R.dmul[0], R.dsh[0]);
  c[0] = local - q * R.Mc[0];
  if constexpr (D == 2) {
    c[1] = q;
  } else {
    const int q2 = div_magic(q, R.dmul[1], R.dsh[1]);
    c[1] = q - q2 * R.Mc[1];
    c[2] = q2;
  }
}

template <int D>
__device__ __forceinline__ int cell_linear(const int (&c)[D], const Replica& R) {
  if constexpr (D == 2)
    return c[0] + R.Mc[0] * c[1];
  else
    return c[0] + R.Mc[0] * (c[1] + R.Mc[1] * c[2]);
}

// Bring an offset back into [0, s) by moving at most one cell, carrying the
// wrap of the cell index into the image counter.  o - s is exact for o in
// [s, 2s) (Sterbenz); when o + s rounds up to s the particle sits on the
// boundary and stays in its cell with offset 0.  Returns false for a jump of
// more than one cell or a non-finite offset (indices stay in range anyway).
__device__ __forceinline__ bool canon(float& o, int& c, int& im, int mc, float s) {
  if (o < 0.f) {
    o = o + s;
    c -= 1;
    if (o >= s) {
      o = 0.f;
      c += 1;
    }
  } else if (o >= s) {
    o = o - s;
    c += 1;
  }
  const bool ok = (o >= 0.f) && (o < s);
  if (c < 0) {
    c += mc;
    im -= 1;
  } else if (c >= mc) {
    c -= mc;
    im += 1;
  }
  return ok;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Exclusive scan of one int per thread over the block; *total gets the sum.
template <int NW = kWaves>
__device__ __forceinline__ int block_excl_scan(int v, int* s_tmp, int* total) {
  const int lane = lane_id(), w = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) s_tmp[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < NW; ++i) {
      int t = s_tmp[i];
      s_tmp[i] = run;
      run += t;
    }
    s_tmp[NW] = run;
  }
  __syncthreads();
  const int excl = incl - v + s_tmp[w];
  *total = s_tmp[NW];
  __syncthreads();
  return excl;
}

__device__ __forceinline__ int block_sum(int v, int* s_tmp) {
  int total;
  (void)block_excl_scan(v, s_tmp, &total);
  return total;
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Add 1 per valid lane to base[key], one LDS/global atomic per distinct key of
// the wave (lanes of a wave mostly share keys because particles are sorted).
__device__ __forceinline__ void wave_agg_add(unsigned* base, int key, bool valid) {
  unsigned long long act = __ballot(valid);
  while (act) {
    const int leader = __ffsll((long long)act) - 1;
    const int lk = __builtin_amdgcn_readlane(key, leader);
    const unsigned long long same = __ballot(valid && key == lk) & act;
    if (lane_id() == leader) atomicAdd(base + lk, (unsigned)__popcll(same));
    act &= ~same;
  }
}

__device__ __forceinline__ void wave_agg_add_i(int* base, int key, bool valid) {
  unsigned long long act = __ballot(valid);
  while (act) {
    const int leader = __ffsll((long long)act) - 1;
    const int lk = __builtin_amdgcn_readlane(key, leader);
    const unsigned long long same = __ballot(valid && key == lk) & act;
    if (lane_id() == leader) atomicAdd(base + lk, (int)__popcll(same));
    act &= ~same;
  }
}

// ---------------------------------------------------------------- utilities

__global__ void k_fill_u32(unsigned* __restrict__ p, unsigned v, long long n) {
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    p[i] = v;
}

__global__ void k_fill_f32(float* __restrict__ p, float v, long long n) {
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    p[i] = v;
}

// ---------------------------------------------------------------- ingest

template <int D>
__global__ __launch_bounds__(kBlock) void k_ingest(IngestArgs a) {
  const int4 ch = a.chunks[blockIdx.x];
  const Replica R = a.reps[ch.x];
  for (int g = ch.y + threadIdx.x; g < ch.z; g += kBlock) {
    float x[D], v[D], o[D];
    int c[D], im[D];
    ldv<D>(a.pos_abs, g, x);
    ldv<D>(a.vel_in, g, v);
    bool ok = true;
    for (int k = 0; k < D; ++k) {
      float q = floorf(x[k] * a.P.inv_s);
      int ci = (q >= 0.f && q < (float)R.Mc[k]) ? (int)q : 0;
      ok = ok && (q >= 0.f && q < (float)R.Mc[k]);
      o[k] = x[k] - (float)ci * a.P.s;
      im[k] = 0;
      c[k] = ci;
      ok = canon(o[k], c[k], im[k], R.Mc[k], a.P.s) && ok;
      ok = ok && isfinite(v[k]);
    }
    if (!ok) atomicOr(a.err, kErrJump);
    stv<D>(a.pos, g, o);
    stv<D>(a.vel, g, v);
    sti<D>(a.img, g, im);
    a.id[g] = g;
    a.cell[g] = R.cell_off + cell_linear<D>(c, R);
  }
}

// ---------------------------------------------------------------- counting sort

// Deterministic counting sort.  Between rebuilds a particle leaves its cell
// by less than one cell, so a rebuild moves it by a step d_a in {-1, 0, 1}
// along every axis, numbered dir = sum_a (d_a + 1) 3^a (kStay: no move).  In
// its new cell c the particles are ordered: first those that stayed in c, in
// their old order; then the arrivals, by direction (all arrivals from one
// direction come from a single old cell) and within one direction in their
// old order.  Every slot is then a function of the old order alone, never of
// the order in which atomics land, so two runs from one state are identical
// bit for bit.  The count pass records per particle its key, its direction and
// lrank, its rank among the particles of its old cell that moved the same
// way; per cell it counts all particles and, in one byte per direction, the
// arrivals.  The scatter places stayers at cell_start[c] + lrank and an
// arrival after every stayer and every arrival from a lower direction.
template <int D>
constexpr int kDirs = (D == 2) ? 9 : 27;
template <int D>
constexpr int kStay = (kDirs<D> - 1) / 2;
// words of arrival counters per cell: the exact number of arrivals, then one
// byte per direction but kStay (a byte that wrapped makes the bytes' sum
// differ from the exact count, which the scatter checks)
template <int D>
constexpr int kArrWords = 1 + (kDirs<D> - 1 + 3) / 4;

// Canonical (cell, offset, image) of a particle from its stored offset o,
// image im and old cell oc (global index); dir receives the rebuild step.
template <int D>
__device__ __forceinline__ bool canon_state(const Replica& R, float s, int oc, float (&o)[D],
                                            int (&c)[D], int (&im)[D], int& dir) {
  cell_coords<D>(oc - R.cell_off, R, c);
  bool ok = true;
  int dd = 0, p3 = 1;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int c0 = c[k];
    ok = canon(o[k], c[k], im[k], R.Mc[k], s) && ok;
    int d = c[k] - c0;
    if (d > 1) d -= R.Mc[k];
    else if (d < -1) d += R.Mc[k];
    dd += (d + 1) * p3;
    p3 *= 3;
  }
  dir = dd;
  return ok;
}

template <int D>
__device__ __forceinline__ bool canon_particle(const SortArgs& a, const Replica& R, int g,
                                               float (&o)[D], int (&c)[D], int (&im)[D],
                                               int* oldcell = nullptr, int* dir = nullptr) {
  ldv<D>(a.pos, g, o);
  ldi<D>(a.img, g, im);
  const int oc = a.cell[g];
  cell_coords<D>(oc - R.cell_off, R, c);
  bool ok = true;
  int dd = 0, p3 = 1;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int c0 = c[k];
    ok = canon(o[k], c[k], im[k], R.Mc[k], a.P.s) && ok;
    // the step, with the periodic wrap undone (at least three cells per axis)
    int d = c[k] - c0;
    if (d > 1) d -= R.Mc[k];
    else if (d < -1) d += R.Mc[k];
    dd += (d + 1) * p3;
    p3 *= 3;
  }
  if (oldcell) *oldcell = oc;
  if (dir) *dir = dd;
  return ok;
}

// Arrival field of a direction other than kStay.
template <int D>
__device__ __forceinline__ int arrival_field(int dir) {
  return dir < kStay<D> ? dir : dir - 1;
}

// Counts and ranks.  Per-cell totals go through a block-local LDS histogram
// over a window of new cells (the chunk's old cells widened by one row on
// either side), one global atomic per distinct cell; keys outside the window
// (moves along z in 3D) take one global atomic each.  Scan-tile totals are
// summed in LDS first: same-address global atomics serialise across the
// device.  The ranks need the directions of the chunk's particles (LDS) and of
// the particles of the chunk's first old cell that precede the chunk.  With
// `first` (input in arbitrary order) slots come from global atomics and the
// ranks are skipped: k_cellsort orders the cells afterwards.
// (eight waves per SIMD: the 2D instance otherwise takes 76 VGPRs and six)
template <int D>
__global__ __attribute__((amdgpu_flat_work_group_size(1, kBlock), amdgpu_waves_per_eu(8))) void k_count(SortArgs a) {
  constexpr int kHist = 2048;
  constexpr int kPer = kCountChunkMax / kBlock;
  // scan-tile totals of the block: the window's tiles and those a particle
  // moving by one cell along the slowest axis reaches
  constexpr int kTiles = 64;
  // particles of the chunk's first old cell that lie before the chunk
  constexpr int kPrev = kBlock;
  __shared__ int s_cnt[kHist];
  __shared__ int s_tile[kTiles];
  __shared__ unsigned char s_dir[kCountChunkMax];
  __shared__ int s_oc[kCountChunkMax];
  __shared__ unsigned char s_pdir[kPrev];
  __shared__ int s_p0;
  // consecutive chunks on one XCD: the per-cell count atomics of neighbouring
  // chunks then meet in one L2 instead of crossing XCDs
  int cb = blockIdx.x;
  if (a.xcd_remap) {
    const int per = gridDim.x >> 3;
    cb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  }
  if (cb >= a.ncchunks) return;
  // scan-tile totals go to the copy of this block's XCD (consecutive blocks
  // alternate XCDs): same-address atomics from many blocks serialise
  int* __restrict__ tsum = a.tile_sum + (size_t)(blockIdx.x & (kTileCopies - 1)) * a.ntiles;
  const int4 ch = a.cchunks[cb];
  const Replica R = a.reps[ch.x];
  // window: the chunk's old cells (sorted) widened by one row on either side
  const int lo = a.cell[ch.y] - R.Mc[0] - 1;
  const int nwin = a.first ? 0 : min(kHist, a.cell[ch.z - 1] + R.Mc[0] + 2 - lo);
  for (int i = threadIdx.x; i < nwin; i += kBlock) s_cnt[i] = 0;
  if (threadIdx.x < kTiles) s_tile[threadIdx.x] = 0;
  // (the reach below the window is capped so that the window's own tiles
  // always index inside s_tile: (16 + 2) tiles + 2 < kTiles)
  const int layer = min((D == 3) ? R.Mc[0] * R.Mc[1] : R.Mc[0], 16 * kScanTile);
  const int tile0 = max(0, lo - layer) / kScanTile;
  __syncthreads();
  int key[kPer], dir[kPer];
  // the particles' state is loaded kLoad at a time before any of it is used
  // (the counting atomics below would otherwise keep the loads apart); the
  // groups tile the thread's kPer particles exactly
  constexpr int kLoad = kPer < 8 ? kPer : 8;
  static_assert(kPer % kLoad == 0, "load groups must tile a thread's particles");
#pragma unroll
  for (int u0 = 0; u0 < kPer; u0 += kLoad) {
    float o[kLoad][D];
    int im[kLoad][D], oc[kLoad];
#pragma unroll
    for (int v = 0; v < kLoad; ++v) {
      const int g = ch.y + (u0 + v) * kBlock + (int)threadIdx.x;
      if (g < ch.z) {
        ldv<D>(a.pos, g, o[v]);
        ldi<D>(a.img, g, im[v]);
        oc[v] = a.cell[g];
      }
    }
#pragma unroll
    for (int v = 0; v < kLoad; ++v) {
      const int u = u0 + v;
      const int g = ch.y + u * kBlock + (int)threadIdx.x;
      key[u] = -1;
      dir[u] = kStay<D>;
      if (ch.y + u * kBlock >= ch.z) continue;  // the chunk is shorter (uniform)
      bool inwin = false;
      if (g < ch.z) {
        int c[D];
        if (!canon_state<D>(R, a.P.s, oc[v], o[v], c, im[v], dir[u])) atomicOr(a.err, kErrJump);
        key[u] = R.cell_off + cell_linear<D>(c, R);
        s_dir[g - ch.y] = (unsigned char)dir[u];
        s_oc[g - ch.y] = oc[v];
        if (a.first) {
          a.keyslot[g] = make_int2(key[u], atomicAdd(a.count + key[u], 1));
        } else {
          inwin = key[u] >= lo && key[u] < lo + nwin;
          if (inwin) atomicAdd(&s_cnt[key[u] - lo], 1);
          else atomicAdd(a.count + key[u], 1);
        }
      }
      if (key[u] >= 0 && !inwin) {
        const int tl = key[u] / kScanTile - tile0;
        if (tl >= 0 && tl < kTiles) atomicAdd(&s_tile[tl], 1);
      }
      const int tk = key[u] >= 0 ? key[u] / kScanTile - tile0 : 0;
      wave_agg_add_i(tsum, key[u] >= 0 ? key[u] / kScanTile : 0,
                     key[u] >= 0 && !inwin && (tk < 0 || tk >= kTiles));
    }
  }
  if (!a.first) {
    // arrivals per cell: the exact count and the direction's byte (no
    // returned values: nothing waits for these)
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      if (key[u] >= 0 && dir[u] != kStay<D>) {
        const int f = arrival_field<D>(dir[u]);
        unsigned* w = a.mcnt + (size_t)key[u] * kArrWords<D>;
        atomicAdd(w, 1u);
        atomicAdd(w + 1 + (f >> 2), 1u << (8u * (unsigned)(f & 3)));
      }
    }
    if (threadIdx.x == 0) {
      // first particle of the chunk's first old cell (the ranks below count
      // the part of that cell before the chunk)
      int p0 = ch.y;
      if (ch.y > R.part_off && a.cell[ch.y - 1] == a.cell[ch.y]) p0 = a.cell_start[a.cell[ch.y]];
      if (ch.y - p0 > kPrev) {
        atomicOr(a.err, kErrOverflow);
        p0 = ch.y - kPrev;
      }
      s_p0 = p0;
    }
  }
  __syncthreads();
  if (!a.first) {
    const int j = s_p0 + (int)threadIdx.x;
    if (j < ch.y) {
      float o[D];
      int c[D], im[D], dd;
      (void)canon_particle<D>(a, R, j, o, c, im, nullptr, &dd);
      s_pdir[j - s_p0] = (unsigned char)dd;
    }
  }
  for (int i = threadIdx.x; i < nwin; i += kBlock) {
    const int c = s_cnt[i];
    if (c) {
      atomicAdd(a.count + lo + i, c);
      atomicAdd(&s_tile[(lo + i) / kScanTile - tile0], c);
    }
  }
  __syncthreads();
  if (threadIdx.x < kTiles && s_tile[threadIdx.x]) atomicAdd(tsum + tile0 + threadIdx.x, s_tile[threadIdx.x]);
  if (a.first) return;
  // rank among the earlier particles of the old cell that moved the same
  // way.  The lanes of a wave hold consecutive particles, so inside the
  // wave the old cell's run and the lanes of the same direction are bit
  // masks; a run that began before the wave adds its earlier part, walked
  // back through the chunk (LDS) and through the part of the chunk's first
  // old cell that lies before the chunk.
  const int p0 = s_p0;
  const int lane = lane_id();
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    if (ch.y + u * kBlock >= ch.z) continue;  // uniform
    const int g = ch.y + u * kBlock + (int)threadIdx.x;
    const bool valid = key[u] >= 0;
    const int l = g - ch.y;
    const int oc = valid ? s_oc[l] : -1;
    // (the chunk's first particle starts a run unless its old cell began in
    // the previous chunk)
    const bool head = valid && (l == 0 ? p0 == ch.y : s_oc[l - 1] != oc);
    const unsigned long long hm = __ballot(head) & (below | (1ull << lane));
    unsigned long long same = 0ull, act = __ballot(valid);
    while (act) {
      const int leader = __ffsll((long long)act) - 1;
      const int ld = __builtin_amdgcn_readlane(dir[u], leader);
      const unsigned long long m = __ballot(valid && dir[u] == ld) & act;
      if (valid && dir[u] == ld) same = m;
      act &= ~m;
    }
    if (!valid) continue;
    int r;
    if (hm) {
      const int rs = 63 - __clzll((long long)hm);
      r = __popcll(same & below & ~((1ull << rs) - 1ull));
    } else {
      r = __popcll(same & below);
      int j = l - lane - 1;
      while (j >= 0 && s_oc[j] == oc) {
        r += (s_dir[j] == dir[u]) ? 1 : 0;
        --j;
      }
      if (j < 0)
        for (int i = 0; i < ch.y - p0; ++i) r += (s_pdir[i] == dir[u]) ? 1 : 0;
    }
    const int code = (dir[u] == kStay<D>) ? r : (r | ((arrival_field<D>(dir[u]) + 1) << 24));
    a.keyslot[g] = make_int2(key[u], code);
  }
}

__global__ __launch_bounds__(kBlock) void k_scan(ScanArgs a) {
  __shared__ int s_tmp[kWaves + 1];
  const int b = blockIdx.x;
  int pre = 0;
  for (int t = threadIdx.x; t < b; t += kBlock)
#pragma unroll
    for (int c = 0; c < kTileCopies; ++c) pre += a.tile_sum[(size_t)c * a.ntiles + t];
  pre = block_sum(pre, s_tmp);
  const int base = b * kScanTile + threadIdx.x * kScanItems;
  int vals[kScanItems];
  int sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int idx = base + i;
    vals[i] = idx < a.n ? a.count[idx] : 0;
    sum += vals[i];
  }
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < a.n) a.count[base + i] = 0;
  int total;
  int run = pre + block_excl_scan(sum, s_tmp, &total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int idx = base + i;
    if (idx < a.n) a.cell_start[idx] = run;
    run += vals[i];
  }
  if (b == a.ntiles - 1 && threadIdx.x == 0) a.cell_start[a.n] = pre + total;
}

// Permutation of the state into the new cell order.  With `first` the slots
// are the atomics' and k_cellsort follows; otherwise a stayer goes to
// cell_start[c] + lrank and an arrival from field f to cell_start[c + 1] -
// (all arrivals) + (arrivals from fields below f) + lrank.  The other
// parity's arrival counters are cleared for the next rebuild.
template <int D>
__global__ __launch_bounds__(kBlock) void k_scatter(SortArgs a) {
  if (blockIdx.x == 0)
    for (int t = threadIdx.x; t < a.ntiles * kTileCopies; t += kBlock) a.tile_sum[t] = 0;
  {
    const long long nw = (long long)a.P.n_cells * kArrWords<D>;
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < nw;
         i += (long long)gridDim.x * kBlock)
      a.mcnt_clear[i] = 0u;
  }
  // consecutive chunks on one XCD: the cache lines where the destinations
  // of neighbouring chunks meet are then completed in one L2
  int cb = blockIdx.x;
  if (a.xcd_remap) {
    const int per = gridDim.x >> 3;
    cb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  }
  if (cb >= a.nchunks) return;
  const int4 ch = a.chunks[cb];
  const Replica R = a.reps[ch.x];
  // every particle of the thread is loaded before any slot is computed: the
  // slot needs the cell start of its key (a dependent load), so the state's
  // loads and that one are the only round trips before the stores
  constexpr int kS = kPartChunkMax / kBlock;
  float o[kS][D], v[kS][D], po[kS][D];
  int im[kS][D], pu[kS][D], oc[kS], pid[kS];
  int2 ks[kS];
#pragma unroll
  for (int q = 0; q < kS; ++q) {
    const int g = ch.y + q * kBlock + (int)threadIdx.x;
    if (g < ch.z) {
      ldv<D>(a.pos, g, o[q]);
      ldi<D>(a.img, g, im[q]);
      oc[q] = a.cell[g];
      ks[q] = a.keyslot[g];
      ldv<D>(a.vel, g, v[q]);
      pid[q] = a.id[g];
      ldi<D>(a.prev_u, g, pu[q]);
      ldv<D>(a.prev_off, g, po[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < kS; ++q) {
    const int g = ch.y + q * kBlock + (int)threadIdx.x;
    if (g >= ch.z) continue;
    int c[D], dd;
    (void)canon_state<D>(R, a.P.s, oc[q], o[q], c, im[q], dd);
    const int key = ks[q].x;
    const int c0 = a.cell_start[key], c1 = a.cell_start[key + 1];
    int dst;
    if (a.first) {
      dst = c0 + ks[q].y;
    } else {
      const int lr = ks[q].y & 0xffffff;
      const int f1 = (int)((unsigned)ks[q].y >> 24);
      if (f1 == 0) {
        dst = c0 + lr;
      } else {
        const unsigned* __restrict__ w = a.mcnt + (size_t)key * kArrWords<D>;
        int tot = 0, pre = 0;
#pragma unroll
        for (int i = 1; i < kArrWords<D>; ++i) {
          const unsigned x = w[i];
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int n = (int)((x >> (8 * b)) & 255u);
            tot += n;
            pre += (4 * (i - 1) + b < f1 - 1) ? n : 0;
          }
        }
        // a wrapped byte: the slots cannot be trusted (reported below)
        dst = (tot == (int)w[0]) ? c1 - tot + pre + lr : -1;
      }
    }
    // a slot outside the cell's range means inconsistent counts (more than
    // 255 arrivals from one direction): reported, and nothing is written out
    // of range
    if (dst < c0 || dst >= c1) {
      atomicOr(a.err, kErrOverflow);
      continue;
    }
    stv<D>(a.pos_out, dst, o[q]);
    stv<D>(a.vel_out, dst, v[q]);
    sti<D>(a.img_out, dst, im[q]);
    a.id_out[dst] = pid[q];
    a.cell_out[dst] = key;
    sti<D>(a.prev_u_out, dst, pu[q]);
    stv<D>(a.prev_off_out, dst, po[q]);
  }
}

// After the first rebuild of an input in arbitrary order: every cell of the
// scattered state ordered by particle id (rank = particles of the cell with a
// smaller id), copied back into the state arrays.  Runs at creation and
// import only.
template <int D>
__global__ __launch_bounds__(kBlock) void k_cellsort(CellsortArgs a) {
  const int4 ch = a.chunks[blockIdx.x];
  for (int g = ch.y + threadIdx.x; g < ch.z; g += kBlock) {
    const int c = a.cell_src[g];
    const int st = a.cell_start[c], en = a.cell_start[c + 1];
    const int me = a.id_src[g];
    int r = 0;
    for (int j = st; j < en; ++j) r += (a.id_src[j] < me) ? 1 : 0;
    const int dst = st + r;
    float o[D], v[D], po[D];
    int im[D], pu[D];
    ldv<D>(a.pos_src, g, o);
    ldv<D>(a.vel_src, g, v);
    ldi<D>(a.img_src, g, im);
    ldi<D>(a.prev_u_src, g, pu);
    ldv<D>(a.prev_off_src, g, po);
    stv<D>(a.pos, dst, o);
    stv<D>(a.vel, dst, v);
    sti<D>(a.img, dst, im);
    a.id[dst] = me;
    a.cell[dst] = c;
    sti<D>(a.prev_u, dst, pu);
    stv<D>(a.prev_off, dst, po);
  }
}

// Thermostat rescale v <- lambda_r v of every particle of replica r.
template <int D>
__global__ __launch_bounds__(kBlock) void k_rescale(RescaleArgs a) {
  const int4 ch = a.chunks[blockIdx.x];
  const float lam = a.lambda[ch.x];
  for (int g = ch.y + threadIdx.x; g < ch.z; g += kBlock) {
    float v[D];
    ldv<D>(a.vel, g, v);
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = lam * v[k];
    stv<D>(a.vel, g, v);
  }
}

// ---------------------------------------------------------------- forces + VV
//
// One block per brick of MD cells.  The brick and a halo of `ns` cells on every
// side are staged in LDS as int32 fixed-point coordinates in the brick frame,
// X = hx * 2^F + rint(off * 2^F / s), so that a pair separation is an exact
// integer difference converted to float once (no per-cell shifts, and no loss
// of precision from large float coordinates).  Each target then visits only the
// cell columns / rows / layers its cutoff sphere (widened by the rebuild
// margin) can reach, reading contiguous LDS ranges row by row.  The LJ sum is
// computed in units of u = s / 2^F; the acceleration comes out in physical
// units because 24 eps / m was divided by u on the host.
//
// The same brick machinery serves the adjoint kernel, which stages the
// adjoint velocity next to the coordinates.

template <int D>
using Coord = typename std::conditional<D == 2, int2, int4>::type;

// The pair-list builder's coarser copy of a staged coordinate: 14-bit values,
// x and y packed in one word (z in a second word in 3D).
template <int D>
using Coord14 = typename std::conditional<D == 2, unsigned, uint2>::type;

// Padding behind the pair-list builder's staged particles: the last test step
// of a row (16 or 32 candidates) may read that far past its end.
constexpr int kNlPad = 32;

// LDS of a brick: the halo cell table and the staged particles live in the
// dynamic shared memory, sized by the host from the brick extent and the
// density (lmaxh halo cells, lcap staged particles per chunk); the small
// arrays are static.
template <int D, bool ADJ, class CT = Coord<D>>
struct BrickLds {
  int* hs;            // LDS start of every halo cell (exclusive scan of counts)
  int* gs;            // global start of every halo cell
  unsigned short* scell;  // halo cell of every staged slot below cap
  CT* p;              // fixed-point coordinates of the staged particles
  float* lam;         // adjoint velocity of the staged particles (ADJ)
  int* rowpre;
  int* tmp;
  double (*red)[4];
  int cap;
};

template <int D, bool ADJ, class CT>
__device__ __forceinline__ BrickLdsLayout brick_lds_layout_dev(const Phys& P, int pad) {
  return brick_lds_layout(P.lcap, pad, sizeof(CT), ADJ ? D * sizeof(float) : 0, P.lmaxh);
}

template <int D, bool ADJ, class CT = Coord<D>>
__device__ __forceinline__ BrickLds<D, ADJ, CT> brick_lds(char* dyn, int* rowpre, int* tmp,
                                                          double (*red)[4], const Phys& P,
                                                          int pad = 0) {
  const BrickLdsLayout lay = brick_lds_layout_dev<D, ADJ, CT>(P, pad);
  BrickLds<D, ADJ, CT> L;
  L.p = reinterpret_cast<CT*>(dyn);
  L.lam = reinterpret_cast<float*>(dyn + lay.lam);
  L.hs = reinterpret_cast<int*>(dyn + lay.hs);
  L.gs = L.hs + P.lmaxh + 1;
  L.scell = reinterpret_cast<unsigned short*>(dyn + lay.scell);
  L.rowpre = rowpre;
  L.tmp = tmp;
  L.red = red;
  L.cap = P.lcap;
  return L;
}

struct BrickGeom {
  int ns, nsz, x0, y0, z0, wx, wy, wz, HX, HY, HZ, nh, total, nrows, ntg;
  float rHX, rHY, rwy;  // reciprocals of HX, HY and wy (small_div)
};

// q = n / d and r = n % d for 0 <= n < 2^20 and 1 <= d < 2^12, from rd ~ 1 / d
// (v_rcp, within two ulp): the float quotient lies within a third of n / d,
// so its truncation is off by at most one either way, which the remainder
// corrects.
__device__ __forceinline__ int small_div(int n, int d, float rd, int& r) {
  int q = (int)((float)n * rd);
  r = n - q * d;
  if (r < 0) {
    q -= 1;
    r += d;
  } else if (r >= d) {
    q += 1;
    r -= d;
  }
  return q;
}

__device__ __forceinline__ int fixed_coord(int h, float off, const Phys& P) {
  return (h << P.F) + __float2int_rn(off * P.fscale);
}

// 14-bit copy of a fixed-point coordinate (which lies above minus one cell):
// shifted up by two cells and truncated to the list builder's coarser unit.
__device__ __forceinline__ unsigned coord14(int x, const Phys& P) {
  return ((unsigned)x + (2u << P.F)) >> P.sh16;
}

__device__ __forceinline__ void put_coord(int2* p, int i, int x, int y, int, const Phys&) {
  p[i] = make_int2(x, y);
}
__device__ __forceinline__ void put_coord(int4* p, int i, int x, int y, int z, const Phys&) {
  p[i] = make_int4(x, y, z, 0);
}
__device__ __forceinline__ void put_coord(unsigned* p, int i, int x, int y, int, const Phys& P) {
  p[i] = coord14(x, P) | (coord14(y, P) << 16);
}
__device__ __forceinline__ void put_coord(uint2* p, int i, int x, int y, int z, const Phys& P) {
  p[i] = make_uint2(coord14(x, P) | (coord14(y, P) << 16), coord14(z, P));
}

// Halo table of a brick: particle count of every halo cell, exclusive scan
// into L.hs (LDS starts), global starts into L.gs, and the prefix of the
// brick's rows of targets into L.rowpre.
template <int D, int NT, class Lds>
__device__ __forceinline__ BrickGeom brick_setup(const Phys& P, const Replica& R, const int4 br,
                                                 const int* __restrict__ cell_start, Lds& L) {
  BrickGeom G;
  G.ns = P.ns;
  G.nsz = (D == 3) ? P.ns : 0;
  G.x0 = br.y * P.BX;
  G.y0 = br.z * P.BY;
  G.z0 = (D == 3) ? br.w * P.BZ : 0;
  G.wx = min(P.BX, R.Mc[0] - G.x0);
  G.wy = min(P.BY, R.Mc[1] - G.y0);
  G.wz = (D == 3) ? min(P.BZ, R.Mc[2] - G.z0) : 1;
  G.HX = G.wx + 2 * G.ns;
  G.HY = G.wy + 2 * G.ns;
  G.HZ = G.wz + 2 * G.nsz;
  G.nh = G.HX * G.HY * G.HZ;
  G.rHX = __builtin_amdgcn_rcpf((float)G.HX);
  G.rHY = __builtin_amdgcn_rcpf((float)G.HY);
  G.rwy = __builtin_amdgcn_rcpf((float)G.wy);
  const int ipt = (G.nh + NT - 1) / NT;
  const int h0 = threadIdx.x * ipt, h1 = min(G.nh, h0 + ipt);
  int mysum = 0;
  for (int h = h0; h < h1; ++h) {
    int hx, hy;
    const int r = small_div(h, G.HX, G.rHX, hx);
    const int hz = small_div(r, G.HY, G.rHY, hy);
    const int cx = wrap_cell(G.x0 - G.ns + hx, R.Mc[0]);
    const int cy = wrap_cell(G.y0 - G.ns + hy, R.Mc[1]);
    const int cz = (D == 3) ? wrap_cell(G.z0 - G.nsz + hz, R.Mc[2]) : 0;
    const int gc = R.cell_off + cx + R.Mc[0] * (cy + R.Mc[1] * cz);
    const int st = cell_start[gc], en = cell_start[gc + 1];
    L.gs[h] = st;
    L.hs[h] = en - st;
    mysum += en - st;
  }
  int run = block_excl_scan<NT / 64>(mysum, L.tmp, &G.total);
  for (int h = h0; h < h1; ++h) {
    const int cnt = L.hs[h];
    L.hs[h] = run;
    // the halo cell of each of its slots (for the staging; slots past the
    // LDS capacity are staged chunk by chunk and search the table instead)
    for (int v = run, ve = min(run + cnt, L.cap); v < ve; ++v) L.scell[v] = (unsigned short)h;
    run += cnt;
  }
  G.nrows = G.wy * G.wz;
  if (threadIdx.x == 0) L.hs[G.nh] = G.total;
  __syncthreads();
  // exclusive scan of the target counts of the brick's rows, 64 rows per
  // step of the first wave
  if (threadIdx.x < 64) {
    int carry = 0;
    for (int r0 = 0; r0 < G.nrows; r0 += 64) {
      const int r = r0 + (int)threadIdx.x;
      int c = 0;
      if (r < G.nrows) {
        int ry;
        const int rz = small_div(r, G.wy, G.rwy, ry);
        const int hlo = G.ns + G.HX * ((G.ns + ry) + G.HY * (G.nsz + rz));
        c = L.hs[hlo + G.wx] - L.hs[hlo];
      }
      int x = c;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if ((int)threadIdx.x >= o) x += y;
      }
      if (r < G.nrows) L.rowpre[r] = carry + x - c;
      carry += __shfl(x, 63, 64);
    }
    if (threadIdx.x == 0) L.rowpre[G.nrows] = carry;
  }
  __syncthreads();
  G.ntg = L.rowpre[G.nrows];
  return G;
}

// A staging-map entry's second word: the particle's LDS slot in the upper 16
// bits, its halo cell below (8 bits per axis in 2D, 5 in 3D; the layout
// bounds the halo extents accordingly).
template <int D>
__device__ __forceinline__ int pack_map(int hx, int hy, int hz, int slot) {
  if constexpr (D == 2) return hx | (hy << 8) | (slot << 16);
  else return hx | (hy << 5) | (hz << 10) | (slot << 16);
}
template <int D>
__device__ __forceinline__ void unpack_map(int w, int& hx, int& hy, int& hz, int& slot) {
  slot = (int)((unsigned)w >> 16);
  if constexpr (D == 2) {
    hx = w & 255;
    hy = (w >> 8) & 255;
    hz = 0;
  } else {
    hx = w & 31;
    hy = (w >> 5) & 31;
    hz = (w >> 10) & 31;
  }
}

// Stage halo particles [cb, ce) (LDS order) as fixed-point coordinates, and
// their adjoint velocities when `lam` is given.  A slot's halo cell comes from
// the slot table of brick_setup (one chunk), else from a search of the halo
// starts.
template <int D, int NT, class Lds>
__device__ __forceinline__ void brick_stage(const BrickGeom& G, const Phys& P,
                                            const float* __restrict__ pos, const float* __restrict__ lam,
                                            Lds& L, int cb, int ce) {
  // SU particles per thread in flight (their halo cells, then their position
  // reads)
  constexpr int SU = 4;
  const bool table = (ce <= L.cap);
  for (int v0 = cb + (int)threadIdx.x; v0 < ce; v0 += SU * NT) {
    int hh[SU], g[SU];
    float p[SU][D];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int v = v0 + u * NT;
      int lo = 0;
      if (v < ce) {
        if (table) {
          lo = L.scell[v];
        } else {
          int hi = G.nh - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (L.hs[mid] <= v) lo = mid; else hi = mid - 1;
          }
        }
      }
      hh[u] = lo;
      g[u] = L.gs[lo] + (v - L.hs[lo]);
    }
#pragma unroll
    for (int u = 0; u < SU; ++u)
      if (v0 + u * NT < ce) ldv<D>(pos, g[u], p[u]);
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int v = v0 + u * NT;
      if (v < ce) {
        int hx, hy = 0;
        const int r = small_div(hh[u], G.HX, G.rHX, hx);
        const int hz = (D == 2) ? 0 : small_div(r, G.HY, G.rHY, hy);
        if constexpr (D == 2) {
          hy = r;
          put_coord(L.p, v - cb, fixed_coord(hx, p[u][0], P), fixed_coord(hy, p[u][1], P), 0, P);
        } else {
          put_coord(L.p, v - cb, fixed_coord(hx, p[u][0], P), fixed_coord(hy, p[u][1], P),
                    fixed_coord(hz, p[u][2], P), P);
        }
        if (lam) {
          float l[D];
          ldv<D>(lam, g[u], l);
#pragma unroll
          for (int k = 0; k < D; ++k) L.lam[(v - cb) * D + k] = l[k];
        }
      }
    }
  }
}

// Halo coordinates and global index of target t of the brick.
template <int D, class Lds>
__device__ __forceinline__ void brick_target(const BrickGeom& G, const Lds& L, int t, int& hxi,
                                             int& hyi, int& hzi, int& gi, int& vi) {
  int lo = 0, hi = G.nrows - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (L.rowpre[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const int row = lo;
  int ry;
  const int rz = small_div(row, G.wy, G.rwy, ry);
  hyi = G.ns + ry;
  hzi = G.nsz + rz;
  const int hbase = G.HX * (hyi + G.HY * hzi);
  vi = L.hs[hbase + G.ns] + (t - L.rowpre[row]);
  int clo = G.ns, chi = G.ns + G.wx - 1;
  while (clo < chi) {
    const int mid = (clo + chi + 1) >> 1;
    if (L.hs[hbase + mid] <= vi) clo = mid; else chi = mid - 1;
  }
  hxi = clo;
  const int hc = hbase + hxi;
  gi = L.gs[hc] + (vi - L.hs[hc]);
}

// Accumulate the LJ acceleration of one candidate on the target at (X, Y, Z).
// Branch-free: outside the cutoff, and for the target itself (r2 = 0), the
// inverse square distance is replaced by 0 so that the term vanishes.
template <int D, typename C>
__device__ __forceinline__ void lj_pair(const C& q, int X, int Y, int Z, const Phys& P,
                                        float (&f)[D]) {
  const float dx = (float)(q.x - X);
  const float dy = (float)(q.y - Y);
  float r2 = dx * dx + dy * dy;
  float dz = 0.f;
  if constexpr (D == 3) {
    dz = (float)(q.z - Z);
    r2 += dz * dz;
  }
  const bool in = (r2 < P.rc2_u) && (r2 > 0.f);
  const float ir2 = in ? __builtin_amdgcn_rcpf(r2) : 0.f;
  const float sr2 = P.sig2_u * ir2;
  const float sr6 = sr2 * sr2 * sr2;
  // the same operations as lj_pair_listed, so that both paths give the same
  // sums bit for bit (candidates beyond r_cut add exact zeros)
  const float gg = (ir2 * sr6) * fmaf(2.f * P.eps24m_u, sr6, -P.eps24m_u);
  f[0] -= gg * dx;
  f[1] -= gg * dy;
  if constexpr (D == 3) f[D - 1] -= gg * dz;
}

// The same term for a list entry: the list never holds the target itself, and
// its padding points at a sentinel far outside the cutoff, so only the cutoff
// is tested.
template <int D, typename C>
__device__ __forceinline__ void lj_pair_listed(const C& q, int X, int Y, int Z, const Phys& P,
                                               float (&f)[D]) {
  const float dx = (float)(q.x - X);
  const float dy = (float)(q.y - Y);
  float r2 = dx * dx + dy * dy;
  float dz = 0.f;
  if constexpr (D == 3) {
    dz = (float)(q.z - Z);
    r2 += dz * dz;
  }
  const float ir2 = (r2 < P.rc2_u) ? __builtin_amdgcn_rcpf(r2) : 0.f;
  const float sr2 = P.sig2_u * ir2;
  const float sr6 = sr2 * sr2 * sr2;
  // 24 eps / (m r^2) (sigma/r)^6 [2 (sigma/r)^6 - 1], one product fewer
  const float gg = (ir2 * sr6) * fmaf(2.f * P.eps24m_u, sr6, -P.eps24m_u);
  f[0] -= gg * dx;
  f[1] -= gg * dy;
  if constexpr (D == 3) f[D - 1] -= gg * dz;
}

// Fixed-point coordinate of the padding sentinel: 2^30 units from any staged
// particle (whose coordinates lie in [-2^27, 2^31)), far beyond the cutoff.
constexpr int kSentinel = 1 << 30;

// Cell range a target at (X, Y, Z) has to visit: every cell whose particles
// (which may sit up to the rebuild margin outside it) can lie within r_cut.
struct Reach {
  int cx0, cx1, cy0, cy1, cz0, cz1;
};

template <int D>
__device__ __forceinline__ Reach target_reach(const BrickGeom& G, const Phys& P, int X, int Y, int Z,
                                              int rq) {
  Reach r;
  r.cx0 = max(0, (X - rq) >> P.F);
  r.cx1 = min(G.HX - 1, (X + rq) >> P.F);
  r.cy0 = max(0, (Y - rq) >> P.F);
  r.cy1 = min(G.HY - 1, (Y + rq) >> P.F);
  r.cz0 = (D == 3) ? max(0, (Z - rq) >> P.F) : 0;
  r.cz1 = (D == 3) ? min(G.HZ - 1, (Z + rq) >> P.F) : 0;
  return r;
}

// Columns of halo row (cy, cz) that can hold a particle within r_cut of the
// target at (X, Y, Z): the row's particles lie within its cells widened by the
// rebuild margin, so the smallest |dy| (and |dz|) to the row bounds the reach
// along x by sqrt(r_cut^2 - dy^2 - dz^2).  Conservative by a few units.
// Returns false when the row is out of reach.
template <int D>
__device__ __forceinline__ bool row_columns(const BrickGeom& G, const Phys& P, int X, int Y, int Z,
                                            int cy, int cz, float rr2, int mq, int& cx0, int& cx1) {
  // distances in exact integer units; the squared radius is inflated by 4e-6
  // so that the float rounding of the squares can only widen the reach.  mq:
  // how far (in units) a particle may sit outside its cell
  const int dyi = max(0, max(((cy << P.F) - mq) - Y, Y - (((cy + 1) << P.F) + mq)));
  const float dy = (float)dyi;
  float r2 = fmaf(rr2, 4e-6f, rr2) - dy * dy;
  if constexpr (D == 3) {
    const int dzi = max(0, max(((cz << P.F) - mq) - Z, Z - (((cz + 1) << P.F) + mq)));
    const float dz = (float)dzi;
    r2 -= dz * dz;
  }
  if (r2 <= 0.f) return false;
  // (v_sqrt, within an ulp or so: the reach is widened by 64 units anyway)
  const int hw = (int)__builtin_amdgcn_sqrtf(r2) + mq + 64;
  cx0 = max(0, (X - hw) >> P.F);
  cx1 = min(G.HX - 1, (X + hw) >> P.F);
  return true;
}

// Velocity-Verlet update of one particle from its acceleration f, shared by
// both force paths; for a drift, also the largest squared half-step speed
// (vmx).
template <int D>
__device__ __forceinline__ void vv_update(const ForceArgs& a, const Phys& P, int gi,
                                          const float (&o)[D], const float (&v)[D],
                                          const float (&f)[D], float& vmx) {
  float vf[D];
  const bool drift = (a.mode == kModeStep || a.mode == kModeStart);
  float on[D], vh[D];
  bool ok = true;
  float v2 = 0.f;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    if (a.mode == kModeStep || a.mode == kModeFinish)
      vf[k] = fmaf(P.half_dt, f[k], v[k]);
    else
      vf[k] = v[k];
    vh[k] = fmaf(P.half_dt, f[k], vf[k]);
    on[k] = fmaf(vh[k], P.dt, o[k]);
    ok = ok && (on[k] >= P.lo) && (on[k] < P.hi);
    v2 = fmaf(vh[k], vh[k], v2);
  }
  if (a.vel_full_out) stv<D>(a.vel_full_out, gi, vf);
  if (drift) {
    if (!ok) atomicOr(a.err, kErrMargin);
    vmx = fmaxf(vmx, v2);
    stv<D>(a.pos_out, gi, on);
    stv<D>(a.vel, gi, vh);
  } else if (a.mode == kModeFinish) {
    stv<D>(a.vel, gi, vf);
  }
  if (a.acc_out) stv<D>(a.acc_out, gi, f);
}

// Largest value over the wave.
__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// Largest value over the wave (unsigned).
__device__ __forceinline__ unsigned wave_max_u(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, o, 64));
  return v;
}

// The pair lists hold every pair within r_cut + 2 skin at their build, so
// they cover every pair within r_cut as long as no particle has moved
// farther than the skin since.  A particle's drift in one step is
// |v_half| dt plus the rounding of the offset update, so the sum over the
// drifts since the build of dt times the step's largest |v_half| (the rows
// of disp, one slot word per lane), plus that rounding, bounds every
// displacement.  The sum runs from launch to launch: drift n adds row n - 1
// (complete once the launch that made it ended) to the sum drift n - 1
// passed on.  One wave; lane 0's value.
__device__ __forceinline__ double disp_running(const unsigned* __restrict__ disp,
                                               const double* __restrict__ psum, int n, float dt,
                                               float dslack) {
  if (n == 0) return 0.0;
  const unsigned w = wave_max_u(disp[(size_t)(n - 1) * kDispRow + lane_id() * kDispStride]);
  return psum[n - 1] + sqrt((double)__uint_as_float(w)) * (double)dt + (double)dslack;
}

// Staged coordinates of the four staging indices packed in e.
template <int D, class Lds>
__device__ __forceinline__ void list_gather(const Lds& L, unsigned long long e, Coord<D> (&q)[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) q[u] = L.p[(unsigned)(e >> (16 * u)) & 0xffffu];
}

// Accumulate the LJ acceleration from the four staging indices packed in e.
template <int D, class Lds>
__device__ __forceinline__ void list_word(const Lds& L, unsigned long long e, int X, int Y, int Z,
                                          const Phys& P, float (&f)[D]) {
  Coord<D> q[4];
  list_gather<D>(L, e, q);
#pragma unroll
  for (int u = 0; u < 4; ++u) lj_pair_listed<D>(q[u], X, Y, Z, P, f);
}

// Target record {particle, LDS slot | words << 16} of the list path, with the
// particle's offset, velocity and first list words.
template <int D, int GW>
__device__ __forceinline__ void list_fetch(const ForceArgs& a, int2 r, bool has, size_t nt,
                                           unsigned long long pad, int& gi, int& t, int& ng,
                                           float (&o)[D], float (&v)[D], unsigned long long (&w)[GW]) {
  gi = r.x;
  t = r.y & 0xffff;
  if (has && (size_t)(unsigned)gi >= nt) {
    // records come from the list builder; one that names no particle is
    // reported and read as particle 0 rather than followed out of bounds
    atomicOr(a.err, kErrRecord);
    gi = 0;
  }
  ng = has ? ((unsigned)r.y >> 16) : 0;
  if (has) {
    ldv<D>(a.pos_in, gi, o);
    ldv<D>(a.vel, gi, v);
  }
#pragma unroll
  for (int u = 0; u < GW; ++u) w[u] = (u < ng) ? a.nl[(size_t)u * nt + gi] : pad;
}

template <int D, int NT>
__device__ __forceinline__ void force_brick(const ForceArgs& a, int boff) {
#include "mdlg_force_block.inc"
}

// Pair lists of one brick, built right after each cell-list rebuild (all
// particles then lie inside their cells).  For every target the list holds
// the halo particles within r_cut + 2 skin (the skin at most the rebuild
// margin), so that it covers every pair within r_cut while no particle has
// moved farther than the skin since (the force kernel checks that bound).  Entries are 16-bit indices
// into the brick's LDS staging of its halo (halo cells in order, from the
// cell table, which stays fixed until the next rebuild), four to a word, the
// last word padded with the index of a sentinel slot beyond the halo (a zero
// term).  A brick whose halo exceeds one LDS chunk, or with a target of more
// than kmax neighbours, is marked for the cell walk.
typedef short Short2 __attribute__((ext_vector_type(2)));

// List-radius test of candidate q against the target (Txy, Tz) in 14-bit
// units: |d|^2 - rl16, negative when q is near.  The x and y differences are
// taken as a packed 16-bit pair and squared and summed by a dot product onto
// dz^2 - rl16 (a 24-bit multiply-add); no term can overflow, as each
// coordinate stays below 2^14.
// The three-operand forms are written out: the compiler otherwise emits the
// two-operand accumulating dot product (v_dot2c) after a copy of the addend,
// and a separate multiply and subtract for dz^2 - rl16, one instruction more
// per candidate either way.  (Arithmetic only: no memory access here.)
template <int D>
__device__ __forceinline__ int list_test14(Coord14<D> q, unsigned Txy, int Tz, int thr) {
  unsigned qxy;
  if constexpr (D == 2) qxy = q;
  else qxy = q.x;
  const unsigned d = __builtin_bit_cast(
      unsigned, __builtin_bit_cast(Short2, qxy) - __builtin_bit_cast(Short2, Txy));
  int r;
  if constexpr (D == 2) {
    asm("v_dot2_i32_i16 %0, %1, %1, %2" : "=v"(r) : "v"(d), "s"(-thr));
  } else {
    const int dz = (int)q.y - Tz;
    int acc;
    asm("v_mad_i32_i24 %0, %1, %1, %2" : "=v"(acc) : "v"(dz), "s"(-thr));
    asm("v_dot2_i32_i16 %0, %1, %1, %2" : "=v"(r) : "v"(d), "v"(acc));
  }
  return r;
}

// Append entry e to a list being built four 16-bit entries per word: the
// word (hi, lo) shifts down by one entry and e enters at the top, so that the
// first of four entries ends in the lowest bits; completed words go to *wp,
// which then steps to the next word (stride nt).
__device__ __forceinline__ void list_push(unsigned long long*& wp, unsigned& hi, unsigned& lo, int& cnt,
                                          unsigned e, size_t nt) {
  lo = __builtin_amdgcn_alignbit(hi, lo, 16);
  hi = __builtin_amdgcn_alignbit(e, hi, 16);
  if ((++cnt & 3) == 0) {
    *wp = ((unsigned long long)hi << 32) | lo;
    wp += nt;
  }
}

// One row of a target's candidates, LDS range [jlo, jhi): test GR candidates
// at a time into a bit mask (the last step reads into the next row or the
// padding and is masked), then append the accepted ones, so that appends cost
// per accepted entry rather than per candidate.  Entries are the candidates'
// LDS indices, which the force kernel's staging reproduces.
template <int D, int GR>
__device__ __forceinline__ void nl_row(const Coord14<D>* __restrict__ p, int jlo, int jhi, int vi,
                                       unsigned Txy, int Tz, int thr, int kmax, size_t nt,
                                       unsigned long long*& wp, unsigned& whi, unsigned& wlo, int& cnt,
                                       int& seen) {
  for (int j0 = jlo; j0 < jhi; j0 += GR) {
    int r[GR];
#pragma unroll
    for (int e = 0; e < GR; ++e) r[e] = list_test14<D>(p[j0 + e], Txy, Tz, thr);
    // sign bits into a mask (m << 1 | sign); candidate e then sits at bit
    // GR - 1 - e: reverse
    unsigned m = 0;
#pragma unroll
    for (int e = 0; e < GR; ++e) m = __builtin_amdgcn_alignbit(m, (unsigned)r[e], 31);
    unsigned mask = __builtin_bitreverse32(m);
    if constexpr (GR < 32) mask >>= 32 - GR;
    const int nb = jhi - j0;
    if (nb < GR) mask &= (1u << nb) - 1u;
    const unsigned self = (unsigned)(vi - j0);
    if (self < (unsigned)GR) mask &= ~(1u << self);
    const int add = __popc(mask);
    seen += add;
    // a list longer than kmax sends the brick to the cell walk: its entries
    // need not be complete, only kept within the slots
    if (cnt + add > kmax) mask = 0;
    while (mask) {
      const int j = j0 + __builtin_ctz(mask);
      mask &= mask - 1;
      list_push(wp, whi, wlo, cnt, (unsigned)j, nt);
    }
  }
}

// The force kernel's staging map of a brick: the staged halo particles that
// some target's list may name, each as {particle, LDS slot and halo cell}, in
// LDS order.  At the build every target lies in the brick's cells, so in 3D a
// particle farther than the list radius from their box is in no list: it is
// left out, and the slot it holds here stays unstaged in the force kernel (no
// entry names it).  The test takes the list test's own 14-bit units, so it
// keeps every particle that the list test can accept.  (In 2D a halo of one
// cell keeps nearly all of its particles, and the map holds every slot.)
// s_cnt holds 64 ints of scratch.  Returns the number of entries.
template <int D, int NT, class Lds>
__device__ __forceinline__ int nl_stage_map(const BrickGeom& G, const Phys& P, Lds& L,
                                            int2* __restrict__ smap, int* s_cnt) {
  constexpr int NW = NT / 64;
  const int rounds = (G.total + NT - 1) / NT;
  // the box of the brick's cells in 14-bit units (a target's offset may round
  // up to the cell side, so its upper bound is inclusive)
  const unsigned lift = 2u << P.F;
  auto lo14 = [&](int h) { return (int)((((unsigned)h << P.F) + lift) >> P.sh16); };
  const int bx0 = lo14(G.ns), bx1 = lo14(G.ns + G.wx);
  const int by0 = lo14(G.ns), by1 = lo14(G.ns + G.wy);
  const int bz0 = lo14(G.nsz), bz1 = lo14(G.nsz + G.wz);
  const bool filter = (D == 3) && rounds * NW <= 64;  // (block-uniform)
  auto near = [&](int v) {
    const Coord14<D> q = L.p[v];
    unsigned qxy;
    if constexpr (D == 2) qxy = q;
    else qxy = q.x;
    const int qx = (int)(qxy & 0xffffu), qy = (int)(qxy >> 16);
    const int dx = max(0, max(bx0 - qx, qx - bx1));
    const int dy = max(0, max(by0 - qy, qy - by1));
    int d2 = dx * dx + dy * dy;
    if constexpr (D == 3) {
      const int qz = (int)q.y;
      const int dz = max(0, max(bz0 - qz, qz - bz1));
      d2 += dz * dz;
    }
    return d2 < P.rl16;
  };
  auto put = [&](int v, int slot) {
    const int h = L.scell[v];
    int hx, hy = 0, hz = 0;
    const int r = small_div(h, G.HX, G.rHX, hx);
    if constexpr (D == 2) hy = r;
    else hz = small_div(r, G.HY, G.rHY, hy);
    smap[slot] = make_int2(L.gs[h] + (v - L.hs[h]), pack_map<D>(hx, hy, hz, v));
  };
  if (!filter) {
    for (int v = (int)threadIdx.x; v < G.total; v += NT) put(v, v);
    return G.total;
  }
  // slot v = k NT + thread of round k: the wave's count of kept slots per
  // round, then each kept slot's entry from the counts before it
  const int lane = lane_id(), w = (int)threadIdx.x >> 6;
  unsigned long long kb = 0ull;  // kept slots of this thread, bit k for round k
  for (int k = 0; k < rounds; ++k) {
    const int v = k * NT + (int)threadIdx.x;
    const bool keep = v < G.total && near(v);
    if (keep) kb |= 1ull << k;
    const unsigned long long m = __ballot(keep);
    if (lane == 0) s_cnt[k * NW + w] = __popcll(m);
  }
  __syncthreads();
  const unsigned long long lt = (1ull << lane) - 1ull;
  int base = 0;
  for (int k = 0; k < rounds; ++k) {
    const bool keep = (kb >> k) & 1ull;
    const unsigned long long m = __ballot(keep);
    int pre = 0, sum = 0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
      const int c = s_cnt[k * NW + ww];
      sum += c;
      if (ww < w) pre += c;
    }
    if (keep) put(k * NT + (int)threadIdx.x, base + pre + __popcll(m & lt));
    base += sum;
  }
  // (s_cnt is reused by the caller)
  __syncthreads();
  return base;
}

template <int D, int NT, int GR>
__device__ __forceinline__ void nlist_brick(const NlistArgs& a) {
  extern __shared__ __align__(16) char s_dyn_brick[];
  __shared__ int s_rowpre[kMaxRows + 1];
  constexpr int NW = NT / 64;
  __shared__ int s_tmp[NW + 1];
  __shared__ double s_red[NW][4];
  __shared__ int s_over;
  __shared__ int s_cnt[64];
  auto L = brick_lds<D, false, Coord14<D>>(s_dyn_brick, s_rowpre, s_tmp, s_red, a.P, kNlPad);
  // word count of every target's list (dynamic LDS behind the brick's own)
  unsigned char* s_words = reinterpret_cast<unsigned char*>(s_dyn_brick) +
                           brick_lds_layout_dev<D, false, Coord14<D>>(a.P, kNlPad).end;
  const int CAP = L.cap;
  int b = blockIdx.x;
  if (a.xcd_remap) {
    const int per = gridDim.x >> 3;
    b = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  }
  if (b >= a.nbricks) return;
  const Phys& P = a.P;
  const int4 br = a.bricks[b];
  const Replica R = a.reps[br.x];
  if (threadIdx.x == 0) s_over = 0;
  const BrickGeom G = brick_setup<D, NT>(P, R, br, a.cell_start, L);
  const bool fits = G.total < CAP;  // one slot stays free for the padding sentinel
  if (fits) brick_stage<D, NT>(G, P, a.pos, nullptr, L, 0, G.total);
  if (b == 0) {
    // a new displacement bound starts with these lists
    for (int i = threadIdx.x; i < a.ndisp_clear * kDispSlots; i += NT)
      a.disp_clear[(size_t)(i / kDispSlots) * kDispRow + (i % kDispSlots) * kDispStride] = 0u;
    for (int i = threadIdx.x; i < a.ndisp_clear; i += NT) a.stale_clear[i] = 0u;
  }
  __syncthreads();
  // (block-uniform)
  const int nmap = fits ? nl_stage_map<D, NT>(G, P, L, a.smap + (size_t)b * CAP, s_cnt) : 0;
  const size_t nt = (size_t)P.n_total;
  const int kmax = P.kmax;
  const int thr = P.rl16;
  for (int tb = 0; tb < G.ntg; tb += NT) {
    const int t = tb + (int)threadIdx.x;
    if (t >= G.ntg) break;
    if (!fits) break;  // (block-uniform) the brick walks its cells
    int hxi, hyi, hzi, gi, vi;
    brick_target<D>(G, L, t, hxi, hyi, hzi, gi, vi);
    // the target's own 14-bit coordinates and the fixed-point coordinates
    // they stand for, within half a 14-bit unit, which widens the reach and
    // the row bounds
    const Coord14<D> me = L.p[vi];
    unsigned Txy;
    int Tz = 0;
    if constexpr (D == 2) {
      Txy = me;
    } else {
      Txy = me.x;
      Tz = (int)me.y;
    }
    const int eh = P.sh16 > 0 ? 1 << (P.sh16 - 1) : 0;
    const unsigned lift = 2u << P.F;
    const int X = (int)(((Txy & 0xffffu) << P.sh16) - lift) + eh;
    const int Y = (int)(((Txy >> 16) << P.sh16) - lift) + eh;
    const int Z = (D == 3) ? (int)(((unsigned)Tz << P.sh16) - lift) + eh : 0;
    const Reach rr = target_reach<D>(G, P, X, Y, Z, P.rlq + eh);
    unsigned long long* wp = a.nl + gi;  // next list word
    unsigned whi = 0, wlo = 0;
    int cnt = 0, seen = 0;
    for (int cz = rr.cz0; cz <= rr.cz1; ++cz) {
      for (int cy = rr.cy0; cy <= rr.cy1; ++cy) {
        int cx0, cx1;
        if (!row_columns<D>(G, P, X, Y, Z, cy, cz, P.rl2_u, 4 + eh, cx0, cx1)) continue;
        // one contiguous LDS range per row
        const int hrow = G.HX * (cy + G.HY * cz);
        nl_row<D, GR>(L.p, L.hs[hrow + cx0], L.hs[hrow + cx1 + 1], vi, Txy, Tz, thr, kmax, nt, wp,
                      whi, wlo, cnt, seen);
      }
    }
    if (seen > kmax) s_over = 1;
    // pad the last word with the sentinel (far outside the cutoff)
    while (cnt & 3) list_push(wp, whi, wlo, cnt, (unsigned)G.total, nt);
    const int words = (cnt + 3) >> 2;
    s_words[t] = (unsigned char)words;
  }
  __syncthreads();
  // processing order of the targets: decreasing word count (counting sort)
  if (fits) {
    int2* __restrict__ trec = a.trec + (size_t)b * CAP;
    for (int i = threadIdx.x; i < 64; i += NT) s_cnt[i] = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < G.ntg; t += NT) atomicAdd(&s_cnt[63 - s_words[t]], 1);
    __syncthreads();
    if (threadIdx.x < 64) {
      // exclusive scan of the 64 bins across the first wave
      const int c = s_cnt[threadIdx.x];
      int x = c;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if ((int)threadIdx.x >= o) x += y;
      }
      s_cnt[threadIdx.x] = x - c;
    }
    __syncthreads();
    // stable within a bin (targets in brick order): a target's slot is its
    // bin's start plus the targets of the bin before it, counted across the
    // wave with ballots and across the waves in wave order
    const int lane = lane_id(), wv = (int)threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int tb = 0; tb < G.ntg; tb += NT) {
      const int t = tb + (int)threadIdx.x;
      const bool valid = t < G.ntg;
      const int bin = valid ? 63 - (int)s_words[t] : -1;
      unsigned long long same = 0ull, act = __ballot(valid);
      while (act) {
        const int leader = __ffsll((long long)act) - 1;
        const int lb = __builtin_amdgcn_readlane(bin, leader);
        const unsigned long long m = __ballot(valid && bin == lb) & act;
        if (valid && bin == lb) same = m;
        act &= ~m;
      }
      const bool lead = valid && (same & lt) == 0ull;
      int b0 = 0;
      for (int w = 0; w < NW; ++w) {
        if (wv == w && lead) {
          b0 = s_cnt[bin];
          s_cnt[bin] = b0 + __popcll(same);
        }
        __syncthreads();
      }
      const int base = __shfl(b0, valid ? __ffsll((long long)same) - 1 : lane, 64);
      if (valid) {
        int hxi, hyi, hzi, gi, vi;
        brick_target<D>(G, L, t, hxi, hyi, hzi, gi, vi);
        trec[base + __popcll(same & lt)] = make_int2(gi, vi | ((int)s_words[t] << 16));
      }
    }
  }
  if (threadIdx.x == 0) a.binfo[b] = make_int4(G.total, G.ntg, (fits && !s_over) ? 1 : 0, nmap);
}

// The list builder with 16 candidates per test step (short rows) and with 32
// (long rows).
template <int D, int NT>
__global__ __launch_bounds__(NT) void k_nlist_narrow(NlistArgs a) {
  nlist_brick<D, NT, 16>(a);
}

template <int D, int NT>
__global__ __launch_bounds__(NT) void k_nlist_wide(NlistArgs a) {
  nlist_brick<D, NT, 32>(a);
}

// ---------------------------------------------------------------- adjoint
//
// One reverse step of the velocity-Verlet adjoint at positions x_s: for every
// particle i,
//   a_i, da_i/dsigma, and (J lam_v)_i = sum_j K_ij (lam_v,i - lam_v,j) / m with
//   K = g I + (g'(r)/r) r r^T, g(r) = (24 eps / r^2)[2 (sigma/r)^12 - (sigma/r)^6],
// then lam_x,i += c (J lam_v)_i, the parameter gradients gain
// c lam_v,i . a_i / eps and c lam_v,i . da_i/dsigma, and (unless this is the
// first position of the window) lam_v,i += h lam_x,i, written to the other
// lam_v buffer.  Coordinates are fixed point as in k_force; with d = x_j - x_i
// in units u, r = -d and the terms read (E1 = 24 eps / (m u), E2 = E1 / u):
//   a_i      -= E1 ir2 s6 (2 s6 - 1) d
//   da_i/ds  -= (E1 / sigma) ir2 s6 (24 s6 - 6) d
//   (J l)_i  += E2 [ir2 s6 (2 s6 - 1) dl + ir2^2 s6 (8 - 28 s6) (d . dl) d]
template <int D>
__device__ __forceinline__ void adj_pair(const Coord<D>& q, const float* __restrict__ lj, int X, int Y,
                                         int Z, const float (&li)[D], const Phys& P, float (&acc)[D],
                                         float (&dacc)[D], float (&jl)[D]) {
  float d[D], dl[D];
  d[0] = (float)(q.x - X);
  d[1] = (float)(q.y - Y);
  if constexpr (D == 3) d[2] = (float)(q.z - Z);
  float r2 = 0.f, ddl = 0.f;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    dl[k] = li[k] - lj[k];
    r2 += d[k] * d[k];
    ddl += d[k] * dl[k];
  }
  const bool in = (r2 < P.rc2_u) && (r2 > 0.f);
  const float ir2 = in ? __builtin_amdgcn_rcpf(r2) : 0.f;
  const float sr2 = P.sig2_u * ir2;
  const float s6 = sr2 * sr2 * sr2;
  const float t1 = ir2 * s6 * (2.f * s6 - 1.f);
  const float ts = ir2 * s6 * (24.f * s6 - 6.f);
  const float t2 = ir2 * ir2 * s6 * (8.f - 28.f * s6) * ddl;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    acc[k] -= t1 * d[k];
    dacc[k] -= ts * d[k];
    jl[k] += t1 * dl[k] + t2 * d[k];
  }
}

// The updates of one target from its sums: lam_x, lam_v and the parameter
// gradient partials.
template <int D>
__device__ __forceinline__ void adj_update(const AdjArgs& a, const Phys& P, int gi,
                                           const float (&li)[D], const float (&acc)[D],
                                           const float (&dacc)[D], const float (&jl)[D], double& ge,
                                           double& gs) {
  float lx[D], lv[D];
  ldv<D>(a.lam_x, gi, lx);
  double e = 0.0, s = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float a_k = P.eps24m_u * acc[k];
    const float da_k = a.e1_over_sigma * dacc[k];
    const float jl_k = a.e2 * jl[k];
    lx[k] = fmaf(a.c, jl_k, lx[k]);
    e += (double)li[k] * (double)a_k;
    s += (double)li[k] * (double)da_k;
    lv[k] = a.drift ? fmaf(P.dt, lx[k], li[k]) : li[k];
  }
  ge += (double)a.c * e / a.eps;
  gs += (double)a.c * s;
  stv<D>(a.lam_x, gi, lx);
  stv<D>(a.lam_v_out, gi, lv);
}

template <int D, int NT>
__device__ __forceinline__ void adjoint_brick(const AdjArgs& a, int b) {
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) char s_dyn_brick[];
  __shared__ int s_rowpre[kMaxRows + 1];
  __shared__ int s_tmp[NW + 1];
  __shared__ double s_red[NW][4];
  auto L = brick_lds<D, true>(s_dyn_brick, s_rowpre, s_tmp, s_red, a.P);
  const int CAP = L.cap;
  const Phys& P = a.P;
  const int4 br = a.bricks[b];
  const bool interact = !P.forces_off;
  double ge = 0.0, gs = 0.0;
  // the window's pair lists, where the builder's halo fits this kernel's LDS
  // chunk with the padding sentinel; (the flag after the whole forward window
  // covers each of its positions: once set, it stays set)
  const int4 bi = a.nl ? a.binfo[b] : make_int4(0, 0, 0, 0);
  const bool stale = a.nl && a.stale && *a.stale != 0u;
  if (interact && bi.z && !stale && bi.x < CAP) {
    // the halo particles the lists name, staged through the builder's map
    // (each entry with its LDS slot): positions and adjoint velocities, with
    // the first target records requested together with the map entries
    const int2* __restrict__ smap = a.smap + (size_t)b * a.lcap_list;
    const int2* __restrict__ trec = a.trec + (size_t)b * a.lcap_list;
    const int total = bi.x, ntg = bi.y, nmap = bi.w;
    const size_t nt = (size_t)P.n_total;
    const int2 r0 = trec[min((int)threadIdx.x, a.lcap_list - 1)];
    const int elast = max(nmap - 1, 0);
    for (int v0 = (int)threadIdx.x; v0 < nmap; v0 += 2 * NT) {
      int2 e[2];
      float p[2][D], l[2][D];
#pragma unroll
      for (int u = 0; u < 2; ++u) e[u] = smap[min(v0 + u * NT, elast)];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (v0 + u * NT < nmap) {
          ldv<D>(a.pos, e[u].x, p[u]);
          ldv<D>(a.lam_v_in, e[u].x, l[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (v0 + u * NT < nmap) {
          int hx, hy, hz, slot;
          unpack_map<D>(e[u].y, hx, hy, hz, slot);
          if constexpr (D == 2)
            L.p[slot] = make_int2(fixed_coord(hx, p[u][0], P), fixed_coord(hy, p[u][1], P));
          else
            L.p[slot] = make_int4(fixed_coord(hx, p[u][0], P), fixed_coord(hy, p[u][1], P),
                                  fixed_coord(hz, p[u][2], P), 0);
#pragma unroll
          for (int k = 0; k < D; ++k) L.lam[slot * D + k] = l[u][k];
        }
      }
    }
    if (threadIdx.x == 0) {
      // the padding sentinel: far outside the cutoff, zero adjoint velocity
      if constexpr (D == 2) L.p[total] = make_int2(kSentinel, kSentinel);
      else L.p[total] = make_int4(kSentinel, kSentinel, kSentinel, 0);
#pragma unroll
      for (int k = 0; k < D; ++k) L.lam[total * D + k] = 0.f;
    }
    __syncthreads();
    for (int tb = 0; tb < ntg; tb += NT) {
      const int t = tb + (int)threadIdx.x;
      if (t >= ntg) break;
      const int2 r = (tb == 0) ? r0 : trec[t];
      const int gi = r.x;
      const int vi = r.y & 0xffff;
      const int ng = (unsigned)r.y >> 16;
      if ((size_t)(unsigned)gi >= nt || vi >= total) {
        atomicOr(a.err, kErrRecord);
        continue;
      }
      const Coord<D> me = L.p[vi];
      const int X = me.x, Y = me.y;
      int Z = 0;
      if constexpr (D == 3) Z = me.z;
      float li[D], acc[D], dacc[D], jl[D];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        li[k] = L.lam[vi * D + k];
        acc[k] = 0.f;
        dacc[k] = 0.f;
        jl[k] = 0.f;
      }
      const unsigned long long* __restrict__ lp = a.nl + gi;
      for (int k = 0; k < ng; ++k) {
        const unsigned long long wd = lp[(size_t)k * nt];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = (int)((wd >> (16 * u)) & 0xffffu);
          adj_pair<D>(L.p[e], &L.lam[e * D], X, Y, Z, li, P, acc, dacc, jl);
        }
      }
      adj_update<D>(a, P, gi, li, acc, dacc, jl, ge, gs);
    }
  } else {
    // the frozen cells, walked row by row
    const Replica R = a.reps[br.x];
    const BrickGeom G = brick_setup<D, NT>(P, R, br, a.cell_start, L);
    const int nchunks = (G.total + CAP - 1) / CAP;
    if (interact && nchunks == 1) {
      brick_stage<D, NT>(G, P, a.pos, a.lam_v_in, L, 0, G.total);
      __syncthreads();
    }
    for (int tb = 0; tb < G.ntg; tb += NT) {
      const int t = tb + (int)threadIdx.x;
      const bool valid = t < G.ntg;
      int hxi = G.ns, hyi = G.ns, hzi = G.nsz, gi = 0, vi = 0;
      if (valid) brick_target<D>(G, L, t, hxi, hyi, hzi, gi, vi);
      float o[D], li[D], acc[D], dacc[D], jl[D];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        o[k] = 0.f;
        li[k] = 0.f;
        acc[k] = 0.f;
        dacc[k] = 0.f;
        jl[k] = 0.f;
      }
      if (valid) {
        ldv<D>(a.pos, gi, o);
        ldv<D>(a.lam_v_in, gi, li);
      }
      if (interact) {
        const int X = fixed_coord(hxi, o[0], P);
        const int Y = fixed_coord(hyi, o[1], P);
        const int Z = (D == 3) ? fixed_coord(hzi, o[D - 1], P) : 0;
        const Reach rr = target_reach<D>(G, P, X, Y, Z, P.rcq);
        for (int ci = 0; ci < nchunks; ++ci) {
          const int cb = ci * CAP, ce = min(G.total, cb + CAP);
          if (nchunks > 1) {
            __syncthreads();
            brick_stage<D, NT>(G, P, a.pos, a.lam_v_in, L, cb, ce);
            __syncthreads();
          }
          if (valid) {
            for (int cz = rr.cz0; cz <= rr.cz1; ++cz) {
              for (int cy = rr.cy0; cy <= rr.cy1; ++cy) {
                int cx0, cx1;
                if (!row_columns<D>(G, P, X, Y, Z, cy, cz, P.rc2_u, P.mq, cx0, cx1)) continue;
                const int hrow = G.HX * (cy + G.HY * cz);
                const int jlo = max(L.hs[hrow + cx0], cb) - cb;
                const int jhi = min(L.hs[hrow + cx1 + 1], ce) - cb;
                for (int j = jlo; j < jhi; ++j)
                  adj_pair<D>(L.p[j], &L.lam[j * D], X, Y, Z, li, P, acc, dacc, jl);
              }
            }
          }
        }
      }
      if (valid) adj_update<D>(a, P, gi, li, acc, dacc, jl, ge, gs);
    }
  }
  const int w = threadIdx.x >> 6;
  const double se = wave_sum_d(ge), ss = wave_sum_d(gs);
  if (lane_id() == 0) {
    L.red[w][0] = se;
    L.red[w][1] = ss;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int i = 0; i < NW; ++i) t += L.red[i][threadIdx.x];
    a.gpart[(size_t)b * 2 + threadIdx.x] = t;
  }
}

// One block per brick: the force kernel (a force / velocity-Verlet step of
// every particle) and the adjoint's reverse step.
// (at most 96 SGPRs: with the 106 it takes otherwise, the SGPR file holds
// seven waves per SIMD where the 2D instance's 63 VGPRs allow eight; the
// excess is kept in VGPR lanes, not in scratch)
template <int D, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_num_sgpr(96))) void k_force(ForceArgs a) {
  constexpr int boff = 0;
#include "mdlg_force_block.inc"
}

template <int D, int NT>
__global__ __launch_bounds__(NT) void k_adjoint(AdjArgs a) {
  const int b = blockIdx.x;
  if (b >= a.nbricks) return;
  adjoint_brick<D, NT>(a, b);
}

// A reverse step and, in the same launch, an independent force step (the
// recomputation of an earlier segment of the window, on other buffers): the
// reverse step's bricks first, then the force step's.  Each block runs one
// or the other exactly as its own kernel would.
template <int D, int NT>
__global__ __launch_bounds__(NT) void k_adjoint_force(AdjForceArgs a) {
  const int b = blockIdx.x;
  if (b < a.adj.nbricks) adjoint_brick<D, NT>(a.adj, b);
  else force_brick<D, NT>(a.force, a.adj.nbricks);
}

// Loss of the window and its gradient with respect to the final positions.
// Cells are fixed during the window, so x_j(W) - x_j(0) = off_W - off_0.
template <int D>
__global__ __launch_bounds__(kBlock) void k_adj_loss(AdjLossArgs a) {
  __shared__ double s_red[kWaves];
  double L = 0.0;
  const double inv_nd = 1.0 / ((double)a.n * D), inv_n = 1.0 / (double)a.n;
  for (int g = blockIdx.x * kBlock + threadIdx.x; g < a.n; g += gridDim.x * kBlock) {
    float o0[D], o1[D], lx[D], zero[D];
    ldv<D>(a.off0, g, o0);
    ldv<D>(a.offW, g, o1);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double dd = (double)o1[k] - (double)o0[k];
      zero[k] = 0.f;
      if (a.loss == 0) {
        L += dd * dd * inv_nd;
        lx[k] = (float)(2.0 * dd * inv_nd);
      } else {
        if (k == 0) L += dd * inv_n;
        lx[k] = (k == 0) ? (float)inv_n : 0.f;
      }
    }
    stv<D>(a.lam_x, g, lx);
    stv<D>(a.lam_v, g, zero);
  }
  const double s = wave_sum_d(L);
  if (lane_id() == 0) s_red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < kWaves; ++i) t += s_red[i];
    a.lpart[blockIdx.x] = t;
  }
}

// Sum of the per-block partials of the loss and the parameter gradients, in
// a fixed order.
__global__ __launch_bounds__(kBlock) void k_adj_final(AdjFinalArgs a) {
  // one block: thread-strided partial sums (four independent chains per
  // thread, so the loads overlap), then the waves' sums in LDS, added in
  // wave order (a fixed summation order, so the result does not depend on
  // timing)
  __shared__ double s_red[kWaves][3];
  double L = 0.0, ge[4] = {0.0, 0.0, 0.0, 0.0}, gs[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < a.nl; i += kBlock) L += a.lpart[i];
  int b = threadIdx.x;
  for (; b + 3 * kBlock < a.nb; b += 4 * kBlock) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ge[u] += a.gpart[(size_t)(b + u * kBlock) * 2];
      gs[u] += a.gpart[(size_t)(b + u * kBlock) * 2 + 1];
    }
  }
  for (; b < a.nb; b += kBlock) {
    ge[0] += a.gpart[(size_t)b * 2];
    gs[0] += a.gpart[(size_t)b * 2 + 1];
  }
  const double e = wave_sum_d((ge[0] + ge[1]) + (ge[2] + ge[3]));
  const double g = wave_sum_d((gs[0] + gs[1]) + (gs[2] + gs[3]));
  L = wave_sum_d(L);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    s_red[w][0] = L;
    s_red[w][1] = e;
    s_red[w][2] = g;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int i = 0; i < kWaves; ++i) t += s_red[i][threadIdx.x];
    a.out[threadIdx.x] = t;
  }
}

// Velocities by id into the sorted state (start of an adjoint window), and
// the adjoint of v(0) from the sorted order back to id order.
template <int D>
__global__ __launch_bounds__(kBlock) void k_adj_io(AdjIoArgs a) {
  for (int g = blockIdx.x * kBlock + threadIdx.x; g < a.n; g += gridDim.x * kBlock) {
    const int pid = a.id[g];
    float v[D];
    if (a.to_sorted) {
      ldv<D>(a.by_id, pid, v);
      stv<D>(a.sorted, g, v);
    } else {
      ldv<D>(a.sorted, g, v);
      stv<D>(a.by_id, pid, v);
    }
  }
}

__global__ void k_copy_f32(const float* __restrict__ src, float* __restrict__ dst, long long n) {
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    dst[i] = src[i];
}

// ---------------------------------------------------------------- kinetics

// One block per replica: FP64 sums of the per-brick partials in a fixed order.
// FP64 kinetic partials of one particle chunk: each thread sums its strided
// particles, then the waves and the block in a fixed order, so that the sums
// depend on the state alone.
template <int D>
__global__ __launch_bounds__(kBlock) void k_kinpart(KinPartArgs a) {
  __shared__ double s_red[kWaves][4];
  const int4 ch = a.chunks[blockIdx.x];
  double s[D + 1];
#pragma unroll
  for (int k = 0; k <= D; ++k) s[k] = 0.0;
  for (int g = ch.y + threadIdx.x; g < ch.z; g += kBlock) {
    float v[D];
    ldv<D>(a.vel, g, v);
    double e = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      s[k] += a.mass * (double)v[k];
      e += (double)v[k] * (double)v[k];
    }
    s[D] += 0.5 * a.mass * e;
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k <= D; ++k) {
    const double t = wave_sum_d(s[k]);
    if (lane_id() == 0) s_red[w][k] = t;
  }
  __syncthreads();
  if (threadIdx.x <= D) {
    double t = 0.0;
    for (int i = 0; i < kWaves; ++i) t += s_red[i][threadIdx.x];
    a.kpart[(size_t)blockIdx.x * (D + 1) + threadIdx.x] = t;
  }
}

__global__ __launch_bounds__(kBlock) void k_kin(KinArgs a) {
  __shared__ double s_red[kWaves][4];
  const int r = blockIdx.x;
  const Replica R = a.reps[r];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c = R.chunk_off + threadIdx.x; c < R.chunk_off + R.nchunks; c += kBlock)
    for (int k = 0; k <= a.D; ++k) s[k] += a.kpart[(size_t)c * (a.D + 1) + k];
  const int w = threadIdx.x >> 6;
  for (int k = 0; k <= a.D; ++k) {
    const double t = wave_sum_d(s[k]);
    if (lane_id() == 0) s_red[w][k] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < kWaves; ++i)
      for (int k = 0; k <= a.D; ++k) tot[k] += s_red[i][k];
    for (int k = 0; k <= a.D; ++k) a.kin[(size_t)r * (a.D + 1) + k] = tot[k];
    if (a.thermostat) {
      const double ke = tot[a.D];
      a.lambda[r] = (ke > 0.0 && R.n > 1)
                        ? (float)sqrt(a.kT * a.D * (R.n - 1) / (2.0 * ke))
                        : 1.f;
    }
  }
}

// ---------------------------------------------------------------- MDLG binning

template <int D>
__global__ __launch_bounds__(kBlock) void k_bin(BinArgs a) {
  extern __shared__ int s_dyn[];
  __shared__ int s_rp[65];
  __shared__ int s_rg[64];
  __shared__ double s_red[kWaves][2 * D];
  const Phys& P = a.P;
  // (strips in dispatch order: keeping consecutive strips on one XCD
  // measured slower)
  const int sb = blockIdx.x;
  const int4 st = a.strips[sb];
  const Replica R = a.reps[st.x];
  const int k = 1 << P.log2k;
  // a strip: site rows sy0 .. sy0 + wsy - 1 of BSX sites from sx0 (layer sz)
  const int sx0 = st.y, sy0 = st.z, sz = st.w;
  const int wsx = min(a.BSX, R.M[0] - sx0);
  const int wsy = min(a.BSY, R.M[1] - sy0);
  const int Q = P.Q, nm = P.nm;
  const int nsite = a.BSX * a.BSY;
  unsigned* s_h = reinterpret_cast<unsigned*>(s_dyn);  // [BSY][BSX][Q]
  int* s_m = s_dyn + nsite * Q;                        // [BSY][BSX][nm]
  if (!a.snapshot_only) {
    for (int e = threadIdx.x; e < nsite * (Q + nm); e += kBlock) s_dyn[e] = 0;
  }
  // the MD-cell rows covering the strip (at most 64), one per lane of the
  // first wave: their first particle and, by a scan, their start in the
  // strip's particle order
  const int rows_per = (D == 2) ? k : k * k;  // MD-cell rows of one site row
  const int nrows = wsy * rows_per;
  if (threadIdx.x < 64) {
    const int r = threadIdx.x;
    int g0 = 0, cnt = 0;
    if (r < nrows) {
      const int j = r / rows_per, rr = r - j * rows_per;
      const int ry = (sy0 + j) * k + (rr & (k - 1));
      const int rz = (D == 3) ? sz * k + (rr >> P.log2k) : 0;
      const int rowbase = R.cell_off + R.Mc[0] * (ry + R.Mc[1] * rz);
      g0 = a.cell_start[rowbase + sx0 * k];
      cnt = a.cell_start[rowbase + (sx0 + wsx) * k] - g0;
    }
    int x = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (r >= o) x += y;
    }
    if (r < nrows) {
      s_rg[r] = g0;
      s_rp[r] = x - cnt;
    }
    if (r == nrows - 1) s_rp[nrows] = x;
  }
  __syncthreads();
  const int np = s_rp[nrows];
  double ds[D], dq[D];
#pragma unroll
  for (int q = 0; q < D; ++q) {
    ds[q] = 0.0;
    dq[q] = 0.0;
  }
  const int W = 2 * P.vmax + 1;
  for (int base = 0; base < np; base += kBlock) {
    const int t = base + (int)threadIdx.x;
    const bool valid = t < np;
    int sitek = 0, bink = 0;
    bool inside = false;
    int v[D];
#pragma unroll
    for (int q = 0; q < D; ++q) v[q] = 0;
    if (valid) {
      int lo = 0, hi = nrows - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_rp[mid] <= t) lo = mid; else hi = mid - 1;
      }
      const int g = s_rg[lo] + (t - s_rp[lo]);
      int c[D], im[D], u[D], pu[D];
      float o[D], po[D];
      cell_coords<D>(a.cell[g] - R.cell_off, R, c);
      ldi<D>(a.img, g, im);
      ldv<D>(a.pos, g, o);
#pragma unroll
      for (int q = 0; q < D; ++q) u[q] = c[q] + R.Mc[q] * im[q];
      if (!a.snapshot_only) {
        ldi<D>(a.prev_u, g, pu);
        ldv<D>(a.prev_off, g, po);
        inside = true;
        int bin = 0, stride = 1;
#pragma unroll
        for (int q = 0; q < D; ++q) {
          v[q] = (u[q] >> P.log2k) - (pu[q] >> P.log2k);
          inside = inside && (v[q] >= -P.vmax) && (v[q] <= P.vmax);
          bin += (v[q] + P.vmax) * stride;
          stride *= W;
          const double dd = (double)(u[q] - pu[q]) * P.s_d + ((double)o[q] - (double)po[q]);
          ds[q] += dd;
          dq[q] += dd * dd;
        }
        sitek = ((c[1] >> P.log2k) - sy0) * a.BSX + (c[0] >> P.log2k) - sx0;
        bink = sitek * Q + (inside ? bin : 0);
      }
      sti<D>(a.prev_u, g, u);
      stv<D>(a.prev_off, g, o);
    }
    if (!a.snapshot_only) {
      wave_agg_add(s_h, bink, valid && inside);
      wave_agg_add_i(s_m, sitek * nm, valid);
      if (valid) {
        int* m = s_m + sitek * nm;
        if (!inside) atomicAdd(m + 1, 1);
        int kk = 2 + D;
#pragma unroll
        for (int p = 0; p < D; ++p) {
          if (v[p] != 0) atomicAdd(m + 2 + p, v[p]);
#pragma unroll
          for (int q = p; q < D; ++q) {
            const int pr = v[p] * v[q];
            if (pr != 0) atomicAdd(m + kk, pr);
            ++kk;
          }
        }
      }
    }
  }
  if (a.snapshot_only) return;
  if (a.shift_k && sb == 0 && threadIdx.x == 0) *a.shift_k += 1;
  __syncthreads();
  // flush, row by row of the strip: this block is the only writer of its
  // sites; atomics without a return value let every update leave without
  // waiting for the read
  const int sy_lin = (D == 2) ? R.M[0] * sy0 : R.M[0] * (sy0 + R.M[1] * sz);
  const size_t site0 = (size_t)R.site_off + sy_lin + sx0;  // first site of the first row
  {
    const int rq = wsx * Q;
    const float rrq = __builtin_amdgcn_rcpf((float)rq);
    for (int e = threadIdx.x; e < wsy * rq; e += kBlock) {
      int x;
      const int j = small_div(e, rq, rrq, x);
      const unsigned c = s_h[j * a.BSX * Q + x];
      const size_t ga = (site0 + (size_t)j * R.M[0]) * Q + x;
      if (c) atomicAdd(a.A + ga, c);
      if (a.nstep) a.nstep[ga] = c;
    }
    const int rm = wsx * nm;
    const float rrm = __builtin_amdgcn_rcpf((float)rm);
    for (int e = threadIdx.x; e < wsy * rm; e += kBlock) {
      int x;
      const int j = small_div(e, rm, rrm, x);
      const int c = s_m[j * a.BSX * nm + x];
      if (c)
        atomicAdd(reinterpret_cast<unsigned long long*>(a.mom) + (site0 + (size_t)j * R.M[0]) * nm + x,
                  (unsigned long long)(long long)c);
    }
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const double s1 = wave_sum_d(ds[q]);
    const double s2 = wave_sum_d(dq[q]);
    if (lane_id() == 0) {
      s_red[w][q] = s1;
      s_red[w][D + q] = s2;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * D) {
    double s = 0.0;
    for (int i = 0; i < kWaves; ++i) s += s_red[i][threadIdx.x];
    a.dpart[(size_t)sb * 2 * D + threadIdx.x] += s;
  }
}

// ---------------------------------------------------------------- readout

__global__ __launch_bounds__(kBlock) void k_fsum(FsumArgs a) {
  __shared__ unsigned long long s_q[kMaxQ];
  __shared__ long long s_m[16];
  for (int i = threadIdx.x; i < a.Q; i += kBlock) s_q[i] = 0ull;
  if (threadIdx.x < 16) s_m[threadIdx.x] = 0;
  __syncthreads();
  const long long s0 = (long long)blockIdx.x * a.sites_per_block;
  const long long s1 = min((long long)a.n_sites, s0 + a.sites_per_block);
  for (long long e = s0 * a.Q + threadIdx.x; e < s1 * a.Q; e += kBlock) {
    const unsigned c = a.A[e];
    if (c) atomicAdd(&s_q[e % a.Q], (unsigned long long)c);
  }
  for (long long e = s0 * a.nm + threadIdx.x; e < s1 * a.nm; e += kBlock) {
    const long long c = a.mom[e];
    if (c) atomicAdd(reinterpret_cast<unsigned long long*>(&s_m[e % a.nm]),
                     (unsigned long long)c);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < a.Q; i += kBlock)
    if (s_q[i]) atomicAdd(a.fcount + i, s_q[i]);
  if (threadIdx.x < a.nm && s_m[threadIdx.x])
    atomicAdd(reinterpret_cast<unsigned long long*>(a.momsum + threadIdx.x),
              (unsigned long long)s_m[threadIdx.x]);
}

__global__ void k_ffinal(FfinalArgs a) {
  for (int i = threadIdx.x; i < a.Q; i += kBlock)
    a.f[i] = a.denom > 0.0 ? (double)a.fcount[i] / a.denom : 0.0;
  if (threadIdx.x < a.nd) {
    double s = 0.0;
    for (int b = 0; b < a.nstrips; ++b) s += a.dpart[(size_t)b * a.nd + threadIdx.x];
    a.disp[threadIdx.x] = s;
  }
}

__global__ void k_site_avg(SiteAvgArgs a) {
  const long long tid = blockIdx.x * (long long)kBlock + threadIdx.x;
  const long long stride = (long long)gridDim.x * kBlock;
  if (a.f_site)
    for (long long e = tid; e < a.count * a.Q; e += stride)
      a.f_site[e] = (double)a.A[a.first * a.Q + e] * a.inv_T;
  if (a.mom_site)
    for (long long e = tid; e < a.count * a.nm; e += stride)
      a.mom_site[e] = (double)a.mom[a.first * a.nm + e] * a.inv_T;
}

// ---------------------------------------------------------------- state I/O

template <int D>
__global__ __launch_bounds__(kBlock) void k_export(XportArgs a) {
  const int4 ch = a.chunks[blockIdx.x];
  const Replica R = a.reps[ch.x];
  for (int g = ch.y + threadIdx.x; g < ch.z; g += kBlock) {
    float o[D], v[D];
    int c[D], im[D], u[D];
    ldv<D>(a.pos, g, o);
    ldi<D>(a.img, g, im);
    cell_coords<D>(a.cell[g] - R.cell_off, R, c);
    for (int k = 0; k < D; ++k) {
      (void)canon(o[k], c[k], im[k], R.Mc[k], a.P.s);
      u[k] = c[k] + R.Mc[k] * im[k];
    }
    ldv<D>(a.vel, g, v);
    const int pid = a.id[g];
    sti<D>(a.x_u, pid, u);
    stv<D>(a.x_off, pid, o);
    stv<D>(a.x_vel, pid, v);
    if (a.acc && a.x_acc) {
      float f[D];
      ldv<D>(a.acc, g, f);
      stv<D>(a.x_acc, pid, f);
    }
    int pu[D];
    float po[D];
    ldi<D>(a.prev_u, g, pu);
    ldv<D>(a.prev_off, g, po);
    sti<D>(a.x_pu, pid, pu);
    stv<D>(a.x_poff, pid, po);
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_import(XportArgs a) {
  const int4 ch = a.chunks[blockIdx.x];
  const Replica R = a.reps[ch.x];
  for (int g = ch.y + threadIdx.x; g < ch.z; g += kBlock) {
    int u[D], c[D], im[D];
    float o[D], v[D];
    ldi<D>(a.x_u, g, u);
    ldv<D>(a.x_off, g, o);
    ldv<D>(a.x_vel, g, v);
    for (int k = 0; k < D; ++k) {
      im[k] = floor_div(u[k], R.Mc[k]);
      c[k] = u[k] - im[k] * R.Mc[k];
    }
    stv<D>(a.pos, g, o);
    stv<D>(a.vel, g, v);
    sti<D>(a.img, g, im);
    a.id[g] = g;
    a.cell[g] = R.cell_off + cell_linear<D>(c, R);
    if (a.x_pu) {
      int pu[D];
      float po[D];
      ldi<D>(a.x_pu, g, pu);
      ldv<D>(a.x_poff, g, po);
      sti<D>(a.prev_u, g, pu);
      stv<D>(a.prev_off, g, po);
    }
  }
}

// ---------------------------------------------------------------- shifted lattices
//
// eq. (MDni) on lattices displaced by a_j + b_j k lattice spacings at lattice
// time k: a particle's cell is floor(x / dx + a_j + b_j k) per axis.  A drift
// b_j = u bins the Galilean-transformed positions x + u t (the section on the
// velocity dependence of the equilibrium), so the histogram is f_i for mean
// velocity u from one trajectory; static offsets a_j = m / K average over
// lattice placements (the remark on exact momentum after the one-particle
// table).  Per lattice j the block counts the window bins and the overflow
// (wave-aggregated LDS atomics) and sums the lattice displacement and its
// products over all particles; one atomic per non-zero counter and block.
template <int D>
__global__ __launch_bounds__(kBlock) void k_shift(ShiftArgs a) {
  constexpr int NM = D + D * (D + 1) / 2;
  const int Q = a.P.Q;
  const int per = Q + 1 + NM;
  __shared__ unsigned s_cnt[kMaxShifts * (kMaxQ + 1)];
  __shared__ int s_mom[kMaxShifts][NM];
  for (int e = threadIdx.x; e < a.n_shifts * (Q + 1); e += kBlock) s_cnt[e] = 0;
  for (int e = threadIdx.x; e < a.n_shifts * NM; e += kBlock) s_mom[e / NM][e % NM] = 0;
  __syncthreads();
  const double kk = (double)*a.shift_k;
  const int W = 2 * a.P.vmax + 1;
  for (int c = blockIdx.x; c < a.nchunks; c += gridDim.x) {
    const int4 ch = a.chunks[c];
    const Replica R = a.reps[ch.x];
    for (int g0 = ch.y; g0 < ch.z; g0 += kBlock) {
      const int g = g0 + (int)threadIdx.x;
      const bool valid = g < ch.z;
      double y[D], yp[D];
#pragma unroll
      for (int q = 0; q < D; ++q) {
        y[q] = 0.0;
        yp[q] = 0.0;
      }
      if (valid) {
        int cc[D], im[D], pu[D];
        float o[D], po[D];
        cell_coords<D>(a.cell[g] - R.cell_off, R, cc);
        ldi<D>(a.img, g, im);
        ldv<D>(a.pos, g, o);
        ldi<D>(a.prev_u, g, pu);
        ldv<D>(a.prev_off, g, po);
#pragma unroll
        for (int q = 0; q < D; ++q) {
          const int u = cc[q] + R.Mc[q] * im[q];
          y[q] = ((double)u * a.P.s_d + (double)o[q]) / a.dx;
          yp[q] = ((double)pu[q] * a.P.s_d + (double)po[q]) / a.dx;
        }
      }
      for (int j = 0; j < a.n_shifts; ++j) {
        const double* sh = a.shifts + (size_t)j * 2 * D;
        int v[D];
        bool inside = true;
        int bin = 0, stride = 1;
#pragma unroll
        for (int q = 0; q < D; ++q) {
          const double now = sh[q] + sh[D + q] * kk;
          const double before = sh[q] + sh[D + q] * (kk - 1.0);
          v[q] = (int)floor(y[q] + now) - (int)floor(yp[q] + before);
          inside = inside && v[q] >= -a.P.vmax && v[q] <= a.P.vmax;
          bin += (v[q] + a.P.vmax) * stride;
          stride *= W;
        }
        wave_agg_add(s_cnt + j * (Q + 1), inside ? bin : Q, valid);
        // moments summed across the wave first: every lane adds to the same
        // few LDS words, which would serialise
        {
          int kq = D;
#pragma unroll
          for (int p = 0; p < D; ++p) {
            const int sp = wave_sum_i(valid ? v[p] : 0);
            if (lane_id() == 0 && sp != 0) atomicAdd(&s_mom[j][p], sp);
#pragma unroll
            for (int q = p; q < D; ++q) {
              const int sq = wave_sum_i(valid ? v[p] * v[q] : 0);
              if (lane_id() == 0 && sq != 0) atomicAdd(&s_mom[j][kq], sq);
              ++kq;
            }
          }
        }
      }
    }
  }
  __syncthreads();
  // into the copy of this block's XCD (every block adds to the same few
  // counters; same-address atomics from many blocks serialise)
  unsigned long long* __restrict__ acc =
      a.acc + (size_t)(blockIdx.x & (kTileCopies - 1)) * a.n_shifts * per;
  for (int e = threadIdx.x; e < a.n_shifts * (Q + 1); e += kBlock) {
    const unsigned c = s_cnt[e];
    if (c) atomicAdd(acc + (size_t)(e / (Q + 1)) * per + e % (Q + 1), (unsigned long long)c);
  }
  for (int e = threadIdx.x; e < a.n_shifts * NM; e += kBlock) {
    const int m = s_mom[e / NM][e % NM];
    if (m) atomicAdd(acc + (size_t)(e / NM) * per + Q + 1 + e % NM, (unsigned long long)(long long)m);
  }
}

// ---------------------------------------------------------------- collision operator
//
// Xi_i(x, t) = n_i(x + v_i, t + dt_L) - n_i(x, t) (eq. Xi), from the arrival
// histograms of two consecutive lattice steps: n_i(x + v_i, t + dt_L) counts
// the particles that sat in x at t and moved by v_i.  A block takes a run of
// sites; thread t owns bin t % Q for every (256 / Q)-th site of the run, so
// the reads of n_i(x, t) are coalesced and each thread keeps its bin's sums
// of Xi, Xi^2, Xi n, n and n^2 (n = n_i(x, t), the populations Xi acts on)
// in registers.  x + v_i wraps periodically inside the site's replica.  The
// block's per-bin sums go to its own row of partials; k_xi_reduce adds the
// rows into the running totals.
template <int D>
__global__ __launch_bounds__(kBlock) void k_xi(XiArgs a) {
  __shared__ long long s_acc[5][kMaxQ];
  const int Q = a.Q;
  const int lanes = kBlock / Q;
  const int tid = threadIdx.x;
  const bool act = tid < lanes * Q;
  const int i = tid % Q, ls = tid / Q;
  for (int e = tid; e < 5 * Q; e += kBlock) s_acc[e / Q][e % Q] = 0;
  __syncthreads();
  const int W = 2 * a.vmax + 1;
  int v[3] = {i % W - a.vmax, (i / W) % W - a.vmax, 0};
  if constexpr (D == 3) v[2] = i / (W * W) - a.vmax;
  long long acc[5] = {0, 0, 0, 0, 0};
  const int s0 = blockIdx.x * a.sites_per_block;
  const int s1 = min(a.n_sites, s0 + a.sites_per_block);
  if (act) {
    for (int site = s0 + ls; site < s1; site += lanes) {
      int lo = 0, hi = a.n_rep - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.reps[mid].site_off <= site) lo = mid; else hi = mid - 1;
      }
      const Replica& R = a.reps[lo];
      const int local = site - R.site_off;
      int c[3] = {local % R.M[0], (local / R.M[0]) % R.M[1], 0};
      if constexpr (D == 3) c[2] = local / (R.M[0] * R.M[1]);
      int dst = 0, stride = 1;
#pragma unroll
      for (int q = 0; q < D; ++q) {
        int y = c[q] + v[q];
        while (y < 0) y += R.M[q];
        while (y >= R.M[q]) y -= R.M[q];
        dst += y * stride;
        stride *= R.M[q];
      }
      const size_t idx = (size_t)site * Q + i;
      const long long n0 = a.nprev[idx];
      const long long xi = (long long)a.ncur[((size_t)R.site_off + dst) * Q + i] - n0;
      a.xi_site[idx] += xi;
      a.xi_last[idx] = (int)xi;
      acc[0] += xi;
      acc[1] += xi * xi;
      acc[2] += xi * n0;
      acc[3] += n0;
      acc[4] += n0 * n0;
    }
#pragma unroll
    for (int k = 0; k < 5; ++k)
      if (acc[k]) atomicAdd(reinterpret_cast<unsigned long long*>(&s_acc[k][i]),
                            (unsigned long long)acc[k]);
  }
  __syncthreads();
  for (int e = tid; e < 5 * Q; e += kBlock)
    a.part[(size_t)blockIdx.x * 5 * Q + e] = s_acc[e / Q][e % Q];
}

// One block per (sum, bin): its threads stride over the per-block rows.
__global__ __launch_bounds__(kBlock) void k_xi_reduce(XiArgs a) {
  __shared__ long long s_red[kWaves];
  const int e = blockIdx.x;
  long long s = 0;
  for (int b = threadIdx.x; b < a.nblocks; b += kBlock) s += a.part[(size_t)b * 5 * a.Q + e];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane_id() == 0) s_red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int w = 0; w < kWaves; ++w) t += s_red[w];
    a.sums[e] += (unsigned long long)t;
  }
}

// ---------------------------------------------------------------- launchers

thread_local LaunchEvents g_launch_events;

// One launch; with events pending (per-kernel timing) through
// hipExtLaunchKernelGGL, which records them around the kernel.
#define MDLG_GO(kern, grid, block, lds, stream, args)                                         \
  do {                                                                                      \
    if (g_launch_events.start) {                                                            \
      hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), (std::uint32_t)(lds), stream,     \
                            g_launch_events.start, g_launch_events.stop, 0u, args);         \
      g_launch_events = LaunchEvents{};                                                     \
    } else {                                                                                \
      hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, stream, args);                 \
    }                                                                                       \
  } while (0)

#define MDLG_LAUNCH_DIM(D, kern, grid, lds, stream, args)            \
  do {                                                               \
    if ((D) == 2)                                                    \
      MDLG_GO(kern<2>, grid, kBlock, lds, stream, args);             \
    else                                                             \
      MDLG_GO(kern<3>, grid, kBlock, lds, stream, args);             \
  } while (0)

// A single wave that waits until the device's constant-rate wall clock has
// advanced by `ticks` (the clock always advances, so the wait ends).  A kernel
// of known length: event pairs recorded around it read that length plus the
// constant the events themselves add.
__global__ void k_clock_wait(long long ticks) {
  const long long t0 = wall_clock64();
  while (wall_clock64() - t0 < ticks) {
  }
}

void launch_clock_wait(long long ticks, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  hipExtLaunchKernelGGL(k_clock_wait, dim3(1), dim3(64), 0u, s, start, stop, 0u, ticks);
}

void launch_fill_u32(unsigned* p, unsigned v, long long n, hipStream_t s) {
  if (n <= 0) return;
  long long blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(kBlock), 0, s, p, v, n);
}

void launch_fill_f32(float* p, float v, long long n, hipStream_t s) {
  if (n <= 0) return;
  long long blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)blocks), dim3(kBlock), 0, s, p, v, n);
}

void launch_ingest(int D, int nchunks, const IngestArgs& a, hipStream_t s) {
  MDLG_LAUNCH_DIM(D, k_ingest, nchunks, 0, s, a);
}

void launch_count(int D, int nchunks, const SortArgs& a, hipStream_t s) {
  const int grid = a.xcd_remap ? (nchunks + 7) / 8 * 8 : nchunks;
  MDLG_LAUNCH_DIM(D, k_count, grid, 0, s, a);
}

void launch_scan(const ScanArgs& a, hipStream_t s) {
  MDLG_GO(k_scan, a.ntiles, kBlock, 0, s, a);
}

void launch_scatter(int D, int nchunks, const SortArgs& a, hipStream_t s) {
  const int grid = a.xcd_remap ? (nchunks + 7) / 8 * 8 : nchunks;
  MDLG_LAUNCH_DIM(D, k_scatter, grid, 0, s, a);
}

void launch_cellsort(int D, int nchunks, const CellsortArgs& a, hipStream_t s) {
  MDLG_LAUNCH_DIM(D, k_cellsort, nchunks, 0, s, a);
}

void launch_rescale(int D, int nchunks, const RescaleArgs& a, hipStream_t s) {
  MDLG_LAUNCH_DIM(D, k_rescale, nchunks, 0, s, a);
}

size_t brick_lds_bytes(const Phys& P, int D, bool adj) {
  const size_t coord = (D == 2) ? sizeof(int2) : sizeof(int4);
  return brick_lds_layout(P.lcap, 0, coord, adj ? D * sizeof(float) : 0, P.lmaxh).end;
}

// Brick kernels come in 64-, 128- and 256-thread blocks (P.bthreads).
#define MDLG_LAUNCH_BRICK(D, NT, kern, grid, lds, stream, args)                 \
  do {                                                                          \
    if ((NT) == 64) {                                                           \
      if ((D) == 2) MDLG_GO((kern<2, 64>), grid, 64, lds, stream, args);        \
      else MDLG_GO((kern<3, 64>), grid, 64, lds, stream, args);                 \
    } else if ((NT) == 128) {                                                   \
      if ((D) == 2) MDLG_GO((kern<2, 128>), grid, 128, lds, stream, args);      \
      else MDLG_GO((kern<3, 128>), grid, 128, lds, stream, args);               \
    } else {                                                                    \
      if ((D) == 2) MDLG_GO((kern<2, 256>), grid, 256, lds, stream, args);      \
      else MDLG_GO((kern<3, 256>), grid, 256, lds, stream, args);               \
    }                                                                           \
  } while (0)

void launch_force(int D, const ForceArgs& a, hipStream_t s) {
  int grid = a.nbricks;
  if (a.xcd_remap) grid = ((a.nbricks + 7) / 8) * 8;
  MDLG_LAUNCH_BRICK(D, a.P.bthreads, k_force, grid, brick_lds_bytes(a.P, D, false), s, a);
}

void launch_nlist(int D, const NlistArgs& a, hipStream_t s) {
  int grid = a.nbricks;
  if (a.xcd_remap) grid = ((a.nbricks + 7) / 8) * 8;
  // the brick's LDS (14-bit coordinates) plus one byte per target for the
  // list word counts
  const size_t coord = (D == 2) ? sizeof(unsigned) : sizeof(uint2);
  const size_t lds = brick_lds_layout(a.P.lcap, kNlPad, coord, 0, a.P.lmaxh).end + (size_t)a.P.lcap;
  // 16 or 32 candidates per test step: separate instantiations, so that
  // neither carries the other's registers
  if (a.P.nl_wide) MDLG_LAUNCH_BRICK(D, a.P.bthreads, k_nlist_wide, grid, lds, s, a);
  else MDLG_LAUNCH_BRICK(D, a.P.bthreads, k_nlist_narrow, grid, lds, s, a);
}

void launch_kinpart(int D, int nchunks, const KinPartArgs& a, hipStream_t s) {
  MDLG_LAUNCH_DIM(D, k_kinpart, nchunks, 0, s, a);
}

void launch_kin(const KinArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_kin, dim3(a.n_rep), dim3(kBlock), 0, s, a);
}

void launch_bin(int D, int nstrips, const BinArgs& a, hipStream_t s) {
  const size_t lds = (size_t)a.BSX * a.BSY * (a.P.Q + a.P.nm) * sizeof(int);
  MDLG_LAUNCH_DIM(D, k_bin, nstrips, lds, s, a);
}

void launch_shift(int D, const ShiftArgs& a, hipStream_t s) {
  const int grid = a.nchunks < 1024 ? a.nchunks : 1024;
  if (grid <= 0 || a.n_shifts <= 0) return;
  MDLG_LAUNCH_DIM(D, k_shift, grid, 0, s, a);
}

void launch_xi(int D, const XiArgs& a, hipStream_t s) {
  if (a.nblocks <= 0) return;
  MDLG_LAUNCH_DIM(D, k_xi, a.nblocks, 0, s, a);
  hipLaunchKernelGGL(k_xi_reduce, dim3(5 * a.Q), dim3(kBlock), 0, s, a);
}

void launch_fsum(const FsumArgs& a, hipStream_t s) {
  const int blocks = (a.n_sites + a.sites_per_block - 1) / a.sites_per_block;
  hipLaunchKernelGGL(k_fsum, dim3(blocks), dim3(kBlock), 0, s, a);
}

void launch_ffinal(const FfinalArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_ffinal, dim3(1), dim3(kBlock), 0, s, a);
}

void launch_site_avg(const SiteAvgArgs& a, hipStream_t s) {
  long long n = a.count * (a.Q > a.nm ? a.Q : a.nm);
  long long blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_site_avg, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
}

void launch_adjoint(int D, const AdjArgs& a, hipStream_t s) {
  // the layout's block size, as for the force kernel
  MDLG_LAUNCH_BRICK(D, a.P.bthreads, k_adjoint, a.nbricks, brick_lds_bytes(a.P, D, true), s, a);
}

void launch_adjoint_force(int D, const AdjForceArgs& a, hipStream_t s) {
  // both parts take the layout's block size; the LDS is the larger of the two
  const size_t la = brick_lds_bytes(a.adj.P, D, true), lf = brick_lds_bytes(a.force.P, D, false);
  const size_t lds = la > lf ? la : lf;
  MDLG_LAUNCH_BRICK(D, a.adj.P.bthreads, k_adjoint_force, a.adj.nbricks + a.force.nbricks, lds, s, a);
}

static int grid_for(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

void launch_adj_loss(int D, const AdjLossArgs& a, hipStream_t s) {
  MDLG_LAUNCH_DIM(D, k_adj_loss, a.nblocks, 0, s, a);
}

void launch_adj_final(const AdjFinalArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_final, dim3(1), dim3(kBlock), 0, s, a);
}

void launch_adj_io(int D, const AdjIoArgs& a, hipStream_t s) {
  MDLG_LAUNCH_DIM(D, k_adj_io, grid_for(a.n), 0, s, a);
}

void launch_copy_f32(const float* src, float* dst, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(n)), dim3(kBlock), 0, s, src, dst, n);
}

void launch_export(int D, int nchunks, const XportArgs& a, hipStream_t s) {
  MDLG_LAUNCH_DIM(D, k_export, nchunks, 0, s, a);
}

void launch_import(int D, int nchunks, const XportArgs& a, hipStream_t s) {
  MDLG_LAUNCH_DIM(D, k_import, nchunks, 0, s, a);
}

}  // namespace mdlg
