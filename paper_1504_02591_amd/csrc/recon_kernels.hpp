// Kernels of the reconstruction hot path.
//
// Memory layout (per realisation, b-th block of each buffer):
//   real field      [z][y][x]              N^3 float, x fastest
//   int64 grid      [z][y][x]              N^3 int64 (units of 2^-32 weight)
//   spectrum C      [kz][ky][kx]           (N/2+1) N N float2; kz is the halved axis
// Forward 3D transforms run z (real-to-complex, two real columns packed per
// complex column), then y, then x; inverse transforms run x, y, z.  Every
// k-space multiplier is applied inside the pass where its wavenumber index is
// known, so the fan-out Psi_j = i k'_j P and the fan-in div = sum_j i k'_j V_j
// are staged across passes instead of transforming three fields end to end.
#pragma once

#include "recon_device.hpp"

namespace recon {

// Geometry and physics constants shared by the transform kernels.
struct Geo {
  float kf;          // fundamental wavenumber 2 pi / L
  float hs;          // cell size divided by the line-of-sight scale R0 (a power of two)
  float ds[3];       // (box origin - observer) / R0, per axis
  float growth;      // f
  float inv_bn3;     // 1 / (b N^3): Zel'dovich solve including the inverse-transform factor
  float smooth_c;    // R^2 / 2
  float inv_n3;      // 1 / N^3
  float start_scale; // u_0 = start_scale * u_p for the FFTA starts
};

// Per-realisation scalars of the overdensity step.
struct DeltaScal {
  float alpha;       // W_g / W_r
  float inv_rhobar;  // N^3 / W_g (mean-density mode)
};

// Cloud-in-cell frame: u = fl32(fl32(x - o) * s), s = fl32(N / L).
struct CicGeo {
  int n;
  float s;
  float o[3];
};

enum ZIterMode { ZI_PLAIN = 0, ZI_FFTA = 1, ZI_LEARNED = 2, ZI_CROSS = 3 };

// The displacement buffer is planar, [b][3][N^3] floats with x fastest (the layout recon_get_psi
// hands out): the final z pass then writes whole 128-byte lines (a tile's 32 consecutive x of one
// component), 12 bytes per node, and the shift reads each component's rows.

// Tile shapes (compile-time tuning knobs from recon_tuning.h): packed z columns, y-pass columns,
// x-pass rows.  Each block runs one radix-8 fragment per thread, (N/8) * tile threads.
constexpr int cmin(int a, int b) { return a < b ? a : b; }
// Knobs per grid size: the 256^3 and 1024^3 values are tuned on their own (recon_tuning.h), every
// other size takes the general value.
template <int N> constexpr int tile_z() { return N == 256 ? RECON_TILE_Z_256 : RECON_TILE_Z; }
template <int N> constexpr int tile_y() { return N == 256 ? RECON_TILE_Y_256 : RECON_TILE_Y; }
template <int N> constexpr int tile_x() {
  return N == 256 ? RECON_TILE_X_256 : (N == 1024 ? RECON_TILE_X_1024 : RECON_TILE_X);
}
template <int N> constexpr int z_tpb() {
  return N == 256 ? RECON_Z_TPB_256 : (N == 1024 ? RECON_Z_TPB_1024 : RECON_Z_TPB);
}
// (1024-point columns need 8-column tiles to fit the LDS)
template <int N> constexpr int wz() { return N >= 1024 ? 8 : cmin(N / 2, tile_z<N>()); }
template <int N> constexpr int wy() { return N >= 1024 ? 8 : cmin(N, tile_y<N>()); }
template <int N> constexpr int wx() { return tile_x<N>(); }
// z tiles (one y row, 2 wz consecutive x) and tiles per block of the z iteration
template <int N> constexpr int ztiles() { return N * (N / (2 * wz<N>())); }
// (the start and cross modes and the matrix-core radix variants, which hold more live state, take one
// tile per block)
template <int N, int MODE, int SPLIT = 0> constexpr int ztpb() {
  return MODE == ZI_PLAIN && SPLIT == 0 ? cmin(z_tpb<N>(), ztiles<N>()) : 1;
}


__device__ __forceinline__ long long ceil_div_ll(long long a, long long b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Fill, deposit, totals, mask
// ---------------------------------------------------------------------------
__global__ void k_fill_u64(unsigned long long* p, long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__global__ void k_fill_i32(int* p, long long count, int v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__device__ __forceinline__ int find_realisation(const long long* __restrict__ off, int batch, long long i) {
  int lo = 0, hi = batch - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Integer CIC shares of one object: corner k = (dx, dy, dz) gets floor(W_Q c_k / 2^48) with
// c_k = a_x a_y a_z, a = 2^16 - tau or tau per axis, for the first seven corners, and corner (1,1,1)
// the remainder, so the eight shares add up to W_Q exactly.  For a unit weight (W_Q = 2^32) the share
// is floor(c_k / 2^16); c_k <= 2^48 is formed exactly in FP64 at full rate instead of with 64-bit
// integer products (the same integers either way).
__device__ __forceinline__ void cic_shares(unsigned long long wq, const unsigned long long tau[3],
                                           unsigned long long share[8]) {
  unsigned long long sum = 0;
  if (wq == (1ull << 32)) {
    const double ax[2] = {(double)(65536u - (unsigned)tau[0]), (double)(unsigned)tau[0]};
    const double ay[2] = {(double)(65536u - (unsigned)tau[1]), (double)(unsigned)tau[1]};
    const double az[2] = {(double)(65536u - (unsigned)tau[2]), (double)(unsigned)tau[2]};
#pragma unroll
    for (int cnr = 0; cnr < 7; ++cnr) {
      const double c = ax[cnr & 1] * ay[(cnr >> 1) & 1] * az[cnr >> 2];
      const double f = floor(c * 0x1p-16);
      share[cnr] = f >= 0x1p32 ? (1ull << 32) : (unsigned long long)(unsigned)f;
      sum += share[cnr];
    }
  } else {
#pragma unroll
    for (int cnr = 0; cnr < 7; ++cnr) {
      const int dx = cnr & 1, dy = (cnr >> 1) & 1, dz = cnr >> 2;
      const unsigned long long ax = dx ? tau[0] : 65536ull - tau[0];
      const unsigned long long ay = dy ? tau[1] : 65536ull - tau[1];
      const unsigned long long az = dz ? tau[2] : 65536ull - tau[2];
      const unsigned long long c = ax * ay * az;
      const unsigned long long chi = c >> 24, clo = c & 0xFFFFFFull;
      share[cnr] = (wq * chi + ((wq * clo) >> 24)) >> 24;
      sum += share[cnr];
    }
  }
  share[7] = wq - sum;
}

// The rounded value itself, opaque to the compiler: u = fl(fl(x - o) s) stays one rounding, so the
// fraction t = u - floor(u) is formed from it and never fused into fma(s, x - o, -floor(u)) (which the
// backend otherwise does in some kernels and not in others).  No instruction is emitted.
__device__ __forceinline__ float keep_rounded(float v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Nearest-grid-point deposit in the same fixed point: the whole W_Q goes to node i + 1 when the
// FP32 fraction is at least 1/2, else to node i (per axis, periodic).
__global__ void __launch_bounds__(256) k_paint_ngp(const float* __restrict__ pos, const float* __restrict__ w,
                                                   long long n, const long long* __restrict__ off, int batch,
                                                   unsigned long long* __restrict__ grid, CicGeo g,
                                                   int* __restrict__ err) {
  const long long n3 = (long long)g.n * g.n * g.n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    bool ok = true;
    float uu[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float d = __fsub_rn(pos[3 * i + a], g.o[a]);
      uu[a] = keep_rounded(__fmul_rn(d, g.s));
      ok = ok && (fabsf(uu[a]) < 1073741824.0f);
    }
    const float wv = w ? w[i] : 1.0f;
    ok = ok && (wv >= 0.0f) && (wv < 64.0f);
    if (!ok) { atomicAdd(err, 1); continue; }
    long long ii[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float fl = floorf(uu[a]);
      const float t = __fsub_rn(uu[a], fl);
      ii[a] = ((int)fl + (t >= 0.5f ? 1 : 0)) & (g.n - 1);
    }
    const unsigned long long wq = w ? (unsigned long long)__double2ll_rn((double)wv * 4294967296.0)
                                    : (1ull << 32);
    const int b = off ? find_realisation(off, batch, i) : 0;
    const long long cell = (ii[2] * g.n + ii[1]) * g.n + ii[0];
    if (wq && in_bounds(cell, n3)) atomicAdd(grid + (long long)b * n3 + cell, wq);
  }
}

// Integer fixed-point CIC deposit.  Seven corners get floor(W_Q c / 2^48) and
// corner (1,1,1) the remainder, so every object deposits exactly W_Q; integer
// atomics make the grid independent of the order of the objects.
__global__ void __launch_bounds__(256) k_paint(const float* __restrict__ pos, const float* __restrict__ w,
                                               long long n, const long long* __restrict__ off, int batch,
                                               unsigned long long* __restrict__ grid, CicGeo g,
                                               int* __restrict__ err) {
  const long long n3 = (long long)g.n * g.n * g.n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    bool ok = true;
    float uu[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float d = __fsub_rn(pos[3 * i + a], g.o[a]);
      uu[a] = keep_rounded(__fmul_rn(d, g.s));
      ok = ok && (fabsf(uu[a]) < 1073741824.0f);   // false for NaN / inf too
    }
    float wv = w ? w[i] : 1.0f;
    ok = ok && (wv >= 0.0f) && (wv < 64.0f);
    if (!ok) { atomicAdd(err, 1); continue; }
    int ii[3];
    unsigned long long tau[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float fl = floorf(uu[a]);
      float t = __fsub_rn(uu[a], fl);
      tau[a] = (unsigned long long)floorf(t * 65536.0f);
      ii[a] = ((int)fl) & (g.n - 1);
    }
    const unsigned long long wq = w ? (unsigned long long)__double2ll_rn((double)wv * 4294967296.0)
                                    : (1ull << 32);
    const int b = off ? find_realisation(off, batch, i) : 0;
    unsigned long long* gb = grid + (long long)b * n3;
    unsigned long long share[8];
    cic_shares(wq, tau, share);
#pragma unroll
    for (int cnr = 0; cnr < 8; ++cnr) {
      const int dx = cnr & 1, dy = (cnr >> 1) & 1, dz = cnr >> 2;
      const long long ix = (ii[0] + dx) & (g.n - 1);
      const long long iy = (ii[1] + dy) & (g.n - 1);
      const long long iz = (ii[2] + dz) & (g.n - 1);
      const long long cell = (iz * g.n + iy) * g.n + ix;
      if (share[cnr] && in_bounds(cell, n3)) atomicAdd(gb + cell, share[cnr]);
    }
  }
}

// ---------------------------------------------------------------------------
// Brick-binned deposit: objects are counted per BS^3 brick of their base cell,
// scattered into brick order, and each brick is accumulated in LDS before a
// coalesced flush.  Same integer shares as k_paint, so the grid is identical.
// ---------------------------------------------------------------------------
constexpr int kBrick = 16;

// Brick of this block in a launch of one block per brick: each XCD (workgroups are dealt to the 8
// XCDs round robin) takes a contiguous range of bricks, so x-adjacent bricks, which share halo and
// output lines, run together on one L2 (identity when the brick count is not a multiple of 8).
__device__ __forceinline__ long long brick_of_block() {
  const long long nblk = gridDim.x;
  return (nblk & 7) ? (long long)blockIdx.x : (long long)(blockIdx.x & 7) * (nblk >> 3) + (blockIdx.x >> 3);
}
constexpr int kLdsBins = 32768;   // bins a block histograms in LDS (128 KB)

// Cell coordinate of an object; false for a non-finite / far position or a bad weight.
__device__ __forceinline__ bool cic_locate(float px, float py, float pz, float wv, const CicGeo& g, int ii[3],
                                           unsigned long long tau[3]) {
  const float pp[3] = {px, py, pz};
  float uu[3];
  bool ok = (wv >= 0.0f) && (wv < 64.0f);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float d = __fsub_rn(pp[a], g.o[a]);
    uu[a] = keep_rounded(__fmul_rn(d, g.s));
    ok = ok && (fabsf(uu[a]) < 1073741824.0f);
  }
  if (!ok) return false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float fl = floorf(uu[a]);
    float t = __fsub_rn(uu[a], fl);
    tau[a] = (unsigned long long)floorf(t * 65536.0f);
    ii[a] = ((int)fl) & (g.n - 1);
  }
  return true;
}

__device__ __forceinline__ long long brick_key(const int ii[3], int n, int b) {
  const int nbs = (n + kBrick - 1) / kBrick;
  return (long long)b * nbs * nbs * nbs + ((long long)(ii[2] / kBrick) * nbs + ii[1] / kBrick) * nbs + ii[0] / kBrick;
}

// Objects handled per loop trip by the deposit and shift loops: their loads are issued together so that
// their latencies overlap (each thread still takes the same objects in the same order).
constexpr int kObjBatch = RECON_OBJ_BATCH;

// Positions and weights of objects i0 + u * stride, u < U; an index at or past hi loads object hi - 1
// instead (in bounds; the caller skips it).  Requires i0 < hi.
template <int U>
__device__ __forceinline__ void load_objects(const float* __restrict__ pos, const float* __restrict__ w, long long i0,
                                             long long stride, long long hi, float px[U], float py[U], float pz[U],
                                             float wv[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    long long i = i0 + (long long)u * stride;
    if (i >= hi) i = hi - 1;
    px[u] = pos[3 * i];
    py[u] = pos[3 * i + 1];
    pz[u] = pos[3 * i + 2];
    wv[u] = w ? w[i] : 1.0f;
  }
}

__global__ void __launch_bounds__(256) k_bin_count(const float* __restrict__ pos, const float* __restrict__ w,
                                                   long long n, const long long* __restrict__ off, int batch,
                                                   CicGeo g, unsigned* __restrict__ counts, int* __restrict__ err) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    int ii[3];
    unsigned long long tau[3];
    if (!cic_locate(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], w ? w[i] : 1.0f, g, ii, tau)) {
      atomicAdd(err, 1);
      continue;
    }
    const int b = off ? find_realisation(off, batch, i) : 0;
    atomicAdd(counts + brick_key(ii, g.n, b), 1u);
  }
}

__global__ void __launch_bounds__(256) k_bin_scatter(const float* __restrict__ pos, const float* __restrict__ w,
                                                     long long n, const long long* __restrict__ off, int batch,
                                                     CicGeo g, unsigned* __restrict__ cursor,
                                                     float4* __restrict__ sorted, unsigned* __restrict__ slot_of) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    int ii[3];
    unsigned long long tau[3];
    const float px = pos[3 * i], py = pos[3 * i + 1], pz = pos[3 * i + 2], wv = w ? w[i] : 1.0f;
    if (!cic_locate(px, py, pz, wv, g, ii, tau)) {
      slot_of[i] = 0xFFFFFFFFu;   // not in the sorted copy
      continue;
    }
    const int b = off ? find_realisation(off, batch, i) : 0;
    const unsigned slot = atomicAdd(cursor + brick_key(ii, g.n, b), 1u);
    sorted[slot] = make_float4(px, py, pz, wv);
    slot_of[i] = slot;
  }
}

// Count with a per-block LDS histogram over the bins of the realisation that owns the
// chunk's first object; one global atomic per (block, non-empty bin).  Objects whose bin
// lies outside that window (a chunk crossing realisations) use a direct global atomic.
// The block's histogram is also stored in bhist[block][bin] (when not null), so that the scatter,
// which splits the catalogue into the same chunks, need not count again.
// First brick key of the LDS window of the binning block that takes objects [lo, ...): the block's
// realisation when all of its bricks fit (every size up to 512^3); above that, kLdsBins bricks centred
// on the brick of the chunk's first object, inside its realisation, so that a catalogue stored in
// spatial order (a lattice formed plane by plane) keeps each block's objects in its window.  Objects
// outside the window go to global atomics; the count and the scatter take the same window.
__device__ __forceinline__ long long bin_window(const float* __restrict__ pos, long long lo,
                                                const long long* __restrict__ off, int batch, const CicGeo& g) {
  const int nbs = (g.n + kBrick - 1) / kBrick;
  const long long per = (long long)nbs * nbs * nbs;
  const int b = off ? find_realisation(off, batch, lo) : 0;
  const long long rb = (long long)b * per;
  if (per <= kLdsBins) return rb;
  int ii[3];
  unsigned long long tau[3];
  if (!cic_locate(pos[3 * lo], pos[3 * lo + 1], pos[3 * lo + 2], 1.0f, g, ii, tau)) return rb;
  long long base = brick_key(ii, g.n, b) - kLdsBins / 2;
  if (base < rb) base = rb;
  if (base > rb + per - kLdsBins) base = rb + per - kLdsBins;
  return base;
}

template <int NT>
__global__ void __launch_bounds__(NT) k_bin_count_lds(const float* __restrict__ pos, const float* __restrict__ w,
                                                       long long n, long long chunk,
                                                       const long long* __restrict__ off, int batch, CicGeo g,
                                                       unsigned* __restrict__ counts, int* __restrict__ err,
                                                       unsigned* __restrict__ bhist) {
  __shared__ unsigned hist[kLdsBins];
  const long long lo = blockIdx.x * chunk;
  if (lo >= n) return;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  const int nbs = (g.n + kBrick - 1) / kBrick;
  const long long per = (long long)nbs * nbs * nbs;
  const long long base = bin_window(pos, lo, off, batch, g);
  for (int i = threadIdx.x; i < kLdsBins; i += NT) hist[i] = 0u;
  __syncthreads();
  constexpr int U = kObjBatch;
  for (long long i0 = lo + threadIdx.x; i0 < hi; i0 += (long long)NT * U) {
    float px[U], py[U], pz[U], wv[U];
    load_objects<U>(pos, w, i0, NT, hi, px, py, pz, wv);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = i0 + (long long)u * NT;
      if (i >= hi) break;
      int ii[3];
      unsigned long long tau[3];
      if (!cic_locate(px[u], py[u], pz[u], wv[u], g, ii, tau)) {
        atomicAdd(err, 1);
        continue;
      }
      const int b = off ? find_realisation(off, batch, i) : 0;
      const long long key = brick_key(ii, g.n, b);
      const long long rel = key - base;
      if (rel >= 0 && rel < kLdsBins) atomicAdd(&hist[rel], 1u);
      else atomicAdd(counts + key, 1u);
    }
  }
  __syncthreads();
  const long long nb_total = per * batch;
  for (int i = threadIdx.x; i < kLdsBins; i += NT) {
    const unsigned c = hist[i];
    if (c && base + i < nb_total) atomicAdd(counts + base + i, c);
    if (bhist) bhist[(long long)blockIdx.x * kLdsBins + i] = c;
  }
}

// Scatter into brick order: each block reserves one contiguous slot range per non-empty
// bin of its window, then ranks its objects inside the range with LDS atomics.
template <int NT>
__global__ void __launch_bounds__(NT) k_bin_scatter_lds(const float* __restrict__ pos, const float* __restrict__ w,
                                                         long long n, long long chunk,
                                                         const long long* __restrict__ off, int batch, CicGeo g,
                                                         unsigned* __restrict__ cursor, float4* __restrict__ sorted,
                                                         unsigned* __restrict__ slot_of,
                                                         const unsigned* __restrict__ bhist) {
  __shared__ unsigned hist[kLdsBins];
  const long long lo = blockIdx.x * chunk;
  if (lo >= n) return;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  const int nbs = (g.n + kBrick - 1) / kBrick;
  const long long per = (long long)nbs * nbs * nbs;
  const long long base = bin_window(pos, lo, off, batch, g);
  const long long nb_total = per * batch;
  if (bhist) {
    // the count kernel's histogram of this very chunk
    for (int i = threadIdx.x; i < kLdsBins; i += NT) hist[i] = bhist[(long long)blockIdx.x * kLdsBins + i];
  } else {
    for (int i = threadIdx.x; i < kLdsBins; i += NT) hist[i] = 0u;
    __syncthreads();
    for (long long i = lo + threadIdx.x; i < hi; i += NT) {
      int ii[3];
      unsigned long long tau[3];
      if (!cic_locate(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], w ? w[i] : 1.0f, g, ii, tau)) continue;
      const int b = off ? find_realisation(off, batch, i) : 0;
      const long long rel = brick_key(ii, g.n, b) - base;
      if (rel >= 0 && rel < kLdsBins) atomicAdd(&hist[rel], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kLdsBins; i += NT) {
    const unsigned c = hist[i];
    if (c && base + i < nb_total) hist[i] = atomicAdd(cursor + base + i, c);
  }
  __syncthreads();
  constexpr int U = kObjBatch;
  for (long long i0 = lo + threadIdx.x; i0 < hi; i0 += (long long)NT * U) {
    float px[U], py[U], pz[U], wv[U];
    load_objects<U>(pos, w, i0, NT, hi, px, py, pz, wv);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = i0 + (long long)u * NT;
      if (i >= hi) break;
      int ii[3];
      unsigned long long tau[3];
      if (!cic_locate(px[u], py[u], pz[u], wv[u], g, ii, tau)) {
        slot_of[i] = 0xFFFFFFFFu;   // not in the sorted copy
        continue;
      }
      const int b = off ? find_realisation(off, batch, i) : 0;
      const long long key = brick_key(ii, g.n, b);
      const long long rel = key - base;
      const unsigned slot = (rel >= 0 && rel < kLdsBins) ? atomicAdd(&hist[rel], 1u) : atomicAdd(cursor + key, 1u);
      sorted[slot] = make_float4(px[u], py[u], pz[u], wv[u]);
      slot_of[i] = slot;
    }
  }
}

// Exclusive scan of uint32 counts in three kernels: block totals, scan of the totals, apply.
constexpr int kScanItems = 16;
__global__ void __launch_bounds__(256) k_scan_blocks(const unsigned* __restrict__ in, long long n,
                                                     unsigned* __restrict__ bsum) {
  const long long base = (long long)blockIdx.x * 256 * kScanItems;
  unsigned s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const long long i = base + (long long)k * 256 + threadIdx.x;
    if (i < n) s += in[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  __shared__ unsigned ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) bsum[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// In-place exclusive scan of nb block totals by one block.
__global__ void __launch_bounds__(256) k_scan_top(unsigned* __restrict__ bsum, int nb) {
  __shared__ unsigned sh[256];
  unsigned carry = 0;
  for (int base = 0; base < nb; base += 256) {
    const int i = base + threadIdx.x;
    const unsigned v = i < nb ? bsum[i] : 0u;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      unsigned t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0u;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + sh[threadIdx.x] - v;
    carry += sh[255];
    __syncthreads();
  }
}

// out[i] = exclusive prefix of in (out has n + 1 entries; out[n] = total); cursor = copy of out[0..n).
__global__ void __launch_bounds__(256) k_scan_apply(const unsigned* __restrict__ in, long long n,
                                                    const unsigned* __restrict__ bsum, unsigned* __restrict__ out,
                                                    unsigned* __restrict__ cursor) {
  __shared__ unsigned sh[256];
  const long long base = (long long)blockIdx.x * 256 * kScanItems;
  unsigned carry = bsum[blockIdx.x];
  for (int k = 0; k < kScanItems; ++k) {
    const long long i = base + (long long)k * 256 + threadIdx.x;
    const unsigned v = i < n ? in[i] : 0u;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      unsigned t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0u;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    const unsigned ex = carry + sh[threadIdx.x] - v;
    if (i < n) { out[i] = ex; cursor[i] = ex; }
    if (i == n - 1) out[n] = ex + v;
    carry += sh[255];
    __syncthreads();
  }
}

// One block per brick: LDS accumulation of the (BS+1)^3 footprint, then a flush with
// 64-bit atomics (bricks overlap by one cell on their upper faces).  NT threads walk the brick's
// objects side by side (a brick of the survey's randoms holds about 8,700 of them).
template <int NT>
__global__ void __launch_bounds__(NT) k_brick_deposit(const float4* __restrict__ sorted,
                                                      const unsigned* __restrict__ start, CicGeo g,
                                                      unsigned long long* __restrict__ grid) {
  constexpr int T = kBrick + 1;
  __shared__ unsigned long long acc[T * T * T];
  const long long key = brick_of_block();
  const unsigned lo = start[key], hi = start[key + 1];
  if (lo == hi) return;
  const int nbs = (g.n + kBrick - 1) / kBrick;
  const long long per = (long long)nbs * nbs * nbs;
  const int b = (int)(key / per);
  const long long kk = key - (long long)b * per;
  const int bx = (int)(kk % nbs), by = (int)((kk / nbs) % nbs), bz = (int)(kk / ((long long)nbs * nbs));
  for (int i = threadIdx.x; i < T * T * T; i += NT) acc[i] = 0ull;
  __syncthreads();
  constexpr int U = kObjBatch;
  for (long long j0 = (long long)lo + threadIdx.x; j0 < hi; j0 += (long long)NT * U) {
    float4 rr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long j = j0 + (long long)u * NT;
      rr[u] = sorted[j < hi ? j : hi - 1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (j0 + (long long)u * NT >= hi) break;
      const float4 r = rr[u];
      int ii[3];
      unsigned long long tau[3];
      cic_locate(r.x, r.y, r.z, r.w, g, ii, tau);
      const unsigned long long wq = (unsigned long long)__double2ll_rn((double)r.w * 4294967296.0);
      const int lx = ii[0] - bx * kBrick, ly = ii[1] - by * kBrick, lz = ii[2] - bz * kBrick;
      unsigned long long share[8];
      cic_shares(wq, tau, share);
#pragma unroll
      for (int cnr = 0; cnr < 8; ++cnr) {
        const int dx = cnr & 1, dy = (cnr >> 1) & 1, dz = cnr >> 2;
        if (share[cnr]) atomicAdd(&acc[((lz + dz) * T + (ly + dy)) * T + (lx + dx)], share[cnr]);
      }
    }
  }
  __syncthreads();
  unsigned long long* gb = grid + (long long)b * g.n * g.n * g.n;
  for (int i = threadIdx.x; i < T * T * T; i += NT) {
    const unsigned long long v = acc[i];
    if (!v) continue;
    const int lx = i % T, ly = (i / T) % T, lz = i / (T * T);
    const long long x = (bx * kBrick + lx) & (g.n - 1), y = (by * kBrick + ly) & (g.n - 1),
                    z = (bz * kBrick + lz) & (g.n - 1);
    const long long cell = ((long long)z * g.n + y) * g.n + x;
    if (in_bounds(cell, (long long)g.n * g.n * g.n)) atomicAdd(gb + cell, v);
  }
}

// Brick-sparse integer grids.  valid[key] (one byte per 16^3 brick) marks the bricks whose cells are
// held in memory; every other brick is zero and is neither cleared nor read.  A deposit through the
// bricks touches brick B when B or one of its seven lower neighbours holds objects (a brick's
// footprint reaches one cell into its upper neighbours).  Modes, one block per brick:
//   0 (new grid):   clear the touched bricks, valid = touched
//   1 (accumulate): clear the touched bricks that are not valid yet, valid |= touched
//   2 (densify):    clear every brick that is not valid, valid = 1 (before a deposit that does not go
//                   through the bricks)
// Requires n to be a multiple of the brick size.
__global__ void __launch_bounds__(256) k_brick_prepare(const unsigned* __restrict__ count, int n, int mode,
                                                       unsigned char* __restrict__ valid,
                                                       unsigned long long* __restrict__ grid) {
  const int nbs = n / kBrick;
  const long long per = (long long)nbs * nbs * nbs;
  const long long key = blockIdx.x;
  const int b = (int)(key / per);
  const long long kk = key - (long long)b * per;
  const int bx = (int)(kk % nbs), by = (int)((kk / nbs) % nbs), bz = (int)(kk / ((long long)nbs * nbs));
  bool touched = true;
  if (mode != 2) {
    touched = false;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const int x = (bx - (d & 1) + nbs) % nbs, y = (by - ((d >> 1) & 1) + nbs) % nbs,
                z = (bz - (d >> 2) + nbs) % nbs;
      touched = touched || count[(long long)b * per + ((long long)z * nbs + y) * nbs + x] != 0u;
    }
  }
  const bool was = valid[key] != 0;
  const bool clear = mode == 0 ? touched : (mode == 1 ? (touched && !was) : !was);
  if (clear) {
    // 16-byte stores, two cells each (a brick row starts at an even cell, the grid on 16 bytes)
    unsigned long long* gb = grid + (long long)b * n * n * n;
    constexpr int H = kBrick / 2;
    for (int i = threadIdx.x; i < H * kBrick * kBrick; i += 256) {
      const long long x = bx * kBrick + 2 * (i % H), y = by * kBrick + (i / H) % kBrick,
                      z = bz * kBrick + i / (H * kBrick);
      *reinterpret_cast<uint4*>(gb + (z * n + y) * n + x) = make_uint4(0u, 0u, 0u, 0u);
    }
  }
  if (threadIdx.x == 0) valid[key] = (unsigned char)(mode == 0 ? touched : (mode == 1 ? (was || touched) : 1));
}

// Validity of the brick holding cell (x, y, z) of realisation b (null: every brick is valid).
__device__ __forceinline__ bool brick_valid(const unsigned char* __restrict__ valid, int n, int b, int x, int y,
                                            int z) {
  if (!valid) return true;
  const int nbs = n / kBrick;
  return valid[(((long long)b * nbs + z / kBrick) * nbs + y / kBrick) * nbs + x / kBrick] != 0;
}

// Dense copy of a brick-sparse grid (zeros in the bricks that are not valid).
__global__ void __launch_bounds__(256) k_grid_export(const long long* __restrict__ grid,
                                                     const unsigned char* __restrict__ valid, int n, int batch,
                                                     long long* __restrict__ out) {
  const long long n3 = (long long)n * n * n, total = n3 * batch;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < total; i += (long long)gridDim.x * 256) {
    const int b = (int)(i / n3);
    const long long c = i - b * n3;
    const int x = (int)(c % n), y = (int)((c / n) % n), z = (int)(c / ((long long)n * n));
    out[i] = brick_valid(valid, n, b, x, y, z) ? grid[i] : 0;
  }
}

// Binary survey mask with a sliding window: each wave owns one y row and 64 consecutive x
// (62 outputs plus one halo lane each side); per z it sums the three y rows, adds the two
// x neighbours through lane shuffles, and keeps a running three-plane window along z.
// Sums are exact int64; a cell is inside when the 27-cell sum exceeds thr[b].
__global__ void __launch_bounds__(256) k_mask_win(const long long* __restrict__ gr, int n,
                                                  const long long* __restrict__ thr,
                                                  unsigned char* __restrict__ mask) {
  const int b = blockIdx.y;
  const int nseg = (n + 61) / 62;
  const int seg = blockIdx.x % nseg;
  const int y = (blockIdx.x / nseg) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (y >= n) return;                                   // whole wave leaves together
  const long long n2 = (long long)n * n;
  const long long* g = gr + (long long)b * n2 * n;
  unsigned char* m = mask + (long long)b * n2 * n;
  const long long t = thr[b];
  const int xs = seg * 62 + lane - 1;                   // may be -1 or >= n: wrapped below
  const int x = xs & (n - 1);
  const long long ym = (long long)((y - 1) & (n - 1)) * n, y0 = (long long)y * n,
                  yp = (long long)((y + 1) & (n - 1)) * n;
  const bool out = lane >= 1 && lane <= 62 && xs < n;
  auto plane = [&](int z) -> long long {
    const long long* gz = g + (long long)z * n2 + x;
    const long long r = gz[ym] + gz[y0] + gz[yp];
    const long long l = __shfl(r, (lane + 63) & 63, 64);
    const long long h = __shfl(r, (lane + 1) & 63, 64);
    return l + r + h;
  };
  const long long first = plane(0);
  long long prev = plane(n - 1), cur = first;
  for (int z = 0; z < n; ++z) {
    const long long next = z + 1 < n ? plane(z + 1) : first;
    if (out) m[(long long)z * n2 + y0 + xs] = (prev + cur + next) > t ? 1 : 0;
    prev = cur;
    cur = next;
  }
}

// The same mask on a brick-sparse random grid, one block per 16^3 brick: the 18^3 neighbourhood is
// staged in LDS (bricks that are not valid read as zero and are not loaded), each thread owns one
// (x, y) column of the brick and keeps the 3 x 3 sums of the 18 planes in registers, then slides
// along z.  A brick whose 27 neighbours are all not valid has every window sum 0.  Bricks are
// taken in XCD ranges (brick_of_block): the one-cell halo reads of x-adjacent bricks and the 16-byte
// pieces of the 128-byte mask lines they write meet in one L2 instead of in HBM.  With mflag (zeroed
// before the launch), a row of the brick with any cell inside the mask sets the flag of its z tile
// (one y row, tw consecutive x, every z; tw a multiple of the brick size).
__global__ void __launch_bounds__(256) k_mask_brick(const long long* __restrict__ gr, int n,
                                                    const long long* __restrict__ thr,
                                                    const unsigned char* __restrict__ valid,
                                                    unsigned char* __restrict__ mask,
                                                    unsigned char* __restrict__ mflag = nullptr, int tw = 0) {
  constexpr int H = kBrick + 2, H3 = H * H * H, PER = (H3 + 255) / 256;
  __shared__ __align__(16) long long h[H3];
  __shared__ int nv[27];
  __shared__ int any;
  const int nbs = n / kBrick;
  const long long per = (long long)nbs * nbs * nbs;
  const long long key = brick_of_block();
  const int b = (int)(key / per);
  const long long kk = key - (long long)b * per;
  const int bx = (int)(kk % nbs), by = (int)((kk / nbs) % nbs), bz = (int)(kk / ((long long)nbs * nbs));
  const long long n2 = (long long)n * n;
  const long long* g = gr + (long long)b * n2 * n;
  unsigned char* m = mask + (long long)b * n2 * n;
  const long long t = thr[b];
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  if (threadIdx.x < 27) {
    const int dx = threadIdx.x % 3 - 1, dy = (threadIdx.x / 3) % 3 - 1, dz = threadIdx.x / 9 - 1;
    const int x = (bx + dx + nbs) % nbs, y = (by + dy + nbs) % nbs, z = (bz + dz + nbs) % nbs;
    nv[threadIdx.x] = valid[(long long)b * per + ((long long)z * nbs + y) * nbs + x] != 0;
    if (nv[threadIdx.x]) atomicOr(&any, 1);
  }
  __syncthreads();
  // thread t writes mask row (z, y) = (t / 16, t % 16) of the brick: 16 bytes along x
  const int rz = threadIdx.x / kBrick, ry = threadIdx.x % kBrick;
  uint4* row = (uint4*)(m + (long long)(bz * kBrick + rz) * n2 + (long long)(by * kBrick + ry) * n + bx * kBrick);
  unsigned char* fl = mflag ? mflag + (long long)b * n * (n / tw) + (long long)(by * kBrick + ry) * (n / tw) +
                                    bx * kBrick / tw
                            : nullptr;
  if (!any) {
    const unsigned v = 0 > t ? 0x01010101u : 0u;
    *row = make_uint4(v, v, v, v);
    if (fl && v) *fl = 1;
    return;
  }
  long long vals[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = threadIdx.x + 256 * k;
    vals[k] = 0;
    if (i < H3) {
      const int lx = i % H, ly = (i / H) % H, lz = i / (H * H);
      // neighbour brick of this halo cell: -1, 0 or +1 per axis
      const int ox = lx == 0 ? 0 : (lx == H - 1 ? 2 : 1), oy = ly == 0 ? 0 : (ly == H - 1 ? 2 : 1),
                oz = lz == 0 ? 0 : (lz == H - 1 ? 2 : 1);
      if (nv[(oz * 3 + oy) * 3 + ox]) {
        const long long x = (bx * kBrick + lx - 1 + n) & (n - 1), y = (by * kBrick + ly - 1 + n) & (n - 1),
                        z = (bz * kBrick + lz - 1 + n) & (n - 1);
        vals[k] = g[z * n2 + y * n + x];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (threadIdx.x + 256 * k < H3) h[threadIdx.x + 256 * k] = vals[k];
  __syncthreads();
  // thread (tx, ty) owns one (x, y) column: 3 x 3 sums of the 18 planes, then the z window
  const int tx = threadIdx.x % kBrick, ty = threadIdx.x / kBrick;
  long long sxy[H];
#pragma unroll
  for (int lz = 0; lz < H; ++lz) {
    long long a = 0;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) a += h[(lz * H + ty + dy) * H + tx + dx];
    sxy[lz] = a;
  }
  __syncthreads();                                       // h is reused for the mask bytes below
  unsigned char* mb = (unsigned char*)h;                 // [z][y][x], 16^3 bytes
#pragma unroll
  for (int z = 0; z < kBrick; ++z)
    mb[(z * kBrick + ty) * kBrick + tx] = (sxy[z] + sxy[z + 1] + sxy[z + 2]) > t ? 1 : 0;
  __syncthreads();
  const uint4 w4 = ((const uint4*)mb)[threadIdx.x];
  *row = w4;
  if (fl && (w4.x | w4.y | w4.z | w4.w)) *fl = 1;      // every writer stores the same value
}

// Per-realisation scalars from the exact totals {W_g, W_r, n_occ}:
//   alpha = W_g / W_r, 1/rho_bar = N^3 / (W_g 2^-32), mask threshold floor(tau 27 W_r / n_occ);
// status[b] bit 0: galaxy total is zero, bit 1: random total is zero.
// One block per realisation: sums the per-tile integer partials (exact, any order), then derives
// the scalars; tot[b] keeps the totals.
__global__ void __launch_bounds__(256) k_scalars(const unsigned long long* __restrict__ tpart, int nblk, long long n3,
                                                 double tau, int randoms, unsigned long long* __restrict__ tot,
                                                 DeltaScal* __restrict__ sc, long long* __restrict__ thr,
                                                 int* __restrict__ status) {
  const int b = blockIdx.x;
  unsigned long long acc[3] = {0ull, 0ull, 0ull};
  for (int i = threadIdx.x; i < nblk; i += 256) {
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[k] += tpart[3 * ((long long)b * nblk + i) + k];
  }
  __shared__ unsigned long long red[3][4];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) red[k][threadIdx.x >> 6] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const long long wg = (long long)(red[0][0] + red[0][1] + red[0][2] + red[0][3]);
    const long long wr = (long long)(red[1][0] + red[1][1] + red[1][2] + red[1][3]);
    const long long occ = (long long)(red[2][0] + red[2][1] + red[2][2] + red[2][3]);
    tot[3 * b] = (unsigned long long)wg;
    tot[3 * b + 1] = (unsigned long long)wr;
    tot[3 * b + 2] = (unsigned long long)occ;
    int st = 0;
    DeltaScal d;
    d.inv_rhobar = wg > 0 ? (float)((double)n3 / ((double)wg * 2.3283064365386963e-10)) : 0.f;
    d.alpha = 0.f;
    long long th = 0;
    if (wg <= 0) st |= 1;
    if (randoms) {
      if (wr <= 0 || occ <= 0) st |= 2;
      else {
        d.alpha = (float)((double)wg / (double)wr);
        th = (long long)floor(tau * 27.0 * (double)wr / (double)occ);
      }
    }
    sc[b] = d;
    thr[b] = th;
    status[b] = st;
  }
}

// Mask-tile flags: mflag[b][tile] = 1 when any cell of z tile `tile` (one y row, tw consecutive x,
// every z) lies inside the survey mask.  One block per tile; 16-byte words when the tile row is a
// multiple of 16 bytes, bytes otherwise.
__global__ void __launch_bounds__(256) k_mask_tiles(const unsigned char* __restrict__ mask, int n, int tw,
                                                    unsigned char* __restrict__ mflag) {
  const long long n3 = (long long)n * n * n;
  const int b = blockIdx.y, tpr = n / tw;
  const int y = blockIdx.x / tpr, x0 = (blockIdx.x % tpr) * tw;
  const unsigned char* m = mask + b * n3;
  int mine = 0;
  if (tw % 16 == 0) {
    const int row16 = tw / 16;
    for (int i = threadIdx.x; i < n * row16; i += 256) {
      const long long e = ((long long)(i / row16) * n + y) * n + x0 + 16 * (i % row16);
      if (in_bounds(e + 15, n3)) {
        const uint4 w4 = *(const uint4*)(m + e);
        mine |= (w4.x | w4.y | w4.z | w4.w) != 0u;
      }
    }
  } else {
    for (int i = threadIdx.x; i < n * tw; i += 256) {
      const long long e = ((long long)(i / tw) * n + y) * n + x0 + i % tw;
      if (in_bounds(e, n3)) mine |= m[e] != 0;
    }
  }
  mine = __syncthreads_or(mine);
  if (threadIdx.x == 0) mflag[(long long)b * gridDim.x + blockIdx.x] = mine ? 1 : 0;
}

// ---------------------------------------------------------------------------
// z passes (real <-> half spectrum along z, two real columns packed per complex
// column).  Tile: one y row and 2*WP consecutive x; fragment threads are column-fast
// over the WP packed columns.
// ---------------------------------------------------------------------------
template <int N, int WP>
__device__ __forceinline__ void z_tile_at(int tile, int& y, int& x0) {
  constexpr int TPR = N / (2 * WP);
  y = tile / TPR;
  x0 = (tile % TPR) * 2 * WP;
}

template <int N, int WP>
__device__ __forceinline__ void z_tile_coords(int& y, int& x0) { z_tile_at<N, WP>(blockIdx.x, y, x0); }

// Packed full-length column element k of the half spectra A (column x0+c) and B
// (column x0+c+WP): Z(k) = A(k) + i B(k), extended Hermitian-wise for k > N/2; the
// imaginary parts at k = 0 and N/2 are dropped as for a real inverse transform.
template <int N, int WP>
__device__ __forceinline__ void z_pack_frag(float2* v, const float2* __restrict__ a, int y, int x0, int c, int j) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int k = j + r * (N / 8);
    const int m = k <= N / 2 ? k : N - k;
    const long long base = ((long long)m * N + y) * N + x0 + c;
    constexpr long long CN = (long long)(N / 2 + 1) * N * N;
    const float2 A = in_bounds(base, CN) ? a[base] : float2{}, B = in_bounds(base + WP, CN) ? a[base + WP] : float2{};
    if (k == 0 || k == N / 2) v[r] = make_float2(A.x, B.x);
    else if (k < N / 2) v[r] = make_float2(A.x - B.y, A.y + B.x);
    else v[r] = make_float2(A.x + B.y, B.x - A.y);
  }
}

// LDS-direct staging of a z tile: rows kz = 0..N/2 of columns x0 .. x0 + 2 WP - 1 at plane row y
// land in `stage` as [kz][2 WP] float2 without passing through registers, so the loads of the next
// array run while the current one is transformed.  Each lane moves 16 bytes; one wave instruction
// fills one 1 KB chunk (its LDS base is wave-uniform).  Completion: s_waitcnt vmcnt(0), then a barrier.
template <int N, int WP>
struct ZStage {
  static constexpr int ROWB = 2 * WP * 8;             // bytes per kz row
  static constexpr int LPR = ROWB / 16;               // lanes per row
  static constexpr int RPC = 64 / LPR;                // rows per 1 KB chunk
  static constexpr int ROWS = N / 2 + 1;
  static constexpr int NCH = (ROWS + RPC - 1) / RPC;
  static constexpr int SIZE = NCH * 128;              // float2 elements
};

template <int N, int WP, int NT>
__device__ __forceinline__ void z_stage_issue(float2* stage, const float2* __restrict__ a, int y, int x0) {
  using S = ZStage<N, WP>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = wave; q < S::NCH; q += NT / 64) {
    const int m = q * S::RPC + lane / S::LPR;
    const long long e = ((long long)m * N + y) * N + x0 + 2 * (lane % S::LPR);
    if (m < S::ROWS && in_bounds(e + 1, (long long)(N / 2 + 1) * N * N)) {
      const float2* g = a + e;
      __builtin_amdgcn_global_load_lds((const void*)g, (__attribute__((address_space(3))) void*)(stage + q * 128),
                                       16, 0, kStageCachePolicy);
    }
  }
}

__device__ __forceinline__ void z_stage_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// z_pack_frag from a staged tile.
template <int N, int WP>
__device__ __forceinline__ void z_pack_stage(float2* v, const float2* stage, int c, int j) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int k = j + r * (N / 8);
    const int m = k <= N / 2 ? k : N - k;
    const float2 A = stage[m * 2 * WP + c], B = stage[m * 2 * WP + c + WP];
    if (k == 0 || k == N / 2) v[r] = make_float2(A.x, B.x);
    else if (k < N / 2) v[r] = make_float2(A.x - B.y, A.y + B.x);
    else v[r] = make_float2(A.x + B.y, B.x - A.y);
  }
}

// Split a transformed packed tile (natural order in LDS) into the half spectra of its
// two real columns and store them.  MULK: multiply by i k'_z.
template <int N, int WP, int NT, bool MULK>
__device__ __forceinline__ void z_unpack_store(const float2* buf, float2* __restrict__ out, int y, int x0, float kf) {
  using L = Lay<N, WP, false>;
  for (int e = threadIdx.x; e < (N / 2 + 1) * WP; e += NT) {
    const int p = e % WP, kz = e / WP;
    const float2 Z = buf[L::at(kz, p)];
    const float2 M = buf[L::at((N - kz) & (N - 1), p)];
    float2 A = make_float2(0.5f * (Z.x + M.x), 0.5f * (Z.y - M.y));
    float2 B = make_float2(0.5f * (Z.y + M.y), 0.5f * (M.x - Z.x));
    if (MULK) {
      const float k = kf * deriv_mode<N>(kz);
      A = mul_i(A) * k;
      B = mul_i(B) * k;
    }
    const long long base = ((long long)kz * N + y) * N + x0 + p;
    constexpr long long CN = (long long)(N / 2 + 1) * N * N;
    if (in_bounds(base, CN)) st_stream(out + base, A);
    if (in_bounds(base + WP, CN)) st_stream(out + base + WP, B);
  }
}

// Scaled line-of-sight vector of a node: r = (origin + H i - observer) / R0.
__device__ __forceinline__ float los_comp(const Geo& g, int a, int i) { return fmaf(g.hs, (float)i, g.ds[a]); }
// |r|^2 with a fixed rounding order, so that every z kernel (and every tiling of one) forms the same
// value whatever the compiler hoists or contracts
__device__ __forceinline__ float los_r2(float rx, float ry, float rz) { return fmaf(rz, rz, fmaf(ry, ry, rx * rx)); }

template <int N> constexpr int ntz() { return frag_threads<N, wz<N>()>(); }
template <int N> constexpr int nty() { return frag_threads<N, wy<N>()>(); }
template <int N> constexpr int ntx() { return frag_threads<N, wx<N>()>(); }

// Forward z transform of int64 grids (units 2^-32) into half spectra.
// Also writes the exact totals {sum g0, sum g1, #(g1 != 0)} of the tile to tpart[b][block].
template <int N, int NA>
// With tile flags (zflag != null, [NA][batch][z tiles]): a tile whose bricks are all not valid gets
// flag 0 and its zero half spectra are not written (the forward y pass reads such rows as zeros);
// every other tile gets flag 1.
__global__ void __launch_bounds__(ntz<N>(), 8) k_z_fwd_grid(const long long* __restrict__ g0,
                                                         const long long* __restrict__ g1, float2* __restrict__ o0,
                                                         float2* __restrict__ o1, unsigned long long* __restrict__ tpart,
                                                         const float2* __restrict__ twg,
                                                         const unsigned char* __restrict__ v0 = nullptr,
                                                         const unsigned char* __restrict__ v1 = nullptr,
                                                         unsigned char* __restrict__ zflag = nullptr) {
  constexpr int NT = ntz<N>(), WP = wz<N>();
  using L = Lay<N, WP, false>;
  __shared__ float2 buf[L::SIZE];
  __shared__ float2 tw[N];
  stage_twiddles<N, NT>(tw, twg);
  int y, x0, c, j;
  z_tile_coords<N, WP>(y, x0);
  frag_coords<N, WP, false>(c, j);
  const bool act = threadIdx.x < L::NTF;
  const long long n3 = (long long)N * N * N, cn = (long long)(N / 2 + 1) * N * N;
  const int b = blockIdx.y;
  const float unit = 2.3283064365386963e-10f;   // 2^-32
  unsigned long long sums[3] = {0ull, 0ull, 0ull};
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    const long long* gsrc = (a == 0 ? g0 : g1) + b * n3;
    // brick-validity of the two columns' bricks along z (brick-sparse grids; null: all valid)
    const unsigned char* vg = a == 0 ? v0 : v1;
    constexpr int NBS = N / kBrick;
    const unsigned char* vb = vg ? vg + (long long)b * NBS * NBS * NBS + (y / kBrick) * NBS : nullptr;
    if (vb) {
      // a tile whose bricks are all not valid holds zeros: its half spectra are zero, no transform
      constexpr int XB = (2 * WP + kBrick - 1) / kBrick;   // bricks across the tile's 2 WP columns
      int mine = 0;
      for (int i = threadIdx.x; i < NBS * XB; i += NT) mine |= vb[(i / XB) * NBS * NBS + x0 / kBrick + i % XB];
      if (!__syncthreads_or(mine)) {
        if (zflag) {
          if (threadIdx.x == 0) zflag[((long long)a * gridDim.y + b) * gridDim.x + blockIdx.x] = 0;
        } else {
          float2* out = (a == 0 ? o0 : o1) + b * cn;
          for (int e = threadIdx.x; e < (N / 2 + 1) * 2 * WP; e += NT)
            out[((long long)(e / (2 * WP)) * N + y) * N + x0 + e % (2 * WP)] = make_float2(0.f, 0.f);
        }
        continue;
      }
    }
    if (zflag && threadIdx.x == 0) zflag[((long long)a * gridDim.y + b) * gridDim.x + blockIdx.x] = 1;
    float2 v[8];
    if (act) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int z = j + r * (N / 8);
        const long long base = ((long long)z * N + y) * N + x0 + c;
        const unsigned char* vz = vb ? vb + (z / kBrick) * NBS * NBS : nullptr;
        const bool ok0 = !vz || vz[(x0 + c) / kBrick], ok1 = !vz || vz[(x0 + c + WP) / kBrick];
        const long long q0 = ok0 ? gsrc[base] : 0, q1 = ok1 ? gsrc[base + WP] : 0;
        sums[a] += (unsigned long long)q0 + (unsigned long long)q1;
        if (a == 1) sums[2] += (q0 != 0) + (q1 != 0);
        v[r] = make_float2((float)q0 * unit, (float)q1 * unit);
      }
    }
    fft_rl<N, WP, false, false>(v, buf, tw);
    z_unpack_store<N, WP, NT, false>(buf, (a == 0 ? o0 : o1) + b * cn, y, x0, 0.f);
  }
  __shared__ unsigned long long red[3][NT / 64];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sums[k] += __shfl_xor(sums[k], o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) red[k][threadIdx.x >> 6] = sums[k];
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    unsigned long long t = 0;
    for (int w = 0; w < NT / 64; ++w) t += red[threadIdx.x][w];
    tpart[3 * ((long long)b * gridDim.x + blockIdx.x) + threadIdx.x] = t;
  }
}

// Forward z transform of one real field.
template <int N>
__global__ void __launch_bounds__(ntz<N>()) k_z_fwd_real(const float* __restrict__ f, float2* __restrict__ o,
                                                         const float2* __restrict__ twg) {
  constexpr int NT = ntz<N>(), WP = wz<N>();
  using L = Lay<N, WP, false>;
  __shared__ float2 buf[L::SIZE];
  __shared__ float2 tw[N];
  stage_twiddles<N, NT>(tw, twg);
  int y, x0, c, j;
  z_tile_coords<N, WP>(y, x0);
  frag_coords<N, WP, false>(c, j);
  const long long n3 = (long long)N * N * N, cn = (long long)(N / 2 + 1) * N * N;
  const int b = blockIdx.y;
  f += b * n3;
  float2 v[8];
  if (threadIdx.x < L::NTF) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const long long base = ((long long)(j + r * (N / 8)) * N + y) * N + x0 + c;
      v[r] = make_float2(f[base], f[base + WP]);
    }
  }
  fft_rl<N, WP, false, false>(v, buf, tw);
  z_unpack_store<N, WP, NT, false>(buf, o + b * cn, y, x0, 0.f);
}

// Inverse z transform of the smoothed galaxy (and random) densities, overdensity in
// configuration space, forward z transform of the overdensity (written over a0).
//   with randoms:  delta = m (G - alpha R) / (alpha R), 0 outside the mask or where R <= 0
//   mean density:  delta = G / rho_bar - 1
template <int N, int NA>
__global__ void __launch_bounds__(ntz<N>()) k_z_delta(float2* __restrict__ a0, const float2* __restrict__ a1,
                                                      const unsigned char* __restrict__ mask,
                                                      const DeltaScal* __restrict__ sc, float* __restrict__ delta_out,
                                                      float log_floor, double* __restrict__ partials,
                                                      const float2* __restrict__ twg,
                                                      const unsigned char* __restrict__ mflag = nullptr) {
  constexpr int NT = ntz<N>(), WP = wz<N>();
  using L = Lay<N, WP, false>;
  __shared__ float2 buf[L::SIZE];
  __shared__ float2 tw[N];
  stage_twiddles<N, NT>(tw, twg);
  int y, x0, c, j;
  z_tile_coords<N, WP>(y, x0);
  frag_coords<N, WP, false>(c, j);
  const bool act = threadIdx.x < L::NTF;
  const long long n3 = (long long)N * N * N, cn = (long long)(N / 2 + 1) * N * N;
  const int b = blockIdx.y;
  a0 += b * cn;
  const DeltaScal s = sc[b];
  double lsum = 0.0;
  float2 gv[8], v[8];
  if constexpr (NA == 2) {
    // a tile outside the survey mask (mask-tile flag 0) has delta_s = 0 in every cell (also after the
    // lognormal transform, ln 1 = 0): its spectrum is zero and no transform is needed; it is not
    // written either (the forward y pass reads such rows as zeros), nor were its inputs (the inverse
    // y pass skipped them).  Without flags every tile is transformed.
    if (mflag && !mflag[(long long)b * gridDim.x + blockIdx.x]) {
      if (delta_out)
        for (int e = threadIdx.x; e < N * 2 * WP; e += NT)
          delta_out[b * n3 + ((long long)(e / (2 * WP)) * N + y) * N + x0 + e % (2 * WP)] = 0.f;
      if (log_floor > 0.f && threadIdx.x == 0) {
        partials[2 * ((long long)b * gridDim.x + blockIdx.x)] = 0.0;
        partials[2 * ((long long)b * gridDim.x + blockIdx.x) + 1] = 0.0;
      }
      return;
    }
    // the second array is staged in LDS by direct loads while the first is transformed
    __shared__ float2 stage[ZStage<N, WP>::SIZE];
    z_stage_issue<N, WP, NT>(stage, a0, y, x0);
    z_stage_wait();
    __syncthreads();
    if (act) z_pack_stage<N, WP>(gv, stage, c, j);
    __syncthreads();
    z_stage_issue<N, WP, NT>(stage, a1 + b * cn, y, x0);
    fft_rr<N, WP, true, false>(gv, buf, tw);
    z_stage_wait();
    __syncthreads();
    if (act) z_pack_stage<N, WP>(v, stage, c, j);
    fft_rr<N, WP, true, false>(v, buf, tw);
  } else {
    if (act) z_pack_frag<N, WP>(gv, a0, y, x0, c, j);
    fft_rr<N, WP, true, false>(gv, buf, tw);
  }
  if (act) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const long long cell = ((long long)(j + r * (N / 8)) * N + y) * N + x0 + c;
      float d0, d1;
      if constexpr (NA == 2) {
        const unsigned char* m = mask + b * n3;
        const float ar0 = s.alpha * v[r].x, ar1 = s.alpha * v[r].y;
        d0 = (m[cell] && ar0 > 0.f) ? (gv[r].x - ar0) / ar0 : 0.f;
        d1 = (m[cell + WP] && ar1 > 0.f) ? (gv[r].y - ar1) / ar1 : 0.f;
      } else {
        d0 = gv[r].x * s.inv_rhobar - 1.f;
        d1 = gv[r].y * s.inv_rhobar - 1.f;
      }
      if (log_floor > 0.f) {                           // lognormal option: ln(max(1 + delta, floor))
        d0 = logf(fmaxf(1.f + d0, log_floor));
        d1 = logf(fmaxf(1.f + d1, log_floor));
        lsum += (double)d0 + (double)d1;
      }
      v[r] = make_float2(d0, d1);
      if (delta_out) {
        delta_out[b * n3 + cell] = d0;
        delta_out[b * n3 + cell + WP] = d1;
      }
    }
  }
  if (log_floor > 0.f) {
    double t1, t2;
    block_sum2<NT>(lsum, 0.0, &t1, &t2);
    if (threadIdx.x == 0) {
      partials[2 * ((long long)b * gridDim.x + blockIdx.x)] = t1;
      partials[2 * ((long long)b * gridDim.x + blockIdx.x) + 1] = 0.0;
    }
  }
  fft_rl<N, WP, false, false>(v, buf, tw);
  z_unpack_store<N, WP, NT, false>(buf, a0, y, x0, 0.f);
}

// Lognormal option: add C = -<ln(max(1 + delta, floor))> (sums[2 b] = sum over the n^3 cells of
// realisation b) to the kept configuration-space field.  Only the k = 0 mode of the spectrum would
// change, and that mode does not enter Psi, so the spectrum is left alone.
__global__ void __launch_bounds__(256) k_log_shift(float* __restrict__ delta, long long n3, int batch,
                                                   const double* __restrict__ sums) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n3 * batch; i += (long long)gridDim.x * 256) {
    const long long b = i / n3;
    delta[i] += (float)(-sums[2 * b] / (double)n3);
  }
}

// One iteration's configuration-space step (step A tail + step B head), on the combined fan-out
// state a0 = transverse part r_x Psi_x + r_y Psi_y, a2 = Psi_z (z spectra; r the scaled line of sight):
//   inverse z of both -> s = Psi . r = Z^-1[a0] + r_z Z^-1[a2];  u_p = s / |r|
//   q = u_0 / |r| (V_j = u_0 r_hat_j = q r_j) -> a0 = Z[q], a1 = i k'_z Z[r_z q]
// Start modes (first pass only):
//   ZI_FFTA:    u_0 = start_scale * u_p, Delta = u_0 - u_p stored in corr
//   ZI_LEARNED: u_0 = u_p + corr (corr taken as 0 at the observer), with u_p read from up_in, the
//               start's own inverse z step (the same arithmetic), so no inverse transform is redone
// and both accumulate S1 = sum Delta u_p, S2 = sum Delta^2 into partials.  On the pass after such
// a start, ZI_CROSS iterates as ZI_PLAIN and accumulates S3 = sum Delta u_1 (second entry 0), the
// cross term of ||Psi_1 - Psi_0||^2.
template <int N, int MODE, int SPLIT = 0>
__global__ void __launch_bounds__(ntz<N>()) k_z_iter(float2* __restrict__ a0, float2* __restrict__ a1,
                                                     const float2* __restrict__ a2, Geo g, float* __restrict__ corr,
                                                     double* __restrict__ partials, const int* __restrict__ active,
                                                     const float2* __restrict__ twg,
                                                     const float* __restrict__ up_in = nullptr) {
  constexpr int NT = ntz<N>(), WP = wz<N>(), TPB = ztpb<N, MODE, SPLIT>();
  using L = Lay<N, WP, false>;
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  __shared__ float2 buf[L::SIZE];
  __shared__ float2 tw[N];
  __shared__ float2 stage[ZStage<N, WP>::SIZE];
  stage_twiddles<N, NT>(tw, twg);
  const bool act = threadIdx.x < L::NTF;
  const long long n3 = (long long)N * N * N, cn = (long long)(N / 2 + 1) * N * N;
  a0 += b * cn; a1 += b * cn; a2 += b * cn;
  float acc1 = 0.f, acc2 = 0.f;          // 16 terms per thread and tile; block and grid sums in FP64
  // TPB tiles per block, strided by the grid; the next tile's transverse part is staged in LDS by
  // direct loads while the current tile is finished, and the z component while the transverse
  // part is transformed
  int tile = blockIdx.x, y, x0;
  z_tile_at<N, WP>(tile, y, x0);
  // With RECON_Z_DEFER the second output of a tile (still in the exchange tile after its transform)
  // is stored only after the next tile's first array has been packed, so that the stores drain while
  // the next inverse transform runs instead of delaying the wait for the next tile's staged input;
  // py < 0: nothing deferred
  constexpr bool DEFER = RECON_Z_DEFER && MODE != ZI_LEARNED;
  int py = -1, px0 = 0;
  if (MODE != ZI_LEARNED && tile < ztiles<N>()) z_stage_issue<N, WP, NT>(stage, a0, y, x0);
#pragma unroll 1
  for (int t = 0; t < TPB && tile < ztiles<N>(); ++t) {     // block-uniform bound
    int c, j;
    frag_coords<N, WP, false>(c, j);
    const float ry = los_comp(g, 1, y);
    const float rx0 = los_comp(g, 0, x0 + c), rx1 = los_comp(g, 0, x0 + c + WP);
    float2 s[8], v[8];
    const int next = tile + gridDim.x;
    int ny = y, nx0 = x0;
    if constexpr (MODE != ZI_LEARNED) {
      z_stage_wait();
      __syncthreads();
      if (act) z_pack_stage<N, WP>(s, stage, c, j);
      __syncthreads();                                // every thread has read the staged tile
      if (DEFER && py >= 0) z_unpack_store<N, WP, NT, true>(buf, a1, py, px0, g.kf);
      z_stage_issue<N, WP, NT>(stage, a2, y, x0);
      fft_rr<N, WP, true, false, SPLIT>(s, buf, tw);        // (its first barrier ends the reads of buf above)
      z_stage_wait();
      __syncthreads();
      if (act) z_pack_stage<N, WP>(v, stage, c, j);
      if (t + 1 < TPB && next < ztiles<N>()) {
        __syncthreads();
        z_tile_at<N, WP>(next, ny, nx0);
        z_stage_issue<N, WP, NT>(stage, a0, ny, nx0);
      }
      fft_rr<N, WP, true, false, SPLIT>(v, buf, tw);
    }
    // s = Psi . r (two columns packed as .x / .y) -> q = u_0 / |r|, so that V_j = q r_j
    if (act) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int z = j + r * (N / 8);
        const float rz = los_comp(g, 2, z);
        if (MODE != ZI_LEARNED) s[r] = make_float2(fmaf(rz, v[r].x, s[r].x), fmaf(rz, v[r].y, s[r].y));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const float rx = h ? rx1 : rx0;
          const float r2 = los_r2(rx, ry, rz);
          const float ir = r2 > 0.f ? rsqrtf(r2) : 0.f;
          const long long cell = b * n3 + ((long long)z * N + y) * N + x0 + c + h * WP;
          // u_p = Psi . r_hat
          const float up = MODE == ZI_LEARNED ? up_in[cell] : (h ? s[r].y : s[r].x) * ir;
          float u0 = up;
          if (MODE != ZI_PLAIN) {
            float dlt;
            if (MODE == ZI_FFTA) {
              u0 = g.start_scale * up;
              dlt = u0 - up;
              corr[cell] = dlt;
            } else if (MODE == ZI_CROSS) {
              dlt = r2 > 0.f ? corr[cell] : 0.f;
            } else {
              dlt = r2 > 0.f ? corr[cell] : 0.f;
              u0 = up + dlt;
            }
            acc1 = fmaf(dlt, up, acc1);
            if (MODE != ZI_CROSS) acc2 = fmaf(dlt, dlt, acc2);
          }
          const float q = u0 * ir;
          if (h) s[r].y = q; else s[r].x = q;
        }
        v[r] = s[r] * rz;
      }
    }
    // Z[q] -> a0 and i k'_z Z[r_z q] -> a1; Z[V_x] = r_x Z[q] and Z[V_y] = r_y Z[q] are formed in
    // the y pass
    fft_rl<N, WP, false, false, SPLIT>(s, buf, tw);
    z_unpack_store<N, WP, NT, false>(buf, a0, y, x0, g.kf);
    fft_rl<N, WP, false, false, SPLIT>(v, buf, tw);
    if (DEFER) {
      py = y;
      px0 = x0;
    } else {
      z_unpack_store<N, WP, NT, true>(buf, a1, y, x0, g.kf);
    }
    tile = next; y = ny; x0 = nx0;
  }
  if (DEFER && py >= 0) z_unpack_store<N, WP, NT, true>(buf, a1, py, px0, g.kf);
  if (MODE != ZI_PLAIN) {
    double t1, t2;
    block_sum2<NT>((double)acc1, (double)acc2, &t1, &t2);
    if (threadIdx.x == 0) {
      const long long nb = gridDim.x;
      partials[2 * (b * nb + blockIdx.x) + 0] = t1;
      partials[2 * (b * nb + blockIdx.x) + 1] = t2;
    }
  }
}

// The plain z iteration of k_z_iter with wave-local transforms (N = 512): the wave of packed column
// c transforms that column in its own LDS region, so the only block barriers of a tile are those
// of the staging and of the stores (6 per tile instead of about 22).  The staged tile is skewed: row
// m's 16-byte piece p sits in slot (p - m) mod 16 of the row, so that a wave reading one column down
// 64 consecutive rows spreads over every bank; the per-wave regions are 577 float2 apart, so that the
// stores, which read one row of 16 columns at a time, do too.
template <int N, int WP>
__device__ __forceinline__ void z_stage_issue_skew(float2* stage, const float2* __restrict__ a, int y, int x0) {
  using S = ZStage<N, WP>;
  static_assert(S::LPR == 16, "skewed staging takes rows of 16 pieces");
  constexpr int NT = 1024;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = wave; q < S::NCH; q += NT / 64) {
    const int m = q * S::RPC + lane / S::LPR;
    const long long e = ((long long)m * N + y) * N + x0 + 2 * (((lane % S::LPR) + m) & 15);
    if (m < S::ROWS && in_bounds(e + 1, (long long)(N / 2 + 1) * N * N)) {
      __builtin_amdgcn_global_load_lds((const void*)(a + e),
                                       (__attribute__((address_space(3))) void*)(stage + q * 128), 16, 0,
                                       kStageCachePolicy);
    }
  }
}

template <int N, int WP>
__device__ __forceinline__ float2 z_stage_at_skew(const float2* stage, int m, int col) {
  return stage[m * 2 * WP + 2 * (((col >> 1) - m) & 15) + (col & 1)];
}

// z_pack_stage for the wave layout: column c, rows j + 64 r
template <int N, int WP>
__device__ __forceinline__ void z_pack_stage_w(float2* v, const float2* stage, int c, int j) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int k = j + r * (N / 8);
    const int m = k <= N / 2 ? k : N - k;
    const float2 A = z_stage_at_skew<N, WP>(stage, m, c), B = z_stage_at_skew<N, WP>(stage, m, c + WP);
    if (k == 0 || k == N / 2) v[r] = make_float2(A.x, B.x);
    else if (k < N / 2) v[r] = make_float2(A.x - B.y, A.y + B.x);
    else v[r] = make_float2(A.x + B.y, B.x - A.y);
  }
}

constexpr int kWaveRegion = 512 + 512 / 8 + 1;   // float2 per wave region

// z_unpack_store from the per-wave regions (column p in region p, natural order)
template <int N, int WP, int NT, bool MULK>
__device__ __forceinline__ void z_unpack_store_w(const float2* wreg, float2* __restrict__ out, int y, int x0,
                                                 float kf) {
  for (int e = threadIdx.x; e < (N / 2 + 1) * WP; e += NT) {
    const int p = e % WP, kz = e / WP;
    const float2 Z = wreg[p * kWaveRegion + wat(kz)];
    const float2 M = wreg[p * kWaveRegion + wat((N - kz) & (N - 1))];
    float2 A = make_float2(0.5f * (Z.x + M.x), 0.5f * (Z.y - M.y));
    float2 B = make_float2(0.5f * (Z.y + M.y), 0.5f * (M.x - Z.x));
    if (MULK) {
      const float k = kf * deriv_mode<N>(kz);
      A = mul_i(A) * k;
      B = mul_i(B) * k;
    }
    const long long base = ((long long)kz * N + y) * N + x0 + p;
    constexpr long long CN = (long long)(N / 2 + 1) * N * N;
    if (in_bounds(base, CN)) st_stream(out + base, A);
    if (in_bounds(base + WP, CN)) st_stream(out + base + WP, B);
  }
}

template <int N>
__global__ void __launch_bounds__(1024) k_z_iter_w(float2* __restrict__ a0, float2* __restrict__ a1,
                                                   const float2* __restrict__ a2, Geo g,
                                                   const int* __restrict__ active, const float2* __restrict__ twg) {
  static_assert(N == 512, "wave-local z iteration: one radix-8 fragment per lane of a 64-lane wave");
  constexpr int WP = wz<N>(), NT = 1024, TPB = ztpb<N, ZI_PLAIN>();
  static_assert(WP == 16 && (N / 8) * WP == NT, "one wave per packed column");
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  __shared__ float2 wreg[WP * kWaveRegion];
  __shared__ float2 tw[N];
  __shared__ float2 stage[ZStage<N, WP>::SIZE];
  stage_twiddles<N, NT>(tw, twg);
  const long long cn = (long long)(N / 2 + 1) * N * N;
  a0 += b * cn; a1 += b * cn; a2 += b * cn;
  int tile = blockIdx.x, y, x0;
  z_tile_at<N, WP>(tile, y, x0);
  if (tile < ztiles<N>()) z_stage_issue_skew<N, WP>(stage, a0, y, x0);
  z_stage_wait();
  __syncthreads();                                     // first tile staged
  // Waits: the staging waits (vmcnt(0)) also wait for every store a wave has issued.  The next tile's
  // first array is therefore waited for after the inverse transform of v, not at the top of the loop:
  // the stores of Z[q] have drained under that transform, and the stores of Z[r_z q], issued after
  // the wait, drain under the next tile's packing and first transform.
#pragma unroll 1
  for (int t = 0; t < TPB && tile < ztiles<N>(); ++t) {   // block-uniform bound
    // the lane's row and column are taken afresh in every tile: the addresses and line-of-sight
    // components derived from them are recomputed (a few integer and FMA operations) instead of
    // being held in registers across the loop, which would spill
    int j = threadIdx.x & 63, c = threadIdx.x >> 6;
    asm volatile("" : "+v"(j), "+v"(c));
    float2* reg = wreg + c * kWaveRegion;
    const float ry = los_comp(g, 1, y);
    const float rx0 = los_comp(g, 0, x0 + c), rx1 = los_comp(g, 0, x0 + c + WP);
    const int next = tile + gridDim.x;
    int ny = y, nx0 = x0;
    float2 s[8], v[8];
    z_pack_stage_w<N, WP>(s, stage, c, j);
    __syncthreads();                                   // every wave has read the staged tile
    z_stage_issue_skew<N, WP>(stage, a2, y, x0);
    wfft_rr<true>(s, reg, tw, j);
    z_stage_wait();
    __syncthreads();
    z_pack_stage_w<N, WP>(v, stage, c, j);
    __syncthreads();
    if (t + 1 < TPB && next < ztiles<N>()) {
      z_tile_at<N, WP>(next, ny, nx0);
      z_stage_issue_skew<N, WP>(stage, a0, ny, nx0);
    }
    wfft_rr<true>(v, reg, tw, j);
    // s = Psi . r (two columns packed as .x / .y) -> q = u / |r|, so that V_j = q r_j
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const float rz = los_comp(g, 2, j + r * (N / 8));
      s[r] = make_float2(fmaf(rz, v[r].x, s[r].x), fmaf(rz, v[r].y, s[r].y));
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float r2 = los_r2(h ? rx1 : rx0, ry, rz);
        const float ir = r2 > 0.f ? rsqrtf(r2) : 0.f;
        const float q = ((h ? s[r].y : s[r].x) * ir) * ir;
        if (h) s[r].y = q; else s[r].x = q;
      }
      v[r] = s[r] * rz;
    }
    wfft_rl<false>(s, reg, tw, j);
    __syncthreads();                                   // every column of Z[q] is in its region
    z_unpack_store_w<N, WP, NT, false>(wreg, a0, y, x0, g.kf);
    __syncthreads();                                   // the regions are free
    wfft_rl<false>(v, reg, tw, j);
    z_stage_wait();
    __syncthreads();                                   // Z[r_z q] in the regions; the next tile staged
    z_unpack_store_w<N, WP, NT, true>(wreg, a1, y, x0, g.kf);
    // (the barrier after the next tile's packing orders these reads of the regions before its transforms)
    tile = next; y = ny; x0 = nx0;
  }
}

// Inverse z of the displacement spectra.  Full state (COMB = false, a0..a2 = Psi_x, Psi_y, Psi_z):
// writes Psi (planar [b][3][N^3], when psi != null), u = Psi . r_hat (when u_out != null) and accumulates
// S3 = sum corr * u (when corr != null).  Combined state (COMB = true, a0 = r_x Psi_x + r_y Psi_y,
// a2 = Psi_z): writes u only (psi and corr must be null).
template <int N, bool COMB>
__global__ void __launch_bounds__(ntz<N>()) k_z_final(const float2* __restrict__ a0, const float2* __restrict__ a1,
                                                      const float2* __restrict__ a2, Geo g, float* __restrict__ psi,
                                                      float* __restrict__ u_out, const float* __restrict__ corr,
                                                      double* __restrict__ partials, const int* __restrict__ active,
                                                      const float2* __restrict__ twg) {
  constexpr int NT = ntz<N>(), WP = wz<N>();
  using L = Lay<N, WP, false>;
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  __shared__ float2 buf[L::SIZE];
  __shared__ float2 tw[N];
  stage_twiddles<N, NT>(tw, twg);
  int y, x0, c, j;
  z_tile_coords<N, WP>(y, x0);
  frag_coords<N, WP, false>(c, j);
  const bool act = threadIdx.x < L::NTF;
  const long long n3 = (long long)N * N * N, cn = (long long)(N / 2 + 1) * N * N;
  a0 += b * cn; a1 += b * cn; a2 += b * cn;
  // each array is staged in LDS by direct loads while the previous one is transformed
  __shared__ float2 stage[ZStage<N, WP>::SIZE];
  z_stage_issue<N, WP, NT>(stage, a0, y, x0);
  z_stage_wait();
  __syncthreads();
  float2 px[8], py[8], v[8];
  if (act) z_pack_stage<N, WP>(px, stage, c, j);
  __syncthreads();
  if (!COMB) {
    z_stage_issue<N, WP, NT>(stage, a1, y, x0);
    fft_rr<N, WP, true, false>(px, buf, tw);
    z_stage_wait();
    __syncthreads();
    if (act) z_pack_stage<N, WP>(py, stage, c, j);
    __syncthreads();
  }
  z_stage_issue<N, WP, NT>(stage, a2, y, x0);
  fft_rr<N, WP, true, false>(COMB ? px : py, buf, tw);
  z_stage_wait();
  __syncthreads();
  if (act) z_pack_stage<N, WP>(v, stage, c, j);
  fft_rr<N, WP, true, false>(v, buf, tw);
  const float ry = los_comp(g, 1, y);
  const float rx0 = los_comp(g, 0, x0 + c), rx1 = los_comp(g, 0, x0 + c + WP);
  double acc = 0.0;
  if (act) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int z = j + r * (N / 8);
      const long long cell = b * n3 + ((long long)z * N + y) * N + x0 + c;
      if (!COMB && psi) {
        float* pb = psi + 3 * b * n3;
        const long long c0 = cell - b * n3, c1 = c0 + WP;
        if (in_bounds(c1, n3)) {
          pb[c0] = px[r].x;
          pb[c1] = px[r].y;
          pb[n3 + c0] = py[r].x;
          pb[n3 + c1] = py[r].y;
          pb[2 * n3 + c0] = v[r].x;
          pb[2 * n3 + c1] = v[r].y;
        }
      }
      if (u_out || (!COMB && corr)) {
        const float rz = los_comp(g, 2, z);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const float rx = h ? rx1 : rx0;
          const float r2 = los_r2(rx, ry, rz);
          const float ir = r2 > 0.f ? rsqrtf(r2) : 0.f;
          float u;
          if (COMB) {
            u = fmaf(rz, h ? v[r].y : v[r].x, h ? px[r].y : px[r].x) * ir;
          } else {
            const float sx = h ? px[r].y : px[r].x, sy = h ? py[r].y : py[r].x, sz = h ? v[r].y : v[r].x;
            u = (rx * sx + ry * sy + rz * sz) * ir;
          }
          if (u_out) u_out[cell + h * WP] = u;
          if (!COMB && corr) acc += (double)corr[cell + h * WP] * (double)u;
        }
      }
    }
  }
  if (!COMB && corr) {
    double t1, t2;
    block_sum2<NT>(acc, 0.0, &t1, &t2);
    if (threadIdx.x == 0) {
      partials[2 * ((long long)b * gridDim.x + blockIdx.x)] = t1;
      partials[2 * ((long long)b * gridDim.x + blockIdx.x) + 1] = 0.0;
    }
  }
}

// Radial-ratio diagnostic (Sec. 4, Table 1): per cell q = (Psi_ref . r) / (Psi . r); cells with
// Psi . r != 0 and lo <= q <= hi contribute q and q^2 (FP64 block sums into part[2 blk..]) and
// one count (cnt[blk]).  psi_ref: planar [b][3][n^3]; blockIdx.y = realisation.
template <int NT>
__global__ void __launch_bounds__(NT) k_ratio_stats(const float* __restrict__ psi, const float* __restrict__ psi_ref,
                                                    Geo g, int n, double lo, double hi, double* __restrict__ part,
                                                    unsigned long long* __restrict__ cnt) {
  const long long n3 = (long long)n * n * n;
  const int b = blockIdx.y;
  double s1 = 0.0, s2 = 0.0;
  unsigned long long c = 0;
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n3; i += (long long)gridDim.x * NT) {
    const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((long long)n * n));
    const float rx = los_comp(g, 0, x), ry = los_comp(g, 1, y), rz = los_comp(g, 2, z);
    const float* p = psi + b * 3 * n3;
    const float* q = psi_ref + b * 3 * n3;
    const double a = (double)rx * q[i] + (double)ry * q[n3 + i] + (double)rz * q[2 * n3 + i];
    const double d = (double)rx * p[i] + (double)ry * p[n3 + i] + (double)rz * p[2 * n3 + i];
    if (d != 0.0) {
      const double r = a / d;
      if (r >= lo && r <= hi) {
        s1 += r;
        s2 += r * r;
        ++c;
      }
    }
  }
  double t1, t2;
  block_sum2<NT>(s1, s2, &t1, &t2);
  __shared__ unsigned long long cs[NT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) cs[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tc = 0;
    for (int k = 0; k < NT / 64; ++k) tc += cs[k];
    const long long blk = (long long)b * gridDim.x + blockIdx.x;
    part[2 * blk] = t1;
    part[2 * blk + 1] = t2;
    cnt[blk] = tc;
  }
}

// ---------------------------------------------------------------------------
// y passes.  Tile: one kz plane, W consecutive x, all N rows; column-fast fragments.
// ---------------------------------------------------------------------------
template <int N, int W>
__device__ __forceinline__ void y_tile_coords(int& p, int& x0) {
  p = blockIdx.x / (N / W);
  x0 = (blockIdx.x % (N / W)) * W;
}

// Non-temporal loads in the y passes only where a tile row is a whole 128-byte line (16 columns).
template <int N> constexpr bool y_hint() { return wy<N>() >= 16; }

template <int N>
__device__ __forceinline__ void y_load(float2* v, const float2* __restrict__ a, int p, int x0, int c, int j) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const long long e = ((long long)p * N + j + r * (N / 8)) * N + x0 + c;
    v[r] = in_bounds(e, (long long)(N / 2 + 1) * N * N) ? ld_stream<y_hint<N>()>(a + e) : float2{};
  }
}

template <int N>
__device__ __forceinline__ void y_store(const float2* v, float2* __restrict__ a, int p, int x0, int c, int j) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const long long e = ((long long)p * N + j + r * (N / 8)) * N + x0 + c;
    if (in_bounds(e, (long long)(N / 2 + 1) * N * N)) st_stream(a + e, v[r]);
  }
}

// Row flags (flag != null): one byte per z tile (one y row, 2 wz consecutive x), [NA][batch][z tiles]
// for the forward pass, [batch][z tiles] shared by both arrays for the inverse one.  Forward: rows
// (y, x) whose z tile has flag 0 were not written by the z pass and are read as zeros.  Inverse:
// such rows are not stored (the z pass that follows does not read them).

template <int N, int NA, bool INV>
__global__ void __launch_bounds__(nty<N>()) k_y_plain(float2* __restrict__ a0, float2* __restrict__ a1,
                                                      const float2* __restrict__ twg,
                                                      const unsigned char* __restrict__ flag = nullptr) {
  constexpr int NT = nty<N>(), W = wy<N>(), NZT = N / (2 * wz<N>());
  static_assert((2 * wz<N>()) % W == 0, "a y tile lies inside one z tile");
  constexpr int NF = INV ? 1 : NA;                     // flag sets: per array (forward) or shared (inverse)
  using L = Lay<N, W, false>;
  __shared__ float2 buf[L::SIZE];
  __shared__ float2 tw[N];
  __shared__ unsigned char live[NF][N];                // the tile's row flags, staged with the twiddles
  stage_twiddles<N, NT>(tw, twg);
  int p, x0, c, j;
  y_tile_coords<N, W>(p, x0);
  frag_coords<N, W, false>(c, j);
  const bool act = threadIdx.x < L::NTF;
  const long long cn = (long long)(N / 2 + 1) * N * N;
  const int b = blockIdx.y;
  if (flag) {
    for (int i = threadIdx.x; i < NF * N; i += NT) {
      const int f = i / N, yy = i % N;
      live[f][yy] = flag[((long long)f * gridDim.y + b) * N * NZT + (long long)yy * NZT + x0 / (2 * wz<N>())];
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    float2* arr = (a == 0 ? a0 : a1) + b * cn;
    const unsigned char* lv = live[INV ? 0 : a];
    float2 v[8];
    if (act) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int yy = j + r * (N / 8);
        const long long e = ((long long)p * N + yy) * N + x0 + c;
        v[r] = (in_bounds(e, cn) && (INV || !flag || lv[yy])) ? ld_stream<y_hint<N>()>(arr + e) : float2{};
      }
    }
    fft_rr<N, W, INV, false>(v, buf, tw);
    if (act) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int yy = j + r * (N / 8);
        const long long e = ((long long)p * N + yy) * N + x0 + c;
        if (in_bounds(e, cn) && (!INV || !flag || lv[yy])) st_stream(arr + e, v[r]);
      }
    }
  }
}

// Inverse y with the displacement fan-out.  Full form (COMB = false), the three displacement
// components for the output:
//   a0 <- Y^-1[a0]                    (x component, i k'_x applied in the x pass)
//   a1 <- Y^-1[i k'_y a1]             (y component)
//   a2 <- i k'_z Y^-1[a1]             (z component)
// Combined form (COMB = true), what the z iteration needs: the scaled line-of-sight components r_x
// and r_y are constant along a z column, so the transverse part of Psi . r is formed here, before
// the z transform:
//   a0 <- r_x Y^-1[a0] + r_y Y^-1[i k'_y a1],   a2 <- i k'_z Y^-1[a1]   (a1 is left as it was)
template <int N, bool COMB>
__global__ void __launch_bounds__(nty<N>()) k_y_fanout(float2* __restrict__ a0, float2* __restrict__ a1,
                                                       float2* __restrict__ a2, Geo g, const int* __restrict__ active,
                                                       const float2* __restrict__ twg) {
  constexpr int NT = nty<N>(), W = wy<N>();
  using L = Lay<N, W, false>;
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  __shared__ float2 buf[L::SIZE];
  __shared__ float2 tw[N];
  stage_twiddles<N, NT>(tw, twg);
  int p, x0, c, j;
  y_tile_coords<N, W>(p, x0);
  frag_coords<N, W, false>(c, j);
  const bool act = threadIdx.x < L::NTF;
  const long long cn = (long long)(N / 2 + 1) * N * N;
  a0 += b * cn; a1 += b * cn; a2 += b * cn;
  // a1 first: once its z component is stored only w is live, so a0 is loaded while w is transformed
  // and no transform runs with more than two arrays live (97 VGPRs; holding a0 and a1 through the
  // first transform needs 119)
  float2 v[8], w[8];
  {
    float2 keep[8];
    if (act) {
      y_load<N>(keep, a1, p, x0, c, j);
#pragma unroll
      for (int r = 0; r < 8; ++r) w[r] = mul_i(keep[r]) * (g.kf * deriv_mode<N>(j + r * (N / 8)));
    }
    fft_rr<N, W, true, false>(keep, buf, tw);
    if (act) {
      const float kz = g.kf * deriv_mode<N>(p);     // p in [0, N/2]; N/2 is the Nyquist plane
#pragma unroll
      for (int r = 0; r < 8; ++r) keep[r] = mul_i(keep[r]) * kz;
      y_store<N>(keep, a2, p, x0, c, j);
      y_load<N>(v, a0, p, x0, c, j);               // in flight during the transform of w
    }
  }
  fft_rr<N, W, true, false>(w, buf, tw);
  if (!COMB && act) y_store<N>(w, a1, p, x0, c, j);
  fft_rr<N, W, true, false>(v, buf, tw);
  if (act) {
    if (COMB) {
      const float rx = los_comp(g, 0, x0 + c);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const float ry = los_comp(g, 1, j + r * (N / 8));
        const float2 t = v[r] * rx;
        v[r] = make_float2(fmaf(ry, w[r].x, t.x), fmaf(ry, w[r].y, t.y));
      }
    }
    y_store<N>(v, a0, p, x0, c, j);
  }
}

// Full fan-out state -> combined state, in place: a0 <- r_x a0 + r_y a1 (the same arithmetic as the
// combined fan-out; a2 is shared by both states).  Element-wise over [kz][y][x] spectra.
template <int N>
__global__ void __launch_bounds__(256) k_y_combine(float2* __restrict__ a0, const float2* __restrict__ a1, Geo g,
                                                   const int* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const long long cn = (long long)(N / 2 + 1) * N * N;
  a0 += b * cn; a1 += b * cn;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < cn; i += (long long)gridDim.x * 256) {
    const float rx = los_comp(g, 0, (int)(i % N)), ry = los_comp(g, 1, (int)((i / N) % N));
    const float2 t = a0[i] * rx, w = a1[i];
    a0[i] = make_float2(fmaf(ry, w.x, t.x), fmaf(ry, w.y, t.y));
  }
}

// Forward y with the divergence fan-in.  In: a0 = Z[q], a1 = i k'_z Z[r_z q] (z spectra of the
// iteration's q = u / |r| with r the scaled line of sight, so that V_j = q r_j):
//   a0 <- r_x Y[a0]                   (x component Y Z[V_x]; i k'_x applied in the x pass)
//   a1 <- i k'_y Y[r_y a0] + Y[a1]    (y component plus the z component)
template <int N>
__global__ void __launch_bounds__(nty<N>()) k_y_fanin(float2* __restrict__ a0, float2* __restrict__ a1, Geo g,
                                                      const int* __restrict__ active, const float2* __restrict__ twg) {
  constexpr int NT = nty<N>(), W = wy<N>();
  using L = Lay<N, W, false>;
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  __shared__ float2 buf[L::SIZE];
  __shared__ float2 tw[N];
  stage_twiddles<N, NT>(tw, twg);
  int p, x0, c, j;
  y_tile_coords<N, W>(p, x0);
  frag_coords<N, W, false>(c, j);
  const bool act = threadIdx.x < L::NTF;
  const long long cn = (long long)(N / 2 + 1) * N * N;
  a0 += b * cn; a1 += b * cn;
  float2 v[8], keep[8];
  if (act) {
    y_load<N>(v, a0, p, x0, c, j);
#pragma unroll
    for (int r = 0; r < 8; ++r) keep[r] = v[r] * los_comp(g, 1, j + r * (N / 8));
  }
  fft_rr<N, W, false, false>(v, buf, tw);
  if (act) {
    const float rx = los_comp(g, 0, x0 + c);
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = v[r] * rx;
    y_store<N>(v, a0, p, x0, c, j);
    y_load<N>(v, a1, p, x0, c, j);                  // in flight during the next transform
  }
  fft_rr<N, W, false, false>(keep, buf, tw);
  if (act) {
#pragma unroll
    for (int r = 0; r < 8; ++r) keep[r] = mul_i(keep[r]) * (g.kf * deriv_mode<N>(j + r * (N / 8)));
  }
  fft_rr<N, W, false, false>(v, buf, tw);
  if (act) {
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = v[r] + keep[r];
    y_store<N>(v, a1, p, x0, c, j);
  }
}

// ---------------------------------------------------------------------------
// x passes.  Tile: W consecutive rows (row = kz * N + ky), all N x; row-fast fragments.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void x_load(float2* v, const float2* __restrict__ a, long long row, int j) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const long long e = row * N + j + r * (N / 8);
    v[r] = in_bounds(e, (long long)(N / 2 + 1) * N * N) ? ld_stream(a + e) : float2{};
  }
}

template <int N>
__device__ __forceinline__ void x_store(const float2* v, float2* __restrict__ a, long long row, int j) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const long long e = row * N + j + r * (N / 8);
    if (in_bounds(e, (long long)(N / 2 + 1) * N * N)) st_stream(a + e, v[r]);
  }
}

// k^2 and the derivative components of element (row, kx).
template <int N>
__device__ __forceinline__ void x_wavenumbers(long long row, int kx, float kf, float& k2, float& dx, float& dy,
                                              float& dz, int& kzi) {
  const int ky = (int)(row % N);
  kzi = (int)(row / N);
  const float mx = signed_mode<N>(kx), my = signed_mode<N>(ky), mz = (float)kzi;
  k2 = kf * kf * (mx * mx + my * my + mz * mz);
  dx = kf * deriv_mode<N>(kx);
  dy = kf * deriv_mode<N>(ky);
  dz = kzi == N / 2 ? 0.f : kf * mz;
}

// Forward x, Gaussian smoothing S(k) = exp(-k^2 R^2 / 2) with the 1/N^3 of the inverse, inverse x.
template <int N, int NA>
__global__ void __launch_bounds__(ntx<N>()) k_x_smooth(float2* __restrict__ a0, float2* __restrict__ a1, Geo g,
                                                       const float2* __restrict__ twg) {
  constexpr int NT = ntx<N>(), W = wx<N>();
  using L = Lay<N, W, true>;
  __shared__ float2 buf[L::SIZE];
  __shared__ float2 tw[N];
  stage_twiddles<N, NT>(tw, twg);
  int c, j;
  frag_coords<N, W, true>(c, j);
  const bool act = threadIdx.x < L::NTF;
  const long long cn = (long long)(N / 2 + 1) * N * N;
  const long long row = (long long)blockIdx.x * W + c;
  const int b = blockIdx.y;
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    float2* arr = (a == 0 ? a0 : a1) + b * cn;
    float2 v[8];
    if (act) x_load<N>(v, arr, row, j);
    fft_rr<N, W, false, true>(v, buf, tw);
    if (act) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        float k2, dx, dy, dz;
        int kzi;
        x_wavenumbers<N>(row, j + r * (N / 8), g.kf, k2, dx, dy, dz, kzi);
        v[r] = v[r] * (expf(-k2 * g.smooth_c) * g.inv_n3);
      }
    }
    fft_rr<N, W, true, true>(v, buf, tw);
    if (act) x_store<N>(v, arr, row, j);
  }
}

// Forward x of the overdensity -> D_s (stored); P = D_s / (b k^2 N^3);
// a0 <- X^-1[i k'_x P], a1 <- X^-1[P].
// HELM: the transformed field F is first multiplied by i k'_x and P = i k'_x F / (k^2 N^3); the
// fan-out then yields IFFT[-k'_j k'_x F / k^2], minus the irrotational part of (F) x (Sec. 4.1).
template <int N, bool HELM = false>
__global__ void __launch_bounds__(ntx<N>()) k_x_start(float2* __restrict__ a0, float2* __restrict__ a1,
                                                      float2* __restrict__ ds, Geo g, const float2* __restrict__ twg) {
  constexpr int NT = ntx<N>(), W = wx<N>();
  using L = Lay<N, W, true>;
  __shared__ float2 buf[L::SIZE];
  __shared__ float2 tw[N];
  stage_twiddles<N, NT>(tw, twg);
  int c, j;
  frag_coords<N, W, true>(c, j);
  const bool act = threadIdx.x < L::NTF;
  const long long cn = (long long)(N / 2 + 1) * N * N;
  const long long row = (long long)blockIdx.x * W + c;
  const int b = blockIdx.y;
  a0 += b * cn; a1 += b * cn; ds += b * cn;
  float2 v[8], pr[8];
  if (act) x_load<N>(v, a0, row, j);
  fft_rr<N, W, false, true>(v, buf, tw);
  if (act) {
    x_store<N>(v, ds, row, j);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      float k2, dx, dy, dz;
      int kzi;
      x_wavenumbers<N>(row, j + r * (N / 8), g.kf, k2, dx, dy, dz, kzi);
      if (HELM) v[r] = mul_i(v[r]) * dx;
      pr[r] = k2 > 0.f ? v[r] * ((HELM ? g.inv_n3 : g.inv_bn3) / k2) : make_float2(0.f, 0.f);
      v[r] = mul_i(pr[r]) * dx;
    }
  }
  fft_rr<N, W, true, true>(v, buf, tw);
  if (act) x_store<N>(v, a0, row, j);
  fft_rr<N, W, true, true>(pr, buf, tw);
  if (act) x_store<N>(pr, a1, row, j);
}

// State X (a0 = X^-1[i k'_x P], a1 = X^-1[P], P = D / (b k^2 N^3)) rebuilt from a stored spectrum D;
// the tail of k_x_start without its forward transform.
template <int N>
__global__ void __launch_bounds__(ntx<N>()) k_x_refan(float2* __restrict__ a0, float2* __restrict__ a1,
                                                      const float2* __restrict__ d, Geo g,
                                                      const int* __restrict__ active, const float2* __restrict__ twg) {
  constexpr int NT = ntx<N>(), W = wx<N>();
  using L = Lay<N, W, true>;
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  __shared__ float2 buf[L::SIZE];
  __shared__ float2 tw[N];
  stage_twiddles<N, NT>(tw, twg);
  int c, j;
  frag_coords<N, W, true>(c, j);
  const bool act = threadIdx.x < L::NTF;
  const long long cn = (long long)(N / 2 + 1) * N * N;
  const long long row = (long long)blockIdx.x * W + c;
  a0 += b * cn; a1 += b * cn; d += b * cn;
  float2 v[8], pr[8];
  if (act) {
    x_load<N>(v, d, row, j);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      float k2, dx, dy, dz;
      int kzi;
      x_wavenumbers<N>(row, j + r * (N / 8), g.kf, k2, dx, dy, dz, kzi);
      pr[r] = k2 > 0.f ? v[r] * (g.inv_bn3 / k2) : make_float2(0.f, 0.f);
      v[r] = mul_i(pr[r]) * dx;
    }
  }
  fft_rr<N, W, true, true>(v, buf, tw);
  if (act) x_store<N>(v, a0, row, j);
  fft_rr<N, W, true, true>(pr, buf, tw);
  if (act) x_store<N>(pr, a1, row, j);
}

// Helmholtz split output: irrotational = -Psi (the fan-out of the HELM start), solenoidal =
// f x - irrotational; planar [b][3][n^3]; sol may be null.
__global__ void __launch_bounds__(256) k_helm_out(const float* __restrict__ psi, const float* __restrict__ f,
                                                  int n, int batch, float* __restrict__ irr,
                                                  float* __restrict__ sol) {
  const long long n3 = (long long)n * n * n;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n3 * batch; i += (long long)gridDim.x * 256) {
    const long long b = i / n3, c = i - b * n3;
    const float* p = psi + b * 3 * n3;
    const float ix = -p[c], iy = -p[n3 + c], iz = -p[2 * n3 + c];
    irr[(b * 3 + 0) * n3 + c] = ix;
    irr[(b * 3 + 1) * n3 + c] = iy;
    irr[(b * 3 + 2) * n3 + c] = iz;
    if (sol) {
      sol[(b * 3 + 0) * n3 + c] = f[i] - ix;
      sol[(b * 3 + 1) * n3 + c] = -iy;
      sol[(b * 3 + 2) * n3 + c] = -iz;
    }
  }
}

// One iteration's k-space step:
//   div = i k'_x X[a0] + X[a1];  D_{n+1} = D_s + f div  (stored to dnext); with a relaxation weight
//   omega != 1, D_{n+1} = D_n + omega (D_s + f div - D_n)
//   partial sums of  sum w k'^2 |D_{n+1} - D_n|^2 / k^4  and  sum w k'^2 |D_{n+1}|^2 / k^4
//   (w = 2 inside the halved kz axis) -> convergence norm by Parseval
//   P = D_{n+1} / (b k^2 N^3);  a0 <- X^-1[i k'_x P],  a1 <- X^-1[P]
// dprev and dnext may be the same buffer (element-wise in place).
// RECON_X_WAVES > 0: occupancy hint (waves per SIMD) for the x iteration, which bounds its registers
#if RECON_X_WAVES > 0
#define RECON_X_ITER_BOUNDS(N) __launch_bounds__(ntx<N>(), RECON_X_WAVES)
#else
#define RECON_X_ITER_BOUNDS(N) __launch_bounds__(ntx<N>())
#endif
template <int N>
__global__ void RECON_X_ITER_BOUNDS(N) k_x_iter(float2* __restrict__ a0, float2* __restrict__ a1,
                                                     const float2* __restrict__ ds, const float2* dprev,
                                                     float2* dnext, Geo g, double* __restrict__ partials,
                                                     const int* __restrict__ active, const float2* __restrict__ twg,
                                                     float omega) {
  constexpr int NT = ntx<N>(), W = wx<N>();
  using L = Lay<N, W, true>;
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  __shared__ float2 buf[L::SIZE];
  __shared__ float2 tw[N];
  stage_twiddles<N, NT>(tw, twg);
  int c, j;
  frag_coords<N, W, true>(c, j);
  const bool act = threadIdx.x < L::NTF;
  const long long cn = (long long)(N / 2 + 1) * N * N;
  const long long row = (long long)blockIdx.x * W + c;
  a0 += b * cn; a1 += b * cn; ds += b * cn; dprev += b * cn; dnext += b * cn;
  float2 xa[8], v[8];
  if (act) x_load<N>(xa, a0, row, j);
  fft_rr<N, W, false, true>(xa, buf, tw);
  if (act) x_load<N>(v, a1, row, j);
  fft_rr<N, W, false, true>(v, buf, tw);
  double num = 0.0, den = 0.0;
  if (act) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int kx = j + r * (N / 8);
      float k2, dx, dy, dz;
      int kzi;
      x_wavenumbers<N>(row, kx, g.kf, k2, dx, dy, dz, kzi);
      const float2 div = mul_i(xa[r]) * dx + v[r];
      const long long idx = row * N + kx;
      const float2 dsv = ds[idx];
      const float2 dp = dprev[idx];
      float2 dn = make_float2(fmaf(g.growth, div.x, dsv.x), fmaf(g.growth, div.y, dsv.y));
      if (omega != 1.f) dn = make_float2(fmaf(omega, dn.x - dp.x, dp.x), fmaf(omega, dn.y - dp.y, dp.y));
      dnext[idx] = dn;
      if (k2 > 0.f) {
        const float wgt = (kzi == 0 || kzi == N / 2) ? 1.f : 2.f;
        const float kd2 = dx * dx + dy * dy + dz * dz;
        const float f = wgt * kd2 / (k2 * k2);
        const float ex = dn.x - dp.x, ey = dn.y - dp.y;
        num += (double)(f * (ex * ex + ey * ey));
        den += (double)(f * (dn.x * dn.x + dn.y * dn.y));
        v[r] = dn * (g.inv_bn3 / k2);
      } else {
        v[r] = make_float2(0.f, 0.f);
      }
      xa[r] = mul_i(v[r]) * dx;
    }
  }
  {
    double t1, t2;
    block_sum2<NT>(num, den, &t1, &t2);
    if (threadIdx.x == 0) {
      partials[2 * ((long long)b * gridDim.x + blockIdx.x) + 0] = t1;
      partials[2 * ((long long)b * gridDim.x + blockIdx.x) + 1] = t2;
    }
  }
  fft_rr<N, W, true, true>(xa, buf, tw);
  if (act) x_store<N>(xa, a0, row, j);
  fft_rr<N, W, true, true>(v, buf, tw);
  if (act) x_store<N>(v, a1, row, j);
}

// Fixed-order reduction of per-block partial pairs: out[b] = sum over blocks.
__global__ void __launch_bounds__(1024) k_reduce_pairs(const double* __restrict__ partials, int nblk,
                                                       double* __restrict__ out) {
  // one block per realisation; four independent accumulators per thread keep many loads in flight
  constexpr int NT = 1024;
  const int b = blockIdx.x;
  const double2* p = (const double2*)partials + (long long)b * nblk;
  double s0[4] = {0.0, 0.0, 0.0, 0.0}, s1[4] = {0.0, 0.0, 0.0, 0.0};
  int i = threadIdx.x;
  for (; i + 3 * NT < nblk; i += 4 * NT) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double2 v = p[i + k * NT];
      s0[k] += v.x;
      s1[k] += v.y;
    }
  }
  for (; i < nblk; i += NT) {
    const double2 v = p[i];
    s0[0] += v.x;
    s1[0] += v.y;
  }
  double t0, t1;
  block_sum2<NT>((s0[0] + s0[1]) + (s0[2] + s0[3]), (s1[0] + s1[1]) + (s1[2] + s1[3]), &t0, &t1);
  if (threadIdx.x == 0) { out[2 * b] = t0; out[2 * b + 1] = t1; }
}

// ---------------------------------------------------------------------------
// Shift: CIC interpolation of Psi at each object with the deposit's stencil.
//   galaxies: disp = -Psi - f (Psi . r_hat) r_hat;  randoms: disp = -Psi
// ---------------------------------------------------------------------------
// CIC interpolation of Psi at one valid position, with the deposit's cell index and fractions, and its
// displacement: galaxies -Psi - f (Psi . r_hat) r_hat, randoms -Psi.  fetch(ix, iy, iz, ii) returns
// Psi at the corner ix, iy, iz (wrapped) of base cell ii, from memory or from a staged footprint.
template <class Fetch>
__device__ __forceinline__ void shift_one_f(float px, float py, float pz, const float uu[3], Fetch fetch,
                                            const CicGeo& cg, float ox, float oy, float oz, float growth,
                                            int galaxies, float d[3]) {
  int ii[3];
  float t[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float fl = floorf(uu[a]);
    t[a] = __fsub_rn(uu[a], fl);
    ii[a] = ((int)fl) & (cg.n - 1);
  }
  // every rounding is spelled out and nothing is contracted, so that the direct and the brick-order
  // shift give the same bits
  float p0 = 0.f, p1 = 0.f, p2 = 0.f;
#pragma unroll
  for (int cnr = 0; cnr < 8; ++cnr) {
    const int dx = cnr & 1, dy = (cnr >> 1) & 1, dz = cnr >> 2;
    const float wx = dx ? t[0] : __fsub_rn(1.f, t[0]), wy = dy ? t[1] : __fsub_rn(1.f, t[1]),
                wz = dz ? t[2] : __fsub_rn(1.f, t[2]);
    const float wgt = __fmul_rn(__fmul_rn(wx, wy), wz);
    const float4 v = fetch(dx, dy, dz, ii);
    p0 = fmaf(wgt, v.x, p0);
    p1 = fmaf(wgt, v.y, p1);
    p2 = fmaf(wgt, v.z, p2);
  }
  float d0 = -p0, d1 = -p1, d2 = -p2;
  if (galaxies && growth != 0.f) {
    const float rx = __fsub_rn(px, ox), ry = __fsub_rn(py, oy), rz = __fsub_rn(pz, oz);
    const float r2 = fmaf(rz, rz, fmaf(ry, ry, __fmul_rn(rx, rx)));
    if (r2 > 0.f) {
      const float ir = rsqrtf(r2);
      const float hx = __fmul_rn(rx, ir), hy = __fmul_rn(ry, ir), hz = __fmul_rn(rz, ir);
      const float u = __fmul_rn(growth, fmaf(p2, hz, fmaf(p1, hy, __fmul_rn(p0, hx))));
      d0 = fmaf(-u, hx, d0);
      d1 = fmaf(-u, hy, d1);
      d2 = fmaf(-u, hz, d2);
    }
  }
  d[0] = d0;
  d[1] = d1;
  d[2] = d2;
}

// The same from the displacement in memory (planar, one realisation's [3][N^3]).
__device__ __forceinline__ void shift_one(float px, float py, float pz, const float uu[3], const float* __restrict__ pb,
                                          const CicGeo& cg, float ox, float oy, float oz, float growth,
                                          int galaxies, float d[3]) {
  const int m = cg.n - 1, n = cg.n;
  const long long n3 = (long long)n * n * n;
  shift_one_f(px, py, pz, uu,
              [&](int dx, int dy, int dz, const int ii[3]) {
                const long long c = (((long long)((ii[2] + dz) & m) * n + ((ii[1] + dy) & m)) * n) + ((ii[0] + dx) & m);
                return in_bounds(c, n3) ? make_float4(pb[c], pb[n3 + c], pb[2 * n3 + c], 0.f) : float4{};
              },
              cg, ox, oy, oz, growth, galaxies, d);
}

// Scaled grid coordinates of a position; false for a non-finite or far position.
__device__ __forceinline__ bool shift_coords(float px, float py, float pz, const CicGeo& cg, float uu[3]) {
  const float pp[3] = {px, py, pz};
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float d = __fsub_rn(pp[a], cg.o[a]);
    uu[a] = keep_rounded(__fmul_rn(d, cg.s));
    ok = ok && (fabsf(uu[a]) < 1073741824.0f);
  }
  return ok;
}

__global__ void __launch_bounds__(256) k_shift(const float* __restrict__ pos, long long n,
                                               const long long* __restrict__ off, int batch,
                                               const float* __restrict__ psi, CicGeo cg, float ox, float oy,
                                               float oz, float growth, int galaxies, float* __restrict__ disp,
                                               float* __restrict__ pos_out, int* __restrict__ err) {
  const long long n3 = (long long)cg.n * cg.n * cg.n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float px = pos[3 * i], py = pos[3 * i + 1], pz = pos[3 * i + 2];
    float uu[3];
    if (!shift_coords(px, py, pz, cg, uu)) {
      atomicAdd(err, 1);
#pragma unroll
      for (int a = 0; a < 3; ++a) disp[3 * i + a] = 0.f;
      continue;
    }
    const int b = off ? find_realisation(off, batch, i) : 0;
    float d[3];
    shift_one(px, py, pz, uu, psi + 3 * (long long)b * n3, cg, ox, oy, oz, growth, galaxies, d);
    disp[3 * i] = d[0];
    disp[3 * i + 1] = d[1];
    disp[3 * i + 2] = d[2];
    if (pos_out) {
      pos_out[3 * i] = __fadd_rn(px, d[0]);
      pos_out[3 * i + 1] = __fadd_rn(py, d[1]);
      pos_out[3 * i + 2] = __fadd_rn(pz, d[2]);
    }
  }
}

// The brick-order shift with one block per 16^3 brick: the block stages the displacement at the
// 17^3 nodes its objects' stencils can reach (base cells 0..15 of the brick and their upper corners;
// rows of 17 consecutive x per component) in LDS, then interpolates every object of the brick from
// LDS.  Same arithmetic as k_shift.
template <int NT>
__global__ void __launch_bounds__(NT) k_shift_brick(const float4* __restrict__ sorted,
                                                    const unsigned* __restrict__ start,
                                                    const float* __restrict__ psi, CicGeo cg, float ox, float oy,
                                                    float oz, float growth, int galaxies,
                                                    float4* __restrict__ tmp) {
  constexpr int F = kBrick + 1, F3 = F * F * F;
  __shared__ float px_[F3], py_[F3], pz_[F3];
  const long long key = brick_of_block();
  const unsigned lo = start[key], hi = start[key + 1];
  if (lo == hi) return;
  const int n = cg.n, m = n - 1;
  const int nbs = (n + kBrick - 1) / kBrick;
  const long long per = (long long)nbs * nbs * nbs;
  const int b = (int)(key / per);
  const long long kk = key - (long long)b * per;
  const int bx = (int)(kk % nbs) * kBrick, by = (int)((kk / nbs) % nbs) * kBrick,
            bz = (int)(kk / ((long long)nbs * nbs)) * kBrick;
  const long long n3 = (long long)n * n * n;
  const float* pb = psi + 3 * (long long)b * n3;
  // node (lx, ly, lz) of the footprint is grid node (bx + lx, by + ly, bz + lz), wrapped; consecutive
  // threads take consecutive x of one row
  for (int l = threadIdx.x; l < F3; l += NT) {
    const int lx = l % F, ly = (l / F) % F, lz = l / (F * F);
    const long long c = (((long long)((bz + lz) & m) * n + ((by + ly) & m)) * n) + ((bx + lx) & m);
    const bool ok = in_bounds(c, n3);
    px_[l] = ok ? pb[c] : 0.f;
    py_[l] = ok ? pb[n3 + c] : 0.f;
    pz_[l] = ok ? pb[2 * n3 + c] : 0.f;
  }
  __syncthreads();
  constexpr int U = kObjBatch;
  for (long long j0 = (long long)lo + threadIdx.x; j0 < hi; j0 += (long long)NT * U) {
    float4 rr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long j = j0 + (long long)u * NT;
      rr[u] = sorted[j < hi ? j : hi - 1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long j = j0 + (long long)u * NT;
      if (j >= hi) break;
      const float4 r = rr[u];
      float uu[3], d[3];
      shift_coords(r.x, r.y, r.z, cg, uu);
      shift_one_f(r.x, r.y, r.z, uu,
                  [&](int dx, int dy, int dz, const int ii[3]) {
                    // the base cell lies in this brick (it decided the object's brick)
                    const int l = ((ii[2] - bz + dz) * F + (ii[1] - by + dy)) * F + (ii[0] - bx + dx);
                    return make_float4(px_[l], py_[l], pz_[l], 0.f);
                  },
                  cg, ox, oy, oz, growth, galaxies, d);
      tmp[j] = make_float4(d[0], d[1], d[2], 0.f);
    }
  }
}

// Back to the caller's order: object i takes the displacement of its slot (an object the deposit
// rejected has no slot: counted in err, displacement 0, as in k_shift).  Consecutive objects of one
// scatter chunk have their slots in short runs per brick, so their staged results share lines; the
// 8 XCDs (workgroups are dealt to them round robin) each take a contiguous eighth of the objects,
// and a block takes U adjacent 256-object chunks, so that the chunks in flight on one XCD form a
// single window that moves forward in dispatch order and the lines it gathers are reused in that
// XCD's L2 (gridDim.x is a multiple of 8; the result does not depend on the dispatch order).
__global__ void __launch_bounds__(256) k_shift_unpermute(const unsigned* __restrict__ slot_of,
                                                         const float4* __restrict__ tmp, long long n,
                                                         const float* __restrict__ pos, float* __restrict__ disp,
                                                         float* __restrict__ pos_out, int* __restrict__ err) {
  const long long chunks = (n + 255) / 256, per_x = gridDim.x / 8;
  const int xcd = blockIdx.x % 8;
  const long long c_lo = chunks * xcd / 8, c_hi = chunks * (xcd + 1) / 8;
  constexpr int U = kObjBatch;
  for (long long c0 = c_lo + (long long)(blockIdx.x / 8) * U; c0 < c_hi; c0 += per_x * U) {
    // the U chunks' slot and staged-result loads are issued together
    unsigned sl[U];
    float4 dd[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = (c0 + u) * 256 + threadIdx.x;
      sl[u] = (c0 + u < c_hi && i < n) ? slot_of[i] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) dd[u] = sl[u] < n ? tmp[sl[u]] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long c = c0 + u;
      const long long i = c * 256 + threadIdx.x;
      if (c >= c_hi || i >= n) continue;
      const float4 d = dd[u];
      if (sl[u] >= n) atomicAdd(err, 1);
      disp[3 * i] = d.x;
      disp[3 * i + 1] = d.y;
      disp[3 * i + 2] = d.z;
      if (pos_out) {
        pos_out[3 * i] = __fadd_rn(pos[3 * i], d.x);
        pos_out[3 * i + 1] = __fadd_rn(pos[3 * i + 1], d.y);
        pos_out[3 * i + 2] = __fadd_rn(pos[3 * i + 2], d.z);
      }
    }
  }
}

}  // namespace recon
