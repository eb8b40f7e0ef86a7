// Device helpers for the reconstruction kernels (gfx950, wave64).
//
// The 3D transforms are built from one block-level primitive: a length-N
// complex FFT of W independent columns, computed by self-sorting Stockham
// passes on register fragments that exchange through an LDS tile (see the
// fragment engine below).  Twiddles come from an FP32 table of exp(-2 pi i m/N)
// rounded once from FP64 on the host and staged into LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "recon_tuning.h"

namespace recon {

constexpr int kThreads = 256;

// Bounds checks of the debug build (-DRECON_DEBUG): an index outside [0, n) of the array it addresses
// is counted in recon_debug_count and the access is skipped; the release build compiles the checks
// out (in_bounds is the constant true).  recon_debug_violations() reads the count.
#ifdef RECON_DEBUG
__device__ unsigned long long recon_debug_count;
__device__ __forceinline__ bool in_bounds(long long i, long long n) {
  if (i >= 0 && i < n) return true;
  atomicAdd(&recon_debug_count, 1ull);
  return false;
}
#else
__device__ __forceinline__ constexpr bool in_bounds(long long, long long) { return true; }
#endif

// Streaming accesses of the transform passes.  Each pass reads and writes its spectra once, and a
// spectrum (539 MB at 512^3) is far larger than the caches, so the accesses may carry the
// non-temporal hint: RECON_STREAM bit 0 for stores, bit 1 for loads (the staging loads of the z
// passes included); 0 keeps plain accesses.
typedef float recon_v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_stream(float2* p, float2 v) {
#if RECON_STREAM & 1
  __builtin_nontemporal_store(recon_v2f{v.x, v.y}, reinterpret_cast<recon_v2f*>(p));
#else
  *p = v;
#endif
}
// HINT = false keeps a plain load: the y passes' loads at tiles of fewer than 16 columns (rows of
// 64-byte segments, half a line) ran slower with the hint.
template <bool HINT = true>
__device__ __forceinline__ float2 ld_stream(const float2* p) {
#if RECON_STREAM & 2
  if constexpr (HINT) {
    const recon_v2f t = __builtin_nontemporal_load(reinterpret_cast<const recon_v2f*>(p));
    return make_float2(t.x, t.y);
  }
#endif
  return *p;
}
constexpr int kStageCachePolicy = (RECON_STREAM & 2) ? 2 : 0;   // the nt bit of the staging loads

__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

__device__ __forceinline__ float2 operator+(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 operator-(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 operator*(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }
// i * a
__device__ __forceinline__ float2 mul_i(float2 a) { return make_float2(-a.y, a.x); }

// Multiply by the quarter-turn root: -i for the forward transform, +i for the inverse.
template <bool INV>
__device__ __forceinline__ float2 quarter(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2* v) {
  float2 t = v[0];
  v[0] = t + v[1];
  v[1] = t - v[1];
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& y0, float2& y1, float2& y2, float2& y3) {
  float2 t0 = y0 + y2, t1 = y0 - y2, t2 = y1 + y3, t3 = quarter<INV>(y1 - y3);
  y0 = t0 + t2;
  y2 = t0 - t2;
  y1 = t1 + t3;
  y3 = t1 - t3;
}

template <bool INV>
__device__ __forceinline__ void dft4v(float2* v) { dft4<INV>(v[0], v[1], v[2], v[3]); }

// 8-point DFT, one decimation-in-frequency radix-2 stage followed by two 4-point DFTs.
template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
  const float r = 0.70710678118654752440f;
  float2 a0 = v[0] + v[4], a1 = v[1] + v[5], a2 = v[2] + v[6], a3 = v[3] + v[7];
  float2 b0 = v[0] - v[4], b1 = v[1] - v[5], b2 = v[2] - v[6], b3 = v[3] - v[7];
  if (INV) {
    b1 = make_float2((b1.x - b1.y) * r, (b1.x + b1.y) * r);
    b3 = make_float2((-b3.x - b3.y) * r, (b3.x - b3.y) * r);
  } else {
    b1 = make_float2((b1.x + b1.y) * r, (b1.y - b1.x) * r);
    b3 = make_float2((b3.y - b3.x) * r, (-b3.x - b3.y) * r);
  }
  b2 = quarter<INV>(b2);
  dft4<INV>(a0, a1, a2, a3);
  dft4<INV>(b0, b1, b2, b3);
  v[0] = a0; v[2] = a1; v[4] = a2; v[6] = a3;
  v[1] = b0; v[3] = b1; v[5] = b2; v[7] = b3;
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(float2* v) {
  if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 4) dft4v<INV>(v);
  else dft8<INV>(v);
}

// ---------------------------------------------------------------------------
// Register-fragment FFT engine.
//
// A tile holds W independent length-N columns.  Each of the (N/8) W fragment
// threads owns one radix-8 butterfly: element r of its fragment v[8] is row
// i = j + r N/8 of column c.  Two thread layouts exist:
//   column-fast (JF = false): c = t % W, j = t / W   (tiles whose columns are contiguous in memory)
//   row-fast    (JF = true):  j = t % (N/8), c = t / (N/8)   (tiles whose rows are contiguous)
// so that global loads and stores in fragment layout are coalesced either way.
// The first radix-8 pass (sub-transform length NS = 1) consumes the fragment from
// registers, the middle passes run LDS to LDS, and the last radix-8 pass
// (NS = N/8) leaves the result in the same fragment layout in registers, so an
// N = 512 transform costs two LDS exchanges.  Radix-2/4 passes (log2 N not a
// multiple of 3) sit in the middle; each fragment thread then handles 8/R of them.
// LDS layouts: column-fast [N][W+1]; row-fast [W][N + N/8] with one pad slot per 8 rows.  In the
// row-fast layout a wave holds one column, so its lanes write rows 8 j + r (first pass) and read
// rows j + (N/8) r: with the pad the first pattern lands on word offsets 18 j, distinct modulo the
// 64 banks over 32 lanes, and the second is contiguous.
// ---------------------------------------------------------------------------
template <int N, int W, bool JF>
struct Lay {
  static constexpr int LDC = W + 1;
  static constexpr int LDJ = N + N / 8;
  static constexpr int SIZE = JF ? W * LDJ : N * LDC;
  static constexpr int NTF = (N / 8) * W;   // fragment threads
  __device__ __forceinline__ static int at(int i, int c) { return JF ? c * LDJ + i + (i >> 3) : i * LDC + c; }
};

// Block size that runs one fragment per thread (at least one wave).
template <int N, int W>
constexpr int frag_threads() { return (N / 8) * W < 64 ? 64 : (N / 8) * W; }

template <int N, int W, int R, bool JF>
__device__ __forceinline__ void bfly_coords(int b, int& c, int& j) {
  if (JF) { j = b % (N / R); c = b / (N / R); }
  else { c = b % W; j = b / W; }
}

// Fragment coordinates of this thread (valid when threadIdx.x < NTF).
template <int N, int W, bool JF>
__device__ __forceinline__ void frag_coords(int& c, int& j) { bfly_coords<N, W, 8, JF>(threadIdx.x, c, j); }

// Generic LDS-to-LDS Stockham pass (radix R, completed sub-transform length NS).
template <int N, int W, int R, int NS, bool INV, bool JF>
__device__ __forceinline__ void lds_pass(float2* buf, const float2* tw) {
  using L = Lay<N, W, JF>;
  constexpr int Q = 8 / R;
  const int t = threadIdx.x;
  float2 v[Q][R];
  if (t < L::NTF) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      int c, j;
      bfly_coords<N, W, R, JF>(t + q * L::NTF, c, j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[L::at(j + r * (N / R), c)];
    }
  }
  __syncthreads();
  if (t < L::NTF) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      int c, j;
      bfly_coords<N, W, R, JF>(t + q * L::NTF, c, j);
      const int k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[r * k * (N / (NS * R))];
          if (INV) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
      dftR<R, INV>(v[q]);
      const int idx = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[L::at(idx + r * NS, c)] = v[q][r];
    }
  }
  __syncthreads();
}

// First radix-8 pass from the register fragment into LDS (preceded by a barrier that
// protects earlier readers of the tile).
template <int N, int W, bool INV, bool JF>
__device__ __forceinline__ void first_pass(float2* v, float2* buf) {
  using L = Lay<N, W, JF>;
  __syncthreads();
  if (threadIdx.x < L::NTF) {
    int c, j;
    frag_coords<N, W, JF>(c, j);
    dft8<INV>(v);
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[L::at(j * 8 + r, c)] = v[r];
  }
  __syncthreads();
}

// Last radix-8 pass (NS = N/8) from LDS into the register fragment.
template <int N, int W, bool INV, bool JF>
__device__ __forceinline__ void last_pass(float2* v, const float2* buf, const float2* tw) {
  using L = Lay<N, W, JF>;
  if (threadIdx.x < L::NTF) {
    int c, j;
    frag_coords<N, W, JF>(c, j);
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = buf[L::at(j + r * (N / 8), c)];
#pragma unroll
    for (int r = 1; r < 8; ++r) {
      float2 w = tw[r * j];
      if (INV) w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
    dft8<INV>(v);
  }
}

// Middle passes between NS = 8 and NS = N/8 (factor N/64).  The split of the factor for 512 and
// 1024 is a tuning knob (RECON_MID_512: 0 = 8, 1 = 2 x 4, 2 = 4 x 2; RECON_MID_1024: 0 = 4 x 4,
// 1 = 2 x 8, 2 = 8 x 2), chosen by the autotuner (autotune.py).
template <int N, int W, bool INV, bool JF>
__device__ __forceinline__ void middle_passes(float2* buf, const float2* tw) {
  if constexpr (N == 128) lds_pass<N, W, 2, 8, INV, JF>(buf, tw);
  else if constexpr (N == 256) lds_pass<N, W, 4, 8, INV, JF>(buf, tw);
  else if constexpr (N == 512) {
    if constexpr (RECON_MID_512 == 1) {
      lds_pass<N, W, 2, 8, INV, JF>(buf, tw);
      lds_pass<N, W, 4, 16, INV, JF>(buf, tw);
    } else if constexpr (RECON_MID_512 == 2) {
      lds_pass<N, W, 4, 8, INV, JF>(buf, tw);
      lds_pass<N, W, 2, 32, INV, JF>(buf, tw);
    } else {
      lds_pass<N, W, 8, 8, INV, JF>(buf, tw);
    }
  } else if constexpr (N == 1024) {
    if constexpr (RECON_MID_1024 == 1) {
      lds_pass<N, W, 2, 8, INV, JF>(buf, tw);
      lds_pass<N, W, 8, 16, INV, JF>(buf, tw);
    } else if constexpr (RECON_MID_1024 == 2) {
      lds_pass<N, W, 8, 8, INV, JF>(buf, tw);
      lds_pass<N, W, 2, 64, INV, JF>(buf, tw);
    } else {
      lds_pass<N, W, 4, 8, INV, JF>(buf, tw);
      lds_pass<N, W, 4, 32, INV, JF>(buf, tw);
    }
  }
}

// ---------------------------------------------------------------------------
// Optional radix-8 stage on the matrix cores with split-bfloat16 compensated products (the
// precision study's DFT-as-GEMM variant; the default transforms are FP32 throughout).
//
// A radix-8 butterfly is the product of the 8-point DFT matrix (in real form, 16 x 16) with the 16
// real inputs of the butterfly after their twiddle factors.  Sixteen butterflies form the 16
// columns of one v_mfma_f32_16x16x16bf16_1k product.  Operands are split into bfloat16 terms,
// x = x_1 + x_2 (+ x_3), x_1 = bf16(x), x_2 = bf16(x - x_1), x_3 = bf16(x - x_1 - x_2), and the
// products whose terms are not both of the smallest order are accumulated in FP32 (TERMS = 2: three
// products, relative error about 2^-16; TERMS = 3: six products, about 2^-24).
// Operand layout: lane l holds A[l%16][4(l/16) + 0..3] and B[4(l/16) + 0..3][l%16]; the result is
// D[4(l/16) + 0..3][l%16].  Lane l therefore feeds complex inputs 2(l/16), 2(l/16) + 1 of butterfly
// l%16 and receives the complex outputs of the same indices.
// ---------------------------------------------------------------------------
typedef short mf_s4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

// Split four values into TERMS bfloat16 operand vectors.
template <int TERMS>
__device__ __forceinline__ void bf16_split4(const float* x, mf_s4* t) {
  float r[4] = {x[0], x[1], x[2], x[3]};
#pragma unroll
  for (int k = 0; k < TERMS; ++k) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const unsigned short h = bf16_rne(r[i]);
      t[k][i] = (short)h;
      r[i] -= bf16_val(h);
    }
  }
}

// Real form of the 8-point DFT, element (m, kk): output (m/2, re|im), input (kk/2, re|im).
template <bool INV>
__device__ __forceinline__ float dft8_real(int m, int kk) {
  const float s = 0.70710678118654752440f;
  const float c8[8] = {1.f, s, 0.f, -s, -1.f, -s, 0.f, s};
  const float s8[8] = {0.f, s, 1.f, s, 0.f, -s, -1.f, -s};
  const int a = ((m >> 1) * (kk >> 1)) & 7;
  const float wr = c8[a], wi = INV ? s8[a] : -s8[a];    // omega^(p r), omega = exp(-+ 2 pi i / 8)
  if ((m & 1) == 0) return (kk & 1) ? -wi : wr;
  return (kk & 1) ? wr : wi;
}

// LDS-to-LDS radix-8 Stockham pass (completed sub-transform length NS) on the matrix cores.  Every
// wave handles the 64 butterflies of its 64 fragment threads, 16 per product.  Needs (N/8) W to be a
// multiple of 64 (whole waves).
template <int N, int W, int NS, bool INV, bool JF, int TERMS>
__device__ __forceinline__ void lds_pass_r8_mfma(float2* buf, const float2* tw) {
  using L = Lay<N, W, JF>;
  static_assert(L::NTF % 64 == 0, "the matrix-core radix-8 pass runs whole waves");
  const int t = threadIdx.x, lane = t & 63, wbase = t - lane, n = lane & 15, q = lane >> 4;
  float x[4][4];
  if (t < L::NTF) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      int c, j;
      bfly_coords<N, W, 8, JF>(wbase + 16 * g + n, c, j);
      const int k = j % NS;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = 2 * q + h;
        float2 v = buf[L::at(j + r * (N / 8), c)];
        if constexpr (NS > 1) {
          float2 w = tw[r * k * (N / (NS * 8))];
          if (INV) w.y = -w.y;
          v = cmul(v, w);
        }
        x[g][2 * h] = v.x;
        x[g][2 * h + 1] = v.y;
      }
    }
  }
  __syncthreads();
  if (t < L::NTF) {
    float a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = dft8_real<INV>(n, 4 * q + i);
    mf_s4 at[TERMS];
    bf16_split4<TERMS>(a, at);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      mf_s4 bt[TERMS];
      bf16_split4<TERMS>(x[g], bt);
      mf_f4 acc = {0.f, 0.f, 0.f, 0.f};
      // smallest products first
      if constexpr (TERMS == 3) {
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(at[1], bt[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(at[2], bt[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(at[0], bt[2], acc, 0, 0, 0);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(at[1], bt[0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(at[0], bt[1], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(at[0], bt[0], acc, 0, 0, 0);
      int c, j;
      bfly_coords<N, W, 8, JF>(wbase + 16 * g + n, c, j);
      const int k = j % NS;
      const int idx = (j / NS) * NS * 8 + k;
      buf[L::at(idx + (2 * q) * NS, c)] = make_float2(acc[0], acc[1]);
      buf[L::at(idx + (2 * q + 1) * NS, c)] = make_float2(acc[2], acc[3]);
    }
  }
  __syncthreads();
}

// Length-N FFT of the tile, register fragment in and out.  The caller must place a
// barrier before its next write to the tile.  SPLIT > 0 (N >= 64): the last radix-8 stage runs on
// the matrix cores with SPLIT bfloat16 terms per operand (lds_pass_r8_mfma).
template <int N, int W, bool INV, bool JF, int SPLIT = 0>
__device__ __forceinline__ void fft_rr(float2* v, float2* buf, const float2* tw) {
  using L = Lay<N, W, JF>;
  if constexpr (N == 8) {
    if (threadIdx.x < L::NTF) dft8<INV>(v);
  } else if constexpr (N < 64) {
    first_pass<N, W, INV, JF>(v, buf);
    lds_pass<N, W, N / 8, 8, INV, JF>(buf, tw);
    if (threadIdx.x < L::NTF) {
      int c, j;
      frag_coords<N, W, JF>(c, j);
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = buf[L::at(j + r * (N / 8), c)];
    }
  } else if constexpr (SPLIT > 0) {
    first_pass<N, W, INV, JF>(v, buf);
    middle_passes<N, W, INV, JF>(buf, tw);
    lds_pass_r8_mfma<N, W, N / 8, INV, JF, SPLIT>(buf, tw);
    if (threadIdx.x < L::NTF) {
      int c, j;
      frag_coords<N, W, JF>(c, j);
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = buf[L::at(j + r * (N / 8), c)];
    }
  } else {
    first_pass<N, W, INV, JF>(v, buf);
    middle_passes<N, W, INV, JF>(buf, tw);
    last_pass<N, W, INV, JF>(v, buf, tw);
  }
}

// Length-N FFT of the tile, register fragment in, natural order in LDS out (ends with a barrier).
// SPLIT as in fft_rr.
template <int N, int W, bool INV, bool JF, int SPLIT = 0>
__device__ __forceinline__ void fft_rl(float2* v, float2* buf, const float2* tw) {
  using L = Lay<N, W, JF>;
  if constexpr (N == 8) {
    __syncthreads();
    if (threadIdx.x < L::NTF) {
      int c, j;
      frag_coords<N, W, JF>(c, j);
      dft8<INV>(v);
#pragma unroll
      for (int r = 0; r < 8; ++r) buf[L::at(r, c)] = v[r];
    }
    __syncthreads();
  } else if constexpr (N < 64) {
    first_pass<N, W, INV, JF>(v, buf);
    lds_pass<N, W, N / 8, 8, INV, JF>(buf, tw);
  } else {
    first_pass<N, W, INV, JF>(v, buf);
    middle_passes<N, W, INV, JF>(buf, tw);
    if constexpr (SPLIT > 0) lds_pass_r8_mfma<N, W, N / 8, INV, JF, SPLIT>(buf, tw);
    else lds_pass<N, W, 8, N / 8, INV, JF>(buf, tw);
  }
}

// ---------------------------------------------------------------------------
// Wave-local transforms of length 512: one column per wave, lane j owning rows j + 64 r (one radix-8
// fragment), exchanging through the wave's own LDS region (row i at i + i/8, one pad slot per 8 rows),
// so that no block barrier is needed inside a transform and the waves of a block drift freely between
// the block's staging barriers.  Three radix-8 Stockham passes: registers -> LDS, LDS -> LDS, and
// LDS -> registers (wfft_rr) or LDS -> LDS in natural order (wfft_rl).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ int wat(int i) { return i + (i >> 3); }

template <bool INV>
__device__ __forceinline__ void wfft_first(float2* v, float2* reg, int j) {
  dft8<INV>(v);
#pragma unroll
  for (int r = 0; r < 8; ++r) reg[wat(8 * j + r)] = v[r];
  wave_sync();
}

template <int NS, bool INV>
__device__ __forceinline__ void wfft_mid(float2* reg, const float2* tw, int j) {
  constexpr int N = 512;
  float2 v[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = reg[wat(j + r * (N / 8))];
  wave_sync();                                        // every lane has read before any lane writes
  const int k = j % NS;
#pragma unroll
  for (int r = 1; r < 8; ++r) {
    float2 w = tw[r * k * (N / (NS * 8))];
    if (INV) w.y = -w.y;
    v[r] = cmul(v[r], w);
  }
  dft8<INV>(v);
  const int idx = (j / NS) * NS * 8 + k;
#pragma unroll
  for (int r = 0; r < 8; ++r) reg[wat(idx + r * NS)] = v[r];
  wave_sync();
}

// register fragment in and out (rows j + 64 r); the region is free again when it returns
template <bool INV>
__device__ __forceinline__ void wfft_rr(float2* v, float2* reg, const float2* tw, int j) {
  wfft_first<INV>(v, reg, j);
  wfft_mid<8, INV>(reg, tw, j);
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = reg[wat(j + r * 64)];
#pragma unroll
  for (int r = 1; r < 8; ++r) {
    float2 w = tw[r * j];
    if (INV) w.y = -w.y;
    v[r] = cmul(v[r], w);
  }
  dft8<INV>(v);
  wave_sync();                                        // the region's reads are done
}

// register fragment in, natural order in the region out
template <bool INV>
__device__ __forceinline__ void wfft_rl(float2* v, float2* reg, const float2* tw, int j) {
  wfft_first<INV>(v, reg, j);
  wfft_mid<8, INV>(reg, tw, j);
  wfft_mid<64, INV>(reg, tw, j);
}

template <int N, int NT>
__device__ __forceinline__ void stage_twiddles(float2* tw_lds, const float2* __restrict__ tw) {
  for (int i = threadIdx.x; i < N; i += NT) tw_lds[i] = tw[i];
}

// Wavenumber index m in [0, N) -> signed mode m' (Nyquist as -N/2).
template <int N>
__device__ __forceinline__ float signed_mode(int m) { return (float)(m < N / 2 ? m : m - N); }
// Derivative mode: zero at the Nyquist index.
template <int N>
__device__ __forceinline__ float deriv_mode(int m) { return m == N / 2 ? 0.f : signed_mode<N>(m); }

// Deterministic block reduction of two doubles (fixed shuffle tree, then fixed LDS order).
template <int NT>
__device__ __forceinline__ void block_sum2(double a, double b, double* out_a, double* out_b) {
  __shared__ double red[2][NT / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) { red[0][wave] = a; red[1][wave] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) { sa += red[0][w]; sb += red[1][w]; }
    *out_a = sa;
    *out_b = sb;
  }
}

}  // namespace recon
