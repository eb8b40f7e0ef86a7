// Device helpers for the reconstruction kernels (gfx950, wave64).
//
// The 3D transforms are built from one block-level primitive: a length-N
// complex FFT applied to W independent columns held in LDS as a row-major
// [N][W+1] tile of float2 (one pad column keeps both the column-wise and the
// row-wise access patterns free of bank conflicts).  The tile is transformed
// by self-sorting Stockham passes (a radix-2 or radix-4 pass when log2 N is
// not a multiple of 3, then radix-8 passes), each pass staging its
// butterflies through registers: read all inputs, barrier, write all
// outputs, barrier.  Twiddles come from an FP32 table of exp(-2 pi i m/N)
// rounded once from FP64 on the host and staged into LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace recon {

constexpr int kThreads = 256;

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

// One self-sorting Stockham pass of radix R on a [N][LD] LDS tile holding W columns.
// NS is the length of the sub-transforms already completed by earlier passes.
template <int N, int W, int NT, int R, int NS, bool INV>
__device__ __forceinline__ void stockham_pass(float2* buf, const float2* tw) {
  constexpr int LD = W + 1;
  constexpr int NB = (N / R) * W;
  constexpr int PER = (NB + NT - 1) / NT;
  float2 v[PER][R];
#pragma unroll
  for (int it = 0; it < PER; ++it) {
    const int b = threadIdx.x + it * NT;
    if (NB % NT == 0 || b < NB) {
      const int c = b % W, j = b / W;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = buf[(j + r * (N / R)) * LD + c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < PER; ++it) {
    const int b = threadIdx.x + it * NT;
    if (NB % NT == 0 || b < NB) {
      const int c = b % W, j = b / W;
      const int k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[r * k * (N / (NS * R))];
          if (INV) w.y = -w.y;
          v[it][r] = cmul(v[it][r], w);
        }
      }
      dftR<R, INV>(v[it]);
      const int idx = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(idx + r * NS) * LD + c] = v[it][r];
    }
  }
  __syncthreads();
}

template <int N, int W, int NT, int NS, bool INV>
__device__ __forceinline__ void radix8_passes(float2* buf, const float2* tw) {
  if constexpr (NS < N) {
    stockham_pass<N, W, NT, 8, NS, INV>(buf, tw);
    radix8_passes<N, W, NT, NS * 8, INV>(buf, tw);
  }
}

// In-place length-N FFT of the W columns of an [N][W+1] LDS tile.  The caller
// must have issued a barrier after filling the tile; the function ends with one.
template <int N, int W, int NT, bool INV>
__device__ __forceinline__ void tile_fft(float2* buf, const float2* tw) {
  constexpr int REM = ilog2(N) % 3;
  if constexpr (REM == 1) {
    stockham_pass<N, W, NT, 2, 1, INV>(buf, tw);
    radix8_passes<N, W, NT, 2, INV>(buf, tw);
  } else if constexpr (REM == 2) {
    stockham_pass<N, W, NT, 4, 1, INV>(buf, tw);
    radix8_passes<N, W, NT, 4, INV>(buf, tw);
  } else {
    radix8_passes<N, W, NT, 1, INV>(buf, tw);
  }
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
