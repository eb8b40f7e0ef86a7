// Learned-start network kernels (not part of the paper's method): three periodic
// 3x3x3 convolutions, channels-last bfloat16 activations, FP32 accumulation.
//
//   x0 = [delta_s, S_U u_p, r_x, r_y, r_z, 0, 0, 0]     (assembled on the fly)
//   a1 = relu(conv(x0; W1, b1))      8 -> 16   BF16 MFMA
//   a2 = relu(conv(a1; W2, b2))     16 -> 16   BF16 MFMA
//   y  =      conv(a2; W3, b3)      16 -> 1    BF16 MFMA (k_conv_out_mfma)
//   Delta u = y / S_U
//
// Parameter vector (FP32, device): W1 [16][27][8], b1 [16], W2 [16][27][16], b2 [16],
// W3 [1][27][16], b3 [1]; tap t = (dz+1)*9 + (dy+1)*3 + (dx+1), offset (dx, dy, dz).
//
// Forward convolutions (k_conv_fwd, k_conv_out_mfma) are implicit GEMMs on
// v_mfma_f32_16x16x32_bf16 over 16 x 8 x 8 output tiles (see there).  The training
// kernels (data gradient k_conv16, weight gradient k_wgrad16) use v_mfma_f32_16x16x16bf16_1k:
// M = 16 output positions (one x row of a 16 x 4 x 4 output tile), N = 16 output channels,
// K = 27 taps x C_in input channels in blocks of 16.  Operand layout of that instruction:
// lane l holds A[l%16][4(l/16)+0..3], B[4(l/16)+0..3][l%16], and the result
// D[4(l/16)+0..3][l%16].
#pragma once

#include "recon_kernels.hpp"

namespace recon {
namespace cnn {

constexpr int CIN = 8, CH = 16;
constexpr float S_U = 0.1f;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + CH * 27 * CIN, OFF_W2 = OFF_B1 + CH, OFF_B2 = OFF_W2 + CH * 27 * CH,
              OFF_W3 = OFF_B2 + CH, OFF_B3 = OFF_W3 + 27 * CH, NPARAM = OFF_B3 + 1;
constexpr int K1 = 27 * CIN, K1P = 224;      // layer-1 K padded to a multiple of 16
constexpr int K2 = 27 * CH;                  // 432
// output tile: 16 (x) by 4 (y) by 4 (z) positions, halo tile 18 x 6 x 6 cells
constexpr int TX = 16, TY = 4, TZ = 4, HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HCELLS = HX * HY * HZ;
constexpr int TPOS = TX * TY * TZ;   // 256

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

struct Geo3 {
  int n;
  float hs;
  float ds[3];
};

// Tile origin of this block: blockIdx.x runs over (x tiles, y tiles, z tiles), blockIdx.y = realisation.
__device__ __forceinline__ void tile_origin(int n, int& x0, int& y0, int& z0) {
  const int ntx = n / TX, nty = n / TY;
  const int t = blockIdx.x;
  x0 = (t % ntx) * TX;
  y0 = ((t / ntx) % nty) * TY;
  z0 = (t / (ntx * nty)) * TZ;
}

__device__ __forceinline__ long long halo_cell_global(int n, int x0, int y0, int z0, int hc) {
  const int hx = hc % HX, hy = (hc / HX) % HY, hz = hc / (HX * HY);
  const long long x = (x0 - 1 + hx) & (n - 1), y = (y0 - 1 + hy) & (n - 1), z = (z0 - 1 + hz) & (n - 1);
  return (z * n + y) * n + x;
}

// Stage the halo tile of a channels-last bf16 tensor with C channels into LDS.
template <int C>
__device__ __forceinline__ void stage_bf16(unsigned short* tile, const unsigned short* __restrict__ src, int n, int x0,
                                           int y0, int z0) {
  constexpr int CH4 = C / 4;
  for (int e = threadIdx.x; e < HCELLS * CH4; e += 256) {
    const int hc = e / CH4, q = e % CH4;
    const long long g = halo_cell_global(n, x0, y0, z0, hc);
    *(uint2*)(tile + hc * C + 4 * q) = *(const uint2*)(src + g * C + 4 * q);
  }
}

// Stage the assembled 8-channel input x0 = [delta, S_U u_p, r_hat, 0, 0, 0].
__device__ __forceinline__ void stage_x0(unsigned short* tile, const float* __restrict__ delta,
                                         const float* __restrict__ up, const Geo3& g, int x0, int y0, int z0) {
  for (int hc = threadIdx.x; hc < HCELLS; hc += 256) {
    const int hx = hc % HX, hy = (hc / HX) % HY, hz = hc / (HX * HY);
    const int x = (x0 - 1 + hx) & (g.n - 1), y = (y0 - 1 + hy) & (g.n - 1), z = (z0 - 1 + hz) & (g.n - 1);
    const long long c = ((long long)z * g.n + y) * g.n + x;
    const float rx = fmaf(g.hs, (float)x, g.ds[0]), ry = fmaf(g.hs, (float)y, g.ds[1]),
                rz = fmaf(g.hs, (float)z, g.ds[2]);
    const float r2 = rx * rx + ry * ry + rz * rz;
    const float ir = r2 > 0.f ? rsqrtf(r2) : 0.f;
    unsigned short* t = tile + hc * CIN;
    t[0] = to_bf16(delta[c]);
    t[1] = to_bf16(S_U * up[c]);
    t[2] = to_bf16(rx * ir);
    t[3] = to_bf16(ry * ir);
    t[4] = to_bf16(rz * ir);
    t[5] = 0;
    t[6] = 0;
    t[7] = 0;
  }
}

// Halo-tile cell of output row (zr, yr), position m, shifted by tap t.
__device__ __forceinline__ int tap_cell(int zr, int yr, int m, int t) {
  const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
  return ((zr + 1 + dz) * HY + (yr + 1 + dy)) * HX + (m + 1 + dx);
}

// Convolution with C input channels and 16 output channels on MFMA.
//   SRC 0: input is a bf16 tensor [n^3][C];  SRC 1: input is x0 assembled from (delta, u_p) (C = 8).
//   EPI 0: out = bf16(relu(acc + bias));     EPI 1: out = bf16(acc) where gate > 0, else 0.
// wk: weights in MFMA layout [16 out][KP] bf16 (KP >= 27 C, zero padded).
template <int C, int KP, int SRC, int EPI>
__global__ void __launch_bounds__(256) k_conv16(const unsigned short* __restrict__ in, const float* __restrict__ delta,
                                                const float* __restrict__ up, Geo3 g, const unsigned short* __restrict__ wk,
                                                const float* __restrict__ bias, const unsigned short* __restrict__ gate,
                                                unsigned short* __restrict__ out) {
  constexpr int KB = KP / 16;
  __shared__ unsigned short tile[HCELLS * C];
  const long long n3 = (long long)g.n * g.n * g.n;
  const int b = blockIdx.y;
  int x0, y0, z0;
  tile_origin(g.n, x0, y0, z0);
  if (SRC == 0) stage_bf16<C>(tile, in + b * n3 * C, g.n, x0, y0, z0);
  else stage_x0(tile, delta + b * n3, up + b * n3, g, x0, y0, z0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, q = lane >> 4;
  // B operands (weights) for every K block, kept in registers
  s4 bw[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) bw[kb] = *(const s4*)(wk + m * KP + kb * 16 + 4 * q);
  __syncthreads();
#pragma unroll
  for (int row = 0; row < 4; ++row) {
    const int rr = wave * 4 + row, zr = rr / TY, yr = rr % TY;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int k = kb * 16 + 4 * q;
      int t = k / C;
      if (t > 26) t = 26;                            // padded K: weights are zero there
      const s4 a = *(const s4*)(tile + tap_cell(zr, yr, m, t) * C + (k % C));
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw[kb], acc, 0, 0, 0);
    }
    // lane holds D[pos = 4q + i][channel = m]
    const long long rowbase = ((long long)(z0 + zr) * g.n + (y0 + yr)) * g.n + x0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long long cell = b * n3 + rowbase + 4 * q + i;
      float v = acc[i];
      if (EPI == 0) v = fmaxf(v + bias[m], 0.f);
      else v = from_bf16(gate[cell * CH + m]) > 0.f ? v : 0.f;
      out[cell * CH + m] = to_bf16(v);
    }
  }
}

// ---------------------------------------------------------------------------
// Forward convolution on v_mfma_f32_16x16x32_bf16 (inference and the training forward).
//
// Block tile 16 (x) x 8 (y) x 8 (z) output cells, halo 18 x 10 x 10 cells staged once in LDS;
// each wave owns 16 x 4 x 4 outputs (16 output rows of 16 cells).  The wave walks the 6 x 6 input
// rows of its halo: an input row's A fragment (16 cells x K = 32) is loaded from LDS once and
// multiplied into every output row that uses it (up to 9), so one LDS read feeds up to 9 MFMAs.
// K = 32 of one fragment: C = 16: half 0 = taps dx = -1, 0 (16 channels each), half 1 = dx = +1
// and 16 zero columns;  C = 8: dx = -1, 0, +1 and 8 zero columns.
// Operand layout of that instruction: lane l holds A[l%16][8(l/16)+0..7], B[8(l/16)+0..7][l%16],
// and the result D[4(l/16)+0..3][l%16].
constexpr int FX = 16, FY = 8, FZ = 8, GX = FX + 2, GY = FY + 2, GZ = FZ + 2, GCELLS = GX * GY * GZ;
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Byte offset of the 16-byte half h of halo cell c (C = 16: halves swapped on every other group of
// four cells so that 8 consecutive lanes reading one half hit distinct banks).
template <int C>
__device__ __forceinline__ int frag_off(int c, int h) {
  if (C == 16) return c * 32 + ((h ^ ((c >> 2) & 1)) << 4);
  return c * 16;
}

// Weight fragments: C = 16: wf[(g * 2 + h) * 64 + lane], C = 8: wf[g * 64 + lane], with
// g = (dz+1)*3 + (dy+1); 8 bf16 per lane in the B layout above.
__global__ void __launch_bounds__(256) k_prep_frag(const float* __restrict__ th, uint4* __restrict__ wf1,
                                                   uint4* __restrict__ wf2) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= 9 * 64 + 9 * 2 * 64) return;
  unsigned short v[8];
  if (e < 9 * 64) {
    const int g = e / 64, lane = e % 64, o = lane % 16, q = lane / 16;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int t = g * 3 + q;                     // dx = q - 1
      v[j] = q < 3 ? to_bf16(th[OFF_W1 + (o * 27 + t) * CIN + j]) : (unsigned short)0;
    }
    wf1[e] = make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16), v[6] | (v[7] << 16));
  } else {
    const int f = e - 9 * 64, g = f / 128, h = (f / 64) % 2, lane = f % 64, o = lane % 16, q = lane / 16;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * q + j, ch = k % 16;
      const int dx = h == 0 ? (k < 16 ? -1 : 0) : 1;
      const bool zero = h == 1 && k >= 16;
      v[j] = zero ? (unsigned short)0 : to_bf16(th[OFF_W2 + (o * 27 + g * 3 + dx + 1) * CH + ch]);
    }
    wf2[f] = make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16), v[6] | (v[7] << 16));
  }
}

// Stage the 18 x 10 x 10 halo of a channels-last bf16 tensor into LDS: every thread issues all of
// its 16-byte loads before the first LDS store so the loads are in flight together.
template <int C>
__device__ __forceinline__ void stage_halo(unsigned char* lds, const unsigned short* __restrict__ src, int n, int x0,
                                           int y0, int z0) {
  constexpr int CPC = C / 8, TOTAL = GCELLS * CPC, PER = (TOTAL + 255) / 256;
  const int msk = n - 1;
  uint4 v[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e0 = threadIdx.x + k * 256;
    const int e = e0 < TOTAL ? e0 : TOTAL - 1;        // tail lanes reload the last chunk
    const int c = e / CPC, h = e % CPC;
    const int hx = c % GX, hy = (c / GX) % GY, hz = c / (GX * GY);
    const long long gc = ((long long)((z0 - 1 + hz) & msk) * n + ((y0 - 1 + hy) & msk)) * n + ((x0 - 1 + hx) & msk);
    v[k] = *(const uint4*)(src + gc * C + 8 * h);
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + k * 256;
    if (e < TOTAL) *(uint4*)(lds + frag_off<C>(e / CPC, e % CPC)) = v[k];
  }
}

//   SRC 0: input is a bf16 tensor [n^3][C];  SRC 1: input is x0 assembled from (delta, u_p), C = 8.
//   out = bf16(relu(acc + bias)), channels-last [n^3][16].
template <int C, int SRC>
__global__ void __launch_bounds__(256) k_conv_fwd(const unsigned short* __restrict__ in,
                                                     const float* __restrict__ delta, const float* __restrict__ up,
                                                     Geo3 g, const uint4* __restrict__ wf,
                                                     const float* __restrict__ bias, unsigned short* __restrict__ out) {
  constexpr int NH = C == 16 ? 2 : 1;
  // halo of the input (bf16 channels) during the products, then the output tile (16 channels, bf16)
  constexpr int LDS_IN = GCELLS * C * 2, LDS_OUT = FX * FY * FZ * 32;
  __shared__ __align__(16) unsigned char lds[LDS_IN > LDS_OUT ? LDS_IN : LDS_OUT];
  const long long n3 = (long long)g.n * g.n * g.n;
  const int b = blockIdx.y, msk = g.n - 1;
  const int nbx = g.n / FX, nby = g.n / FY;
  const int x0 = (blockIdx.x % nbx) * FX, y0 = ((blockIdx.x / nbx) % nby) * FY, z0 = (blockIdx.x / (nbx * nby)) * FZ;
  if (SRC == 0) {
    stage_halo<C>(lds, in + b * n3 * C, g.n, x0, y0, z0);
  } else {
    const float* dl = delta + b * n3;
    const float* ul = up + b * n3;
    constexpr int PER = (GCELLS + 255) / 256;
    float dv[PER], uv[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int c = threadIdx.x + k * 256;
      if (c < GCELLS) {
        const int hx = c % GX, hy = (c / GX) % GY, hz = c / (GX * GY);
        const long long gc = ((long long)((z0 - 1 + hz) & msk) * g.n + ((y0 - 1 + hy) & msk)) * g.n + ((x0 - 1 + hx) & msk);
        dv[k] = dl[gc];
        uv[k] = ul[gc];
      }
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int c = threadIdx.x + k * 256;
      if (c < GCELLS) {
        const int hx = c % GX, hy = (c / GX) % GY, hz = c / (GX * GY);
        const int x = (x0 - 1 + hx) & msk, y = (y0 - 1 + hy) & msk, z = (z0 - 1 + hz) & msk;
        const float rx = fmaf(g.hs, (float)x, g.ds[0]), ry = fmaf(g.hs, (float)y, g.ds[1]),
                    rz = fmaf(g.hs, (float)z, g.ds[2]);
        const float r2 = rx * rx + ry * ry + rz * rz;
        const float ir = r2 > 0.f ? rsqrtf(r2) : 0.f;
        const unsigned a0 = to_bf16(dv[k]), a1 = to_bf16(S_U * uv[k]);
        const unsigned a2 = to_bf16(rx * ir), a3 = to_bf16(ry * ir), a4 = to_bf16(rz * ir);
        *(uint4*)(lds + c * 16) = make_uint4(a0 | (a1 << 16), a2 | (a3 << 16), a4, 0u);
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, q = lane >> 4;
  bf8 bw[9][NH];
#pragma unroll
  for (int gi = 0; gi < 9; ++gi)
#pragma unroll
    for (int h = 0; h < NH; ++h) bw[gi][h] = __builtin_bit_cast(bf8, wf[(gi * NH + h) * 64 + lane]);
  __syncthreads();
  const int wy0 = 4 * (wave & 1), wz0 = 4 * (wave >> 1);
  f4 acc[4][4];
#pragma unroll
  for (int oz = 0; oz < 4; ++oz)
#pragma unroll
    for (int oy = 0; oy < 4; ++oy) acc[oz][oy] = f4{0.f, 0.f, 0.f, 0.f};
  const bf8 zero8 = __builtin_bit_cast(bf8, make_uint4(0u, 0u, 0u, 0u));
#pragma unroll
  for (int iz = 0; iz < 6; ++iz) {
#pragma unroll
    for (int iy = 0; iy < 6; ++iy) {
      const int rowc = ((wz0 + iz) * GY + (wy0 + iy)) * GX;
      bf8 a[NH];
      if (C == 16) {
        a[0] = __builtin_bit_cast(bf8, *(const uint4*)(lds + frag_off<C>(rowc + m + (q >> 1), q & 1)));
        const bf8 t1 = __builtin_bit_cast(bf8, *(const uint4*)(lds + frag_off<C>(rowc + m + 2, q & 1)));
        a[NH - 1] = q < 2 ? t1 : zero8;
      } else {
        const bf8 t0 = __builtin_bit_cast(bf8, *(const uint4*)(lds + frag_off<C>(rowc + m + (q < 3 ? q : 2), 0)));
        a[0] = q < 3 ? t0 : zero8;
      }
#pragma unroll
      for (int oz = 0; oz < 4; ++oz) {
        const int dz = iz - 1 - oz;
        if (dz < -1 || dz > 1) continue;
#pragma unroll
        for (int oy = 0; oy < 4; ++oy) {
          const int dy = iy - 1 - oy;
          if (dy < -1 || dy > 1) continue;
          const int gi = (dz + 1) * 3 + (dy + 1);
#pragma unroll
          for (int h = 0; h < NH; ++h)
            acc[oz][oy] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[h], bw[gi][h], acc[oz][oy], 0, 0, 0);
        }
      }
    }
  }
  // epilogue: lane (m, q) holds channel m of cells 4q..4q+3 of each output row; channel pairs are
  // exchanged with the neighbouring lane and the packed words go to the output tile in LDS
  // ([cell][16 channels]), from which every lane stores whole 16-byte halves of cells
  const float bm = bias[m];
  const bool even = (m & 1) == 0;
  __syncthreads();                                  // every wave is done with the halo
  unsigned* t32 = (unsigned*)lds;
#pragma unroll
  for (int oz = 0; oz < 4; ++oz) {
#pragma unroll
    for (int oy = 0; oy < 4; ++oy) {
      unsigned mine[4], other[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) mine[i] = to_bf16(fmaxf(acc[oz][oy][i] + bm, 0.f));
#pragma unroll
      for (int i = 0; i < 4; ++i) other[i] = (unsigned)__shfl_xor((int)mine[i], 1);
      const int cell0 = ((wz0 + oz) * FY + (wy0 + oy)) * FX + 4 * q;
      const int ch2 = m >> 1;                       // channel pair
      if (even) {
        t32[(cell0 + 0) * 8 + ch2] = mine[0] | (other[0] << 16);
        t32[(cell0 + 1) * 8 + ch2] = mine[1] | (other[1] << 16);
      } else {
        t32[(cell0 + 2) * 8 + ch2] = other[2] | (mine[2] << 16);
        t32[(cell0 + 3) * 8 + ch2] = other[3] | (mine[3] << 16);
      }
    }
  }
  __syncthreads();
  const uint4* t128 = (const uint4*)lds;
  uint4* o128 = (uint4*)out;
#pragma unroll
  for (int k = 0; k < FX * FY * FZ * 2 / 256; ++k) {
    const int e = threadIdx.x + k * 256;           // 16-byte half e % 2 of tile cell e / 2
    const int cell = e >> 1, lx = cell % FX, ly = (cell / FX) % FY, lz = cell / (FX * FY);
    const long long row = b * n3 + ((long long)(z0 + lz) * g.n + (y0 + ly)) * g.n + x0 + lx;
    o128[row * 2 + (e & 1)] = t128[e];
  }

}

// Output layer (16 -> 1) on MFMA for the forward pass: with one output channel the N dimension of
// the instruction runs over the wave's 16 output rows instead.  For input row (iz, iy) the B
// fragment column n = output row (oz, oy) = (n / 4, n % 4) holds W3 of tap (iz - 1 - oz, iy - 1 - oy, dx)
// (zero when that row is out of reach), so each A fragment is used once for all 16 output rows.
__global__ void __launch_bounds__(256) k_conv_out_mfma(const unsigned short* __restrict__ a2, Geo3 g,
                                                       const float* __restrict__ w3f, const float* __restrict__ b3,
                                                       float scale, float* __restrict__ y_out) {
  __shared__ __align__(16) unsigned char lds[GCELLS * CH * 2];
  __shared__ __align__(16) unsigned short w3b[27 * CH];
  const long long n3 = (long long)g.n * g.n * g.n;
  const int b = blockIdx.y, msk = g.n - 1;
  const int nbx = g.n / FX, nby = g.n / FY;
  const int x0 = (blockIdx.x % nbx) * FX, y0 = ((blockIdx.x / nbx) % nby) * FY, z0 = (blockIdx.x / (nbx * nby)) * FZ;
  stage_halo<CH>(lds, a2 + b * n3 * CH, g.n, x0, y0, z0);
  for (int i = threadIdx.x; i < 27 * CH; i += 256) w3b[i] = to_bf16(w3f[i]);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, q = lane >> 4;
  const int wy0 = 4 * (wave & 1), wz0 = 4 * (wave >> 1);
  const int oz = m >> 2, oy = m & 3;                  // output row of B / D column m
  const bf8 zero8 = __builtin_bit_cast(bf8, make_uint4(0u, 0u, 0u, 0u));
  f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int iz = 0; iz < 6; ++iz) {
#pragma unroll
    for (int iy = 0; iy < 6; ++iy) {
      const int rowc = ((wz0 + iz) * GY + (wy0 + iy)) * GX;
      const bf8 a0 = __builtin_bit_cast(bf8, *(const uint4*)(lds + frag_off<CH>(rowc + m + (q >> 1), q & 1)));
      const bf8 t1 = __builtin_bit_cast(bf8, *(const uint4*)(lds + frag_off<CH>(rowc + m + 2, q & 1)));
      const bf8 a1 = q < 2 ? t1 : zero8;
      const int dz = iz - 1 - oz, dy = iy - 1 - oy;
      const bool ok = dz >= -1 && dz <= 1 && dy >= -1 && dy <= 1;
      const int tb = ok ? (dz + 1) * 9 + (dy + 1) * 3 : 0;   // tap of dx = -1
      // half 0: q < 2 -> dx = -1, q >= 2 -> dx = 0;  half 1: q < 2 -> dx = +1, else zero
      const bf8 w0 = __builtin_bit_cast(bf8, *(const uint4*)(w3b + (tb + (q >> 1)) * CH + 8 * (q & 1)));
      const bf8 w1 = __builtin_bit_cast(bf8, *(const uint4*)(w3b + (tb + 2) * CH + 8 * (q & 1)));
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, ok ? w0 : zero8, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, (ok && q < 2) ? w1 : zero8, acc, 0, 0, 0);
    }
  }
  // lane (m, q) holds output row m, cells 4q .. 4q+3
  const float bb = b3[0];
  const long long row = b * n3 + ((long long)(z0 + wz0 + oz) * g.n + (y0 + wy0 + oy)) * g.n + x0 + 4 * q;
  *(float4*)(y_out + row) = make_float4((acc[0] + bb) * scale, (acc[1] + bb) * scale, (acc[2] + bb) * scale,
                                        (acc[3] + bb) * scale);
}

// Loss residual: r = y - S_U target; dy = 2 r / count; per-block partial of sum r^2.
__global__ void __launch_bounds__(256) k_loss(const float* __restrict__ y, const float* __restrict__ target,
                                              long long count, float* __restrict__ dy, double* __restrict__ partial) {
  double acc = 0.0;
  const float inv = 2.0f / (float)count;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < count; i += (long long)gridDim.x * 256) {
    const float r = y[i] - S_U * target[i];
    dy[i] = inv * r;
    acc += (double)r * (double)r;
  }
  double t1, t2;
  block_sum2<256>(acc, 0.0, &t1, &t2);
  if (threadIdx.x == 0) partial[blockIdx.x] = t1;
}

// Output-layer backward: dpre2[p][i] = bf16((sum_t W3[t][i] dy[p - d_t]) * [a2[p][i] > 0]),
// and per-block partials of dW3[t][i] = sum_p dy[p] a2[p + d_t][i] and db3 = sum_p dy[p].
__global__ void __launch_bounds__(256) k_conv_out_bwd(const float* __restrict__ dy, const unsigned short* __restrict__ a2,
                                                      Geo3 g, const float* __restrict__ w3,
                                                      unsigned short* __restrict__ dpre2, float* __restrict__ part) {
  __shared__ unsigned short tile[HCELLS * CH];
  __shared__ float dyt[HCELLS];
  __shared__ float w[27 * CH];
  const long long n3 = (long long)g.n * g.n * g.n;
  const int b = blockIdx.y;
  int x0, y0, z0;
  tile_origin(g.n, x0, y0, z0);
  stage_bf16<CH>(tile, a2 + b * n3 * CH, g.n, x0, y0, z0);
  for (int hc = threadIdx.x; hc < HCELLS; hc += 256) dyt[hc] = dy[b * n3 + halo_cell_global(g.n, x0, y0, z0, hc)];
  for (int i = threadIdx.x; i < 27 * CH; i += 256) w[i] = w3[i];
  __syncthreads();
  {
    const int m = threadIdx.x % TX, yr = (threadIdx.x / TX) % TY, zr = threadIdx.x / (TX * TY);
    float d[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) d[i] = 0.f;
    for (int t = 0; t < 27; ++t) {
      const float v = dyt[tap_cell(zr, yr, m, 26 - t)];      // dy(p - d_t)
#pragma unroll
      for (int i = 0; i < CH; ++i) d[i] = fmaf(w[t * CH + i], v, d[i]);
    }
    const int hc = tap_cell(zr, yr, m, 13);
    const long long cell = b * n3 + ((long long)(z0 + zr) * g.n + (y0 + yr)) * g.n + x0 + m;
#pragma unroll
    for (int i = 0; i < CH; ++i) dpre2[cell * CH + i] = to_bf16(from_bf16(tile[hc * CH + i]) > 0.f ? d[i] : 0.f);
  }
  // weight partials: entry e = t * 16 + i (432 entries) plus the bias (entry 432)
  const long long blk = (long long)b * gridDim.x + blockIdx.x;
  for (int e = threadIdx.x; e < 27 * CH + 1; e += 256) {
    float acc = 0.f;
    if (e < 27 * CH) {
      const int t = e / CH, i = e % CH;
      for (int p = 0; p < TPOS; ++p) {
        const int m = p % TX, yr = (p / TX) % TY, zr = p / (TX * TY);
        acc = fmaf(dyt[tap_cell(zr, yr, m, 13)], from_bf16(tile[tap_cell(zr, yr, m, t) * CH + i]), acc);
      }
    } else {
      for (int p = 0; p < TPOS; ++p) {
        const int m = p % TX, yr = (p / TX) % TY, zr = p / (TX * TY);
        acc += dyt[tap_cell(zr, yr, m, 13)];
      }
    }
    part[blk * (27 * CH + 1) + e] = acc;
  }
}

// Weight gradient of a 16-output convolution on MFMA:
//   dW[o][t C + i] = sum_p dpre[p][o] x[p + d_t][i],  db[o] = sum_p dpre[p][o]
// M = 16 output channels, N = 16 columns (C = 16: the channels of one tap; C = 8: two taps),
// K = 16 positions per instruction.  One block loops over the x tiles of one (y, z) tile
// row and writes one partial [16][KP + 1] (bias in the last column).
template <int C, int KP, int SRC>
__global__ void __launch_bounds__(256) k_wgrad16(const unsigned short* __restrict__ dpre,
                                                 const unsigned short* __restrict__ in, const float* __restrict__ delta,
                                                 const float* __restrict__ up, Geo3 g, float* __restrict__ part) {
  constexpr int NT = KP / 16;                 // column tiles: C = 16 -> 27 taps, C = 8 -> 14 tap pairs
  constexpr int TPW = (NT + 3) / 4;           // column tiles per wave
  __shared__ unsigned short tile[HCELLS * C];
  __shared__ unsigned short dt[CH][TPOS + 4];   // dpre of the tile, transposed [o][p]
  const long long n3 = (long long)g.n * g.n * g.n;
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, q = lane >> 4;
  f4 acc[TPW];
#pragma unroll
  for (int k = 0; k < TPW; ++k) acc[k] = f4{0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;
  const int ntx = g.n / TX, nty = g.n / TY;
  const int y0 = (blockIdx.x % nty) * TY, z0 = (blockIdx.x / nty) * TZ;
  for (int xt = 0; xt < ntx; ++xt) {
    const int x0 = xt * TX;
    __syncthreads();
    if (SRC == 0) stage_bf16<C>(tile, in + b * n3 * C, g.n, x0, y0, z0);
    else stage_x0(tile, delta + b * n3, up + b * n3, g, x0, y0, z0);
    for (int e = threadIdx.x; e < TPOS * CH / 4; e += 256) {
      const int p = e / (CH / 4), o4 = e % (CH / 4);
      const int pm = p % TX, py = (p / TX) % TY, pz = p / (TX * TY);
      const long long cell = b * n3 + ((long long)(z0 + pz) * g.n + (y0 + py)) * g.n + x0 + pm;
      const uint2 v = *(const uint2*)(dpre + cell * CH + 4 * o4);
      dt[4 * o4 + 0][p] = (unsigned short)(v.x & 0xFFFF);
      dt[4 * o4 + 1][p] = (unsigned short)(v.x >> 16);
      dt[4 * o4 + 2][p] = (unsigned short)(v.y & 0xFFFF);
      dt[4 * o4 + 3][p] = (unsigned short)(v.y >> 16);
    }
    __syncthreads();
    if (threadIdx.x < CH) {
      for (int p = 0; p < TPOS; ++p) bacc += from_bf16(dt[threadIdx.x][p]);
    }
#pragma unroll
    for (int kp = 0; kp < TPOS / 16; ++kp) {
      // A[o][k] = dpre[p = 16 kp + k][o]: lane row o = m, k = 4q..4q+3
      const s4 a = *(const s4*)(&dt[m][kp * 16 + 4 * q]);
      const int p0 = kp * 16 + 4 * q;
#pragma unroll
      for (int k = 0; k < TPW; ++k) {
        const int nt = wave + 4 * k;
        if (nt < NT) {
          // B[k][n] = x[p + d_t][i]: lane column n = m
          const int col = nt * 16 + m;
          int t = col / C;
          const int i = col % C;
          if (t > 26) t = 26;
          s4 bv;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int p = p0 + j;
            const int pm = p % TX, py = (p / TX) % TY, pz = p / (TX * TY);
            bv[j] = (short)tile[tap_cell(pz, py, pm, t) * C + i];
          }
          acc[k] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[k], 0, 0, 0);
        }
      }
    }
  }
  // D[o = 4q + r][col = m] for each column tile
  const long long blk = (long long)b * gridDim.x + blockIdx.x;
  float* pb = part + blk * (CH * (KP + 1));
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    const int nt = wave + 4 * k;
    if (nt < NT) {
#pragma unroll
      for (int r = 0; r < 4; ++r) pb[(4 * q + r) * (KP + 1) + nt * 16 + m] = acc[k][r];
    }
  }
  if (threadIdx.x < CH) pb[threadIdx.x * (KP + 1) + KP] = bacc;
}

// out[c] = sum over nb partial rows of in[row][c] (fixed order).
__global__ void __launch_bounds__(256) k_reduce_cols(const float* __restrict__ part, long long nb, int ncols,
                                                     float* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= ncols) return;
  double acc = 0.0;
  for (long long r = 0; r < nb; ++r) acc += (double)part[r * ncols + c];
  out[c] = (float)acc;
}

__global__ void __launch_bounds__(256) k_reduce_loss(const double* __restrict__ part, int nb, double* __restrict__ out) {
  double a = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) a += part[i];
  double t1, t2;
  block_sum2<256>(a, 0.0, &t1, &t2);
  if (threadIdx.x == 0) out[0] = t1;
}

// Weights in MFMA layouts: wk1 [16][K1P] (k = t*8 + i), wk2 [16][432] (k = t*16 + i),
// wk2t [16][432] with wk2t[i][t*16 + o] = W2[o][26 - t][i] (flipped taps, transposed
// channels: the data gradient as a forward convolution), w3 [432] as bf16-rounded FP32.
__global__ void __launch_bounds__(256) k_prep_weights(const float* __restrict__ th, unsigned short* __restrict__ wk2t,
                                                      float* __restrict__ w3) {
  // wk2t: layer-2 weights flipped and transposed for the data gradient, [16 in][27 x 16 out] bf16;
  // w3: layer-3 weights rounded to bf16 (FP32 storage) for the output-layer backward
  for (int e = blockIdx.x * 256 + threadIdx.x; e < CH * K2 + K2; e += gridDim.x * 256) {
    if (e < CH * K2) {
      const int i = e / K2, k = e % K2, t = k / CH, o = k % CH;
      wk2t[e] = to_bf16(th[OFF_W2 + (o * 27 + (26 - t)) * CH + i]);
    } else {
      w3[e - CH * K2] = from_bf16(to_bf16(th[OFF_W3 + e - CH * K2]));
    }
  }
}

// Gradient assembly from the reduced partials into the parameter layout.
__global__ void __launch_bounds__(256) k_assemble_grad(const float* __restrict__ g1, const float* __restrict__ g2,
                                                       const float* __restrict__ g3, float* __restrict__ grad) {
  for (int e = blockIdx.x * 256 + threadIdx.x; e < NPARAM; e += gridDim.x * 256) {
    float v;
    if (e < OFF_B1) { const int o = e / K1, k = e % K1; v = g1[o * (K1P + 1) + k]; }
    else if (e < OFF_W2) v = g1[(e - OFF_B1) * (K1P + 1) + K1P];
    else if (e < OFF_B2) { const int f = e - OFF_W2, o = f / K2, k = f % K2; v = g2[o * (K2 + 1) + k]; }
    else if (e < OFF_W3) v = g2[(e - OFF_B2) * (K2 + 1) + K2];
    else v = g3[e - OFF_W3];        // W3 (432) then b3 (entry 432)
    grad[e] = v;
  }
}

// Adam (Kingma & Ba 2015) with bias correction; step counts from 1.
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ grad, int n, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const float gr = grad[e];
    const float mm = b1 * m[e] + (1.f - b1) * gr;
    const float vv = b2 * v[e] + (1.f - b2) * gr * gr;
    m[e] = mm;
    v[e] = vv;
    th[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// u = Psi . r_hat from the displacement (planar [b][3][N^3]).
__global__ void __launch_bounds__(256) k_radial(const float* __restrict__ psi, Geo3 g, int batch,
                                                float* __restrict__ u) {
  const long long n3 = (long long)g.n * g.n * g.n;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n3 * batch; i += (long long)gridDim.x * 256) {
    const long long c = i % n3;
    const int x = (int)(c % g.n), y = (int)((c / g.n) % g.n), z = (int)(c / ((long long)g.n * g.n));
    const float rx = fmaf(g.hs, (float)x, g.ds[0]), ry = fmaf(g.hs, (float)y, g.ds[1]),
                rz = fmaf(g.hs, (float)z, g.ds[2]);
    const float r2 = rx * rx + ry * ry + rz * rz;
    const float ir = r2 > 0.f ? rsqrtf(r2) : 0.f;
    const float* p = psi + 3 * (i - c);
    u[i] = (rx * p[c] + ry * p[n3 + c] + rz * p[2 * n3 + c]) * ir;
  }
}

// Full-weighting restriction of periodic n^3 node fields to (n/2)^3: coarse node J sits on fine
// node 2J, weights 1/4, 1/2, 1/4 per axis on fine nodes 2J-1, 2J, 2J+1.  One thread per coarse
// node restricts NF fields, blockIdx.y = realisation.
template <int NF>
__global__ void __launch_bounds__(256) k_restrict(const float* __restrict__ fa, const float* __restrict__ fb, int n,
                                                  float* __restrict__ ca, float* __restrict__ cb) {
  const int m = n >> 1, msk = n - 1;
  const long long mc = (long long)m * m * m;
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= mc) return;
  const int X = (int)(i % m), Y = (int)((i / m) % m), Z = (int)(i / ((long long)m * m));
  const long long off = (long long)blockIdx.y * n * n * n;
  const float w[3] = {0.25f, 0.5f, 0.25f};
  float acc[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) acc[f] = 0.f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const long long z = (2 * Z + c - 1) & msk;
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
      const long long row = off + (z * n + ((2 * Y + bb - 1) & msk)) * n;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const float* src = f == 0 ? fa : fb;
        float r = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) r = fmaf(w[a], src[row + ((2 * X + a - 1) & msk)], r);
        acc[f] = fmaf(w[c] * w[bb], r, acc[f]);
      }
    }
  }
  const long long o = (long long)blockIdx.y * mc + i;
  ca[o] = acc[0];
  if (NF > 1) cb[o] = acc[NF - 1];
}

// The same restriction for n/2 >= 64: a block covers 64 (x) by 4 (y) coarse nodes and marches over
// 16 coarse z planes, so each fine z plane is filtered once in x and y and shared by the two coarse
// planes it feeds (the filtered plane 2Z+1 is carried in registers to the next coarse plane).
template <int NF>
__global__ void __launch_bounds__(256) k_restrict_slab(const float* __restrict__ fa, const float* __restrict__ fb, int n,
                                                       float* __restrict__ ca, float* __restrict__ cb) {
  constexpr int TXW = 64, TYH = 4, ZB = 16;
  const int m = n >> 1, msk = n - 1;
  const int nbx = m / TXW, nby = m / TYH;
  int t = blockIdx.x;
  const int X = (t % nbx) * TXW + (threadIdx.x % TXW);
  t /= nbx;
  const int Y = (t % nby) * TYH + threadIdx.x / TXW;
  const int Z0 = (t / nby) * ZB;
  const long long off = (long long)blockIdx.y * n * n * n, mc = (long long)m * m * m;
  const int xs0 = (2 * X - 1) & msk, xs1 = 2 * X, xs2 = 2 * X + 1;
  const int ys[3] = {(2 * Y - 1) & msk, 2 * Y, 2 * Y + 1};
  auto plane = [&](const float* __restrict__ f, int z) {
    float p = 0.f;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const float* r = f + off + ((long long)z * n + ys[b]) * n;
      const float v = fmaf(0.25f, r[xs0], fmaf(0.5f, r[xs1], 0.25f * r[xs2]));
      p = fmaf(b == 1 ? 0.5f : 0.25f, v, p);
    }
    return p;
  };
  float prev[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) prev[f] = plane(f == 0 ? fa : fb, (2 * Z0 - 1) & msk);
  for (int k = 0; k < ZB; ++k) {
    const int Z = Z0 + k;
    const long long o = (long long)blockIdx.y * mc + ((long long)Z * m + Y) * m + X;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const float* src = f == 0 ? fa : fb;
      const float p0 = plane(src, 2 * Z), p1 = plane(src, 2 * Z + 1);
      const float v = fmaf(0.25f, prev[f], fmaf(0.5f, p0, 0.25f * p1));
      prev[f] = p1;
      (f == 0 ? ca : cb)[o] = v;
    }
  }
}

// Linear prolongation of a periodic (n/2)^3 node field to n^3, times scale: fine node 2J copies
// coarse node J, fine node 2J+1 takes the mean of coarse J and J+1, axis by axis.  One thread per
// coarse node writes its 2 x 2 x 2 block of fine nodes.
__global__ void __launch_bounds__(256) k_prolong(const float* __restrict__ coarse, int n, float scale,
                                                 float* __restrict__ fine) {
  const int m = n >> 1, mm = m - 1;
  const long long mc = (long long)m * m * m;
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= mc) return;
  const int X = (int)(i % m), Y = (int)((i / m) % m), Z = (int)(i / ((long long)m * m));
  const float* c = coarse + (long long)blockIdx.y * mc;
  const int X1 = (X + 1) & mm, Y1 = (Y + 1) & mm, Z1 = (Z + 1) & mm;
  float v[2][2][2];                                   // [z][y][x] corners J, J+1
  const long long zr[2] = {(long long)Z * m, (long long)Z1 * m};
  const int yr[2] = {Y, Y1};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      const long long r = (zr[a] + yr[bb]) * m;
      v[a][bb][0] = c[r + X];
      v[a][bb][1] = c[r + X1];
    }
  // x, then y, then z halves
  float hx[2][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      hx[a][bb][0] = v[a][bb][0];
      hx[a][bb][1] = 0.5f * (v[a][bb][0] + v[a][bb][1]);
    }
  float hy[2][2][2];                                  // [z corner][ey][ex]
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int ex = 0; ex < 2; ++ex) {
      hy[a][0][ex] = hx[a][0][ex];
      hy[a][1][ex] = 0.5f * (hx[a][0][ex] + hx[a][1][ex]);
    }
  float* out = fine + (long long)blockIdx.y * n * n * n;
#pragma unroll
  for (int ez = 0; ez < 2; ++ez)
#pragma unroll
    for (int ey = 0; ey < 2; ++ey) {
      float o[2];
#pragma unroll
      for (int ex = 0; ex < 2; ++ex) o[ex] = scale * (ez ? 0.5f * (hy[0][ey][ex] + hy[1][ey][ex]) : hy[0][ey][ex]);
      const long long fi = (((long long)(2 * Z + ez) * n) + (2 * Y + ey)) * n + 2 * X;
      *(float2*)(out + fi) = make_float2(o[0], o[1]);
    }
}

// Linear prolongation twice = trilinear interpolation at four fine nodes per coarse cell: fine node
// 4J + q takes (1 - q/4) of coarse J and q/4 of coarse J+1 per axis (periodic), times scale.  One
// thread per coarse node writes its 4 x 4 x 4 block of fine nodes, one 16-byte row at a time.
__global__ void __launch_bounds__(256) k_prolong4(const float* __restrict__ coarse, int n, float scale,
                                                  float* __restrict__ fine) {
  const int m = n >> 2, mm = m - 1;
  const long long mc = (long long)m * m * m;
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= mc) return;
  const int X = (int)(i % m), Y = (int)((i / m) % m), Z = (int)(i / ((long long)m * m));
  const float* c = coarse + (long long)blockIdx.y * mc;
  const int X1 = (X + 1) & mm, Y1 = (Y + 1) & mm, Z1 = (Z + 1) & mm;
  float v[2][2][2];                                   // [z][y][x] corners J, J+1
  const long long zr[2] = {(long long)Z * m, (long long)Z1 * m};
  const int yr[2] = {Y, Y1};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      const long long r = (zr[a] + yr[bb]) * m;
      v[a][bb][0] = c[r + X];
      v[a][bb][1] = c[r + X1];
    }
  const float wq[4] = {0.f, 0.25f, 0.5f, 0.75f};
  float* out = fine + (long long)blockIdx.y * n * n * n;
#pragma unroll
  for (int qz = 0; qz < 4; ++qz)
#pragma unroll
    for (int qy = 0; qy < 4; ++qy) {
      float row[2];
#pragma unroll
      for (int ex = 0; ex < 2; ++ex) {
        const float y0 = fmaf(wq[qy], v[0][1][ex] - v[0][0][ex], v[0][0][ex]);
        const float y1 = fmaf(wq[qy], v[1][1][ex] - v[1][0][ex], v[1][0][ex]);
        row[ex] = fmaf(wq[qz], y1 - y0, y0);
      }
      float4 o;
      o.x = scale * row[0];
      o.y = scale * fmaf(0.25f, row[1] - row[0], row[0]);
      o.z = scale * fmaf(0.5f, row[1] - row[0], row[0]);
      o.w = scale * fmaf(0.75f, row[1] - row[0], row[0]);
      const long long fi = (((long long)(4 * Z + qz) * n) + (4 * Y + qy)) * n + 4 * X;
      *(float4*)(out + fi) = o;
    }
}

}  // namespace cnn
}  // namespace recon
