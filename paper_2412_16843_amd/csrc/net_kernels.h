// Learned pressure guess: encoder-decoder network (4 levels, 32/64/128/256
// channels, 3x3 convolutions) trained and evaluated with BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  Its output is only the
// initial guess of the pressure solve.
//
// Tensors are [batch][channel][row][column] (column fastest).  Activations
// and activation gradients are BF16; parameters, their gradients and the
// Adam moments are FP32 (master copy); the convolution weights are repacked
// to BF16 [co][tap][ci] for the matrix cores.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdinet {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;          // 4 waves
constexpr int TCO = 64;          // output-channel tile (16 per wave)
constexpr int TPX = 64;          // pixel tile along a row (4 MFMA column blocks)
constexpr int KC = 32;           // input channels per MFMA step

__device__ __forceinline__ float bf2f(__bf16 v) { return (float)v; }
__device__ __forceinline__ __bf16 f2bf(float v) { return (__bf16)v; }

// ------------------------------------------------------------------ conv 3x3
// y[b,o,i,j] = act(bias[o] + sum_{c,ky,kx} w[o,ky*3+kx,c] x[b,c,i+ky-1,j+kx-1])
// as an implicit GEMM: M = output channels, N = pixels, K = 32 input channels
// per step, 9 taps.  One block computes 64 output channels x 2 rows x 64
// columns; wave w owns output channels [16w, 16w+16) for both rows (8 MFMA
// accumulators), so each staged weight chunk serves 128 pixels.  Weights are
// staged with 16-byte loads; the 4 input rows of a chunk with 16-byte loads
// along x plus the two halo columns.  Zero padding outside the image.
// ci must be a multiple of 32.  relu: 0 none, 1 relu.
// Output either BF16 (yb) or FP32 (yf), whichever is non-null.
// A wave computes CF 16-channel fragments x CROWS rows x 64 columns, so each
// input fragment read from LDS feeds CF matrix-core products; WCH waves lie
// along the output channels and 4 / WCH along the rows (CF = 2: WCH = 1 for
// the 32-channel layers, a 32-channel x 8-row tile; WCH = 2 for the others,
// 64 channels x 4 rows).
constexpr int CROWS = 2;   // rows per wave
//
// First-layer form (xf != nullptr): the input is the 3 FP32 feature planes
// (ci = 32, channels 3..31 zero), rounded to BF16 on staging.
// Decoder form (xlo != nullptr): the input is cat(up2(xlo), x) without being
// stored -- channels [0, clo) are read from xlo (B x clo x H/2 x W/2) at
// (row/2, col/2), channels [clo, ci) from x (B x (ci-clo) x H x W); clo is a
// multiple of 32, so each 32-channel step reads one of the two.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
template <int CF, int WCH>
__global__ void __launch_bounds__(NT) k_conv3_fwd(const __bf16* __restrict__ x,
                                                  const __bf16* __restrict__ wp,
                                                  const float* __restrict__ bias,
                                                  __bf16* __restrict__ yb, float* __restrict__ yf,
                                                  int B, int ci, int co, int H, int W, int relu,
                                                  const __bf16* __restrict__ xlo = nullptr,
                                                  int clo = 0,
                                                  const float* __restrict__ xf = nullptr,
                                                  const float* __restrict__ ow = nullptr,
                                                  const float* __restrict__ ob = nullptr,
                                                  float* __restrict__ yo = nullptr) {
  constexpr int TC = 16 * CF * WCH;                  // output channels of the tile
  constexpr int ROWS = CROWS * (4 / WCH);            // output rows of the tile
  constexpr int XR = ROWS + 2;                       // staged input rows
  // LDS pitch of one pixel's (or one (o, tap)'s) 32 channels: 40 BF16 = 80
  // bytes keeps every 8-channel vector 16-byte aligned and spreads 16
  // consecutive pixels over 16 banks (a 64-byte pitch hits 4)
  constexpr int KP = KC + 8;
  __shared__ __attribute__((aligned(16))) __bf16 s_x[XR * (TPX + 2) * KP];   // [row][px][c]
  __shared__ __attribute__((aligned(16))) __bf16 s_w[TC * 9 * KP];           // [o][tap][c]
  const int nxt = (W + TPX - 1) / TPX;
  const int nyt = (H + ROWS - 1) / ROWS;
  int blk = blockIdx.x;
  const int xt = blk % nxt; blk /= nxt;
  const int row0 = (blk % nyt) * ROWS; blk /= nyt;
  const int b = blk;
  const int co0 = blockIdx.y * TC;
  const int x0 = xt * TPX;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wco = wv % WCH;                          // channel group of this wave
  const int wr0 = (wv / WCH) * CROWS;                // first tile row of this wave
  f32x4 acc[CF][CROWS][4];
#pragma unroll
  for (int f = 0; f < CF; ++f)
#pragma unroll
    for (int r = 0; r < CROWS; ++r)
#pragma unroll
      for (int n = 0; n < 4; ++n) acc[f][r][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  const size_t plane = (size_t)H * W;
  const int kq = 8 * (lane >> 4);
  const int li = lane & 15;
  const int hh = H / 2, wh = W / 2;
  const size_t plane_lo = (size_t)hh * wh;
  const int cskip = ci - clo;
  for (int c0 = 0; c0 < ci; c0 += KC) {
    const bool lo = xlo != nullptr && c0 < clo;   // this step reads the upsampled tensor
    // input rows row0-1 .. row0+ROWS, the 64-column core: a thread gathers
    // 8 channels of one pixel (each load coalesced along the pixels of the
    // wave) and stores them as one 16-byte vector
    for (int e = tid; e < (KC / 8) * XR * TPX; e += NT) {
      const int px = e % TPX;
      const int r = (e / TPX) % XR;
      const int c8 = e / (TPX * XR);
      const int yy = row0 + r - 1, xx = x0 + px;
      bf16x8 v;
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = f2bf(0.f);
      if (yy >= 0 && yy < H && xx < W) {
        if (xf) {   // first layer: 3 FP32 feature planes, the other channels 0
#pragma unroll
          for (int q = 0; q < 3; ++q)
            if (8 * c8 + q < 3) v[q] = f2bf(xf[((size_t)b * 3 + 8 * c8 + q) * plane + (size_t)yy * W + xx]);
        } else if (lo) {
          const __bf16* src = &xlo[((size_t)b * clo + c0 + 8 * c8) * plane_lo + (size_t)(yy >> 1) * wh + (xx >> 1)];
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = src[(size_t)q * plane_lo];
        } else {
          const __bf16* src = xlo != nullptr
              ? &x[((size_t)b * cskip + (c0 - clo) + 8 * c8) * plane + (size_t)yy * W + xx]
              : &x[((size_t)b * ci + c0 + 8 * c8) * plane + (size_t)yy * W + xx];
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = src[(size_t)q * plane];
        }
      }
      *(bf16x8*)&s_x[(r * (TPX + 2) + 1 + px) * KP + 8 * c8] = v;
    }
    // the two halo columns x0-1 and x0+TPX
    for (int e = tid; e < KC * XR * 2; e += NT) {
      const int side = e & 1;
      const int r = (e >> 1) % XR;
      const int c = e / (2 * XR);
      const int yy = row0 + r - 1, xx = side ? x0 + TPX : x0 - 1;
      __bf16 v = f2bf(0.f);
      if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
        if (xf) v = c < 3 ? f2bf(xf[((size_t)b * 3 + c) * plane + (size_t)yy * W + xx]) : f2bf(0.f);
        else if (lo) v = xlo[((size_t)b * clo + c0 + c) * plane_lo + (size_t)(yy >> 1) * wh + (xx >> 1)];
        else if (xlo != nullptr) v = x[((size_t)b * cskip + (c0 - clo) + c) * plane + (size_t)yy * W + xx];
        else v = x[((size_t)b * ci + c0 + c) * plane + (size_t)yy * W + xx];
      }
      s_x[(r * (TPX + 2) + (side ? TPX + 1 : 0)) * KP + c] = v;
    }
    // weights of the tile: 4 vectors of 8 input channels per (o, tap)
    for (int e = tid; e < TC * 9 * (KC / 8); e += NT) {
      const int v8 = e % (KC / 8);
      const int ot = e / (KC / 8);           // o * 9 + tap
      const int o = ot / 9;
      bf16x8 v;
      if (co0 + o < co) {
        v = *(const bf16x8*)&wp[((size_t)(co0 * 9) + ot) * ci + c0 + 8 * v8];
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = f2bf(0.f);
      }
      *(bf16x8*)&s_w[ot * KP + 8 * v8] = v;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int ky = t / 3, kx = t - 3 * ky;
      bf16x8 a[CF];
#pragma unroll
      for (int f = 0; f < CF; ++f)
        a[f] = *(const bf16x8*)&s_w[((16 * (wco * CF + f) + li) * 9 + t) * KP + kq];
#pragma unroll
      for (int r = 0; r < CROWS; ++r)
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          const bf16x8 bv = *(const bf16x8*)&s_x[((wr0 + r + ky) * (TPX + 2) + 16 * n + li + kx) * KP + kq];
#pragma unroll
          for (int f = 0; f < CF; ++f)
            acc[f][r][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f], bv, acc[f][r][n], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  // epilogue: lane holds rows 4(lane/16)+q (output channels), column lane%16
#pragma unroll
  for (int f = 0; f < CF; ++f)
#pragma unroll
  for (int r = 0; r < CROWS; ++r) {
    const int row = row0 + wr0 + r;
    if (row >= H) continue;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int px = x0 + 16 * n + (lane & 15);
      if (px >= W) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = co0 + 16 * (wco * CF + f) + 4 * (lane >> 4) + q;
        if (o >= co) continue;
        float v = acc[f][r][n][q] + (bias ? bias[o] : 0.f);
        if (relu) v = fmaxf(v, 0.f);
        const size_t idx = ((size_t)b * co + o) * plane + (size_t)row * W + px;
        if (yb) yb[idx] = f2bf(v);
        else if (yf) yf[idx] = v;
      }
    }
  }
  // Fused 1x1 output layer (yo != nullptr; a 32-channel tile, WCH = 1, so a
  // wave holds all 32 channels of its pixels): y = ob + sum_o ow[o] v_o with
  // v_o the BF16-rounded activation.  Each lane adds its 2 x 4 channels, then
  // the four lane groups (lane / 16) are added by two xor exchanges (every
  // lane ends with the same bits: each exchange adds the same two values).
  if (yo) {
#pragma unroll
    for (int r = 0; r < CROWS; ++r)
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        float sum = 0.f;
#pragma unroll
        for (int f = 0; f < CF; ++f)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int o = 16 * (wco * CF + f) + 4 * (lane >> 4) + q;
            float v = acc[f][r][n][q] + (bias ? bias[co0 + o] : 0.f);
            if (relu) v = fmaxf(v, 0.f);
            sum += ow[o] * bf2f(f2bf(v));
          }
        sum += __shfl_xor(sum, 16, 64);
        sum += __shfl_xor(sum, 32, 64);
        const int row = row0 + wr0 + r, px = x0 + 16 * n + (lane & 15);
        if (lane < 16 && row < H && px < W) yo[(size_t)b * plane + (size_t)row * W + px] = ob[0] + sum;
      }
  }
}

// ------------------------------------------------------- weight gradient
// dw[o,c,tap] partial sums over the pixels of one chunk of rows:
// sum_{i,j} dy[b,o,i,j] x[b,c,i+ky-1,j+kx-1] as GEMM M = o, N = c, K = 32
// pixels per step.  Grid: (co/64, ci/32, chunks); chunk = (sample, rows
// [r0, r0+rows)).  Partial results go to part[chunk][o][c][tap] (FP32).
__global__ void __launch_bounds__(NT) k_conv3_wgrad(const __bf16* __restrict__ x,
                                                    const __bf16* __restrict__ dy,
                                                    float* __restrict__ part, int B, int ci,
                                                    int co, int H, int W, int rows,
                                                    int chunks_per_b) {
  __shared__ __attribute__((aligned(16))) __bf16 s_dy[TCO * TPX];             // [o][px]
  __shared__ __attribute__((aligned(16))) __bf16 s_x[KC * 3 * (TPX + 2 + 6)]; // [c][row][px]
  constexpr int XP = TPX + 8;   // padded row pitch (16-byte aligned reads at any shift)
  const int co0 = blockIdx.x * TCO, c0 = blockIdx.y * KC;
  // blockIdx.z = b * chunks_per_b + chunk; chunk k covers rows k*rows .. ; the
  // chunks past the last row (chunks_per_b * rows may exceed H) add nothing
  const int b = blockIdx.z / chunks_per_b;
  const int r0 = (blockIdx.z % chunks_per_b) * rows;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, kq = 8 * (lane >> 4);
  f32x4 acc[2][9];
#pragma unroll
  for (int n = 0; n < 2; ++n)
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[n][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const size_t plane = (size_t)H * W;
  for (int row = r0; row < r0 + rows && row < H; ++row) {
    for (int x0 = 0; x0 < W; x0 += TPX) {
      for (int e = tid; e < TCO * TPX; e += NT) {
        const int px = e % TPX, o = e / TPX;
        __bf16 v = f2bf(0.f);
        if (co0 + o < co && x0 + px < W) v = dy[((size_t)b * co + co0 + o) * plane + (size_t)row * W + x0 + px];
        s_dy[e] = v;
      }
      // x: columns x0-1 .. x0+TPX stored at px index 0..TPX+1 (pitch XP)
      for (int e = tid; e < KC * 3 * XP; e += NT) {
        const int px = e % XP;
        const int r = (e / XP) % 3;
        const int c = e / (3 * XP);
        const int yy = row + r - 1, xx = x0 + px - 1;
        __bf16 v = f2bf(0.f);
        if (px < TPX + 2 && yy >= 0 && yy < H && xx >= 0 && xx < W)
          v = x[((size_t)b * ci + c0 + c) * plane + (size_t)yy * W + xx];
        s_x[e] = v;
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < TPX / 32; ++ks) {
        // A: dy[o = 16 wv + li][px = 32 ks + kq .. +8]
        const bf16x8 a = *(const bf16x8*)&s_dy[(16 * wv + li) * TPX + 32 * ks + kq];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          const int ky = t / 3, kx = t - 3 * ky;
#pragma unroll
          for (int n = 0; n < 2; ++n) {
            // B: x[c = 16 n + li][shifted px = 32 ks + kq + kx .. +8] (element-wise gather:
            // the shift by kx breaks 16-byte alignment)
            bf16x8 bv;
            const __bf16* src = &s_x[((16 * n + li) * 3 + ky) * XP + 32 * ks + kq + kx];
#pragma unroll
            for (int q = 0; q < 8; ++q) bv[q] = src[q];
            acc[n][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc[n][t], 0, 0, 0);
          }
        }
      }
      __syncthreads();
    }
  }
  // D: rows (o) 4(lane/16)+q, column (c) lane%16
  float* out = part + (size_t)blockIdx.z * co * ci * 9;
#pragma unroll
  for (int n = 0; n < 2; ++n)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int o = co0 + 16 * wv + 4 * (lane >> 4) + q;
      const int c = c0 + 16 * n + li;
      if (o >= co) continue;
#pragma unroll
      for (int t = 0; t < 9; ++t) out[((size_t)o * ci + c) * 9 + t] = acc[n][t][q];
    }
}

// Sum of the chunk partials (fixed order) into the FP32 gradient of the
// weights in the master layout [o][c][3][3], and the bias gradient.
__global__ void k_wgrad_reduce(const float* __restrict__ part, int chunks, int co, int ci,
                               int ci_used, float* __restrict__ gw) {
  const int n = co * ci_used * 9;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int t = e % 9, c = (e / 9) % ci_used, o = e / (9 * ci_used);
    float s = 0.f;
    for (int k = 0; k < chunks; ++k) s += part[((size_t)k * co * ci + (size_t)o * ci + c) * 9 + t];
    gw[e] = s;
  }
}

// Bias gradient: sum over batch and pixels of dy[b,o,:,:] (one block per o).
__global__ void __launch_bounds__(NT) k_bias_grad(const __bf16* __restrict__ dy, int B, int co,
                                                  int HW, float* __restrict__ gb) {
  __shared__ float sh[NT];
  const int o = blockIdx.x;
  float s = 0.f;
  for (int b = 0; b < B; ++b)
    for (int p = threadIdx.x; p < HW; p += NT) s += bf2f(dy[((size_t)b * co + o) * HW + p]);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) gb[o] = sh[0];
}

// --------------------------------------------------------- weight packing
// Master [o][c][3][3] (c < ci_used) -> BF16 [o][tap][c] with c padded to ci.
// transpose != 0: the backward-data operator, BF16 [c][tap'][o] with the
// taps rotated by 180 degrees (so that the forward kernel computes the
// adjoint convolution).
__global__ void k_pack_w(const float* __restrict__ w, int co, int ci_used, int ci,
                         __bf16* __restrict__ wp, int transpose) {
  const int n = co * 9 * ci;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    if (!transpose) {
      const int c = e % ci, t = (e / ci) % 9, o = e / (9 * ci);
      wp[e] = f2bf(c < ci_used ? w[((size_t)o * ci_used + c) * 9 + t] : 0.f);
    } else {
      // wp layout [c][t'][o] with o fastest, size ci * 9 * co
      const int o = e % co, t = (e / co) % 9, c = e / (9 * co);
      wp[e] = f2bf(c < ci_used ? w[((size_t)o * ci_used + c) * 9 + (8 - t)] : 0.f);
    }
  }
}

// ------------------------------------------------------------- elementwise
// 2x2 mean pooling
__global__ void k_pool(const __bf16* __restrict__ x, __bf16* __restrict__ y, int BC, int H, int W) {
  const int h = H / 2, w = W / 2;
  const size_t n = (size_t)BC * h * w;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int j = e % w, i = (e / w) % h;
    const size_t bc = e / ((size_t)w * h);
    const __bf16* s = x + bc * H * W + (size_t)(2 * i) * W + 2 * j;
    y[e] = f2bf(0.25f * (bf2f(s[0]) + bf2f(s[1]) + bf2f(s[W]) + bf2f(s[W + 1])));
  }
}

// y[b] = cat(up2(lo[b]) (clo channels), skip[b] (cs channels)) at H x W
__global__ void k_upcat(const __bf16* __restrict__ lo, const __bf16* __restrict__ skip,
                        __bf16* __restrict__ y, int B, int clo, int cs, int H, int W) {
  // one output row (b, c, i) per loop step of a block; columns across threads
  const int C = clo + cs;
  const int nrows = B * C * H;
  for (int row = blockIdx.x; row < nrows; row += gridDim.x) {
    const int i = row % H, bc = row / H;
    const int c = bc % C, b = bc / C;
    __bf16* out = y + (size_t)row * W;
    if (c < clo) {
      const __bf16* src = lo + (((size_t)b * clo + c) * (H / 2) + i / 2) * (W / 2);
      for (int j = threadIdx.x; j < W; j += blockDim.x) out[j] = src[j >> 1];
    } else {
      const __bf16* src = skip + (((size_t)b * cs + (c - clo)) * H + i) * W;
      for (int j = threadIdx.x; j < W; j += blockDim.x) out[j] = src[j];
    }
  }
}

// Backward of cat(up2(lo), skip): dlo = sum of the 2x2 block of the first
// clo channels; dskip_out = dcat[clo:] (+ pool_backward(dpool) when given:
// the skip tensor also fed the next level's pooling).
__global__ void k_upcat_bwd_lo(const __bf16* __restrict__ dcat, __bf16* __restrict__ dlo, int B,
                               int clo, int C, int H, int W) {
  const int h = H / 2, w = W / 2;
  const size_t n = (size_t)B * clo * h * w;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int j = e % w, i = (e / w) % h;
    const int c = (e / ((size_t)w * h)) % clo;
    const int b = e / ((size_t)w * h * clo);
    const __bf16* s = dcat + (((size_t)b * C + c) * H + 2 * i) * W + 2 * j;
    dlo[e] = f2bf(bf2f(s[0]) + bf2f(s[1]) + bf2f(s[W]) + bf2f(s[W + 1]));
  }
}

// dskip[b,c,i,j] = dcat[b, clo+c, i, j] + dpool[b,c,i/2,j/2] / 4
__global__ void k_skip_grad(const __bf16* __restrict__ dcat, const __bf16* __restrict__ dpool,
                            __bf16* __restrict__ dskip, int B, int clo, int cs, int H, int W) {
  const int C = clo + cs;
  const size_t n = (size_t)B * cs * H * W;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int j = e % W, i = (e / W) % H;
    const int c = (e / ((size_t)W * H)) % cs;
    const int b = e / ((size_t)W * H * cs);
    float v = bf2f(dcat[(((size_t)b * C + clo + c) * H + i) * W + j]);
    if (dpool) v += 0.25f * bf2f(dpool[(((size_t)b * cs + c) * (H / 2) + i / 2) * (W / 2) + j / 2]);
    dskip[e] = f2bf(v);
  }
}

// d(pre-activation) = d(post) * (post > 0), in place on a BF16 gradient
__global__ void k_relu_bwd(__bf16* __restrict__ g, const __bf16* __restrict__ y, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    if (!(bf2f(y[e]) > 0.f)) g[e] = f2bf(0.f);
}

// Loss gradient dy = 2 (y - t) / N and the output layer's backward:
// dd0[b,c,p] = w[c] dy[b,p] (BF16); per-block partials of dw[c], db, loss.
__global__ void __launch_bounds__(NT) k_out_bwd(const __bf16* __restrict__ d0,
                                                const float* __restrict__ w,
                                                const float* __restrict__ y,
                                                const float* __restrict__ t,
                                                __bf16* __restrict__ dd0,
                                                float* __restrict__ part /* [blocks][C+2] */,
                                                int B, int C, int HW) {
  __shared__ float sh[NT];
  const size_t n = (size_t)B * HW;
  const float inv_n = 1.f / (float)n;
  float acc[34];
  for (int c = 0; c < C + 2; ++c) acc[c] = 0.f;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int p = e % HW;
    const int b = e / HW;
    const float diff = y[e] - t[e];
    const float dyv = 2.f * diff * inv_n;
    for (int c = 0; c < C; ++c) {
      const size_t idx = ((size_t)b * C + c) * HW + p;
      acc[c] += dyv * bf2f(d0[idx]);
      dd0[idx] = f2bf(w[c] * dyv);
    }
    acc[C] += dyv;
    acc[C + 1] += diff * diff * inv_n;
  }
  for (int c = 0; c < C + 2; ++c) {
    sh[threadIdx.x] = acc[c];
    __syncthreads();
    for (int st = NT / 2; st > 0; st >>= 1) {
      if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * (C + 2) + c] = sh[0];
    __syncthreads();
  }
}

__global__ void k_out_reduce(const float* __restrict__ part, int blocks, int C,
                             float* __restrict__ gw, float* __restrict__ gb, float* __restrict__ loss) {
  const int c = threadIdx.x;
  if (c >= C + 2) return;
  float s = 0.f;
  for (int k = 0; k < blocks; ++k) s += part[(size_t)k * (C + 2) + c];
  if (c < C) gw[c] = s;
  else if (c == C) gb[0] = s;
  else loss[0] = s;
}

// Adam (bias-corrected) on the FP32 master parameters.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// Input features (FP32 [B][3][H][W]) -> BF16 [B][32][H][W], channels 3..31 zero.
__global__ void k_pack_input(const float* __restrict__ f, __bf16* __restrict__ x, int B, int HW,
                             int cpad) {
  const size_t n = (size_t)B * cpad * HW;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int p = e % HW;
    const int c = (e / HW) % cpad;
    const int b = e / ((size_t)HW * cpad);
    x[e] = f2bf(c < 3 ? f[((size_t)b * 3 + c) * HW + p] : 0.f);
  }
}

}  // namespace cdinet
