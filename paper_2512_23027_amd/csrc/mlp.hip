// Learned initial guess: the MLP, its training (Adam) and inference kernels.
// Matrix products run on MFMA (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32
// accumulation); the hidden activations are kept in BF16, the precision the
// products read them in; everything else is FP32 elementwise or reduction
// work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "mlp.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16;  // BF16 bits

// FP32 -> BF16, round to nearest even (finite inputs).
__host__ __device__ inline unsigned short f2bf(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(bf16 h) { return __uint_as_float((uint32_t)h << 16); }
__device__ inline short ld_bf(const float* p) { return (short)f2bf(*p); }
__device__ inline short ld_bf(const bf16* p) { return (short)*p; }
__device__ inline float ld_f(const float* p) { return *p; }
__device__ inline float ld_f(const bf16* p) { return bf2f(*p); }
__device__ inline void st_c(float* p, float x) { *p = x; }
__device__ inline void st_c(bf16* p, float x) { *p = f2bf(x); }
// eight FP32 values -> eight BF16 (round to nearest even)
__device__ inline bf16x8 to_bf8(f32x8 f) { return __builtin_convertvector(f, bf16x8); }

// ---------------------------------------------------------------------------
// Fallback GEMM for contraction lengths above 256 (hidden widths above 256):
// C[i][j] = epilogue(sum_k A(i,k) B(k,j)) with A(i,k) = A[i*sai + k*sak] and
// B(k,j) = B[k*sbk + j*sbj] (BF16 weights).  Epilogue: + bias[j] (if bias),
// ReLU (if relu), times [gate[i][j] > 0] (if gate, BF16, leading dimension
// ldc).  A workgroup = 4 waves = a 32x32 tile of C, one 16x16 tile per wave;
// each lane loads its 4-value slices of A and B for every 16-wide k step
// (lane l: A rows l%16, B columns l%16, k = 4*(l/16) .. +3), out-of-range
// entries read as zero.  Result of the MFMA: lane l holds rows 4*(l/16) ..
// +3 of column l%16.
template <typename TA, typename TC>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const TA* __restrict__ A,
                                              long long sai, long long sak,
                                              const bf16* __restrict__ B, long long sbk,
                                              long long sbj, TC* __restrict__ C, int ldc,
                                              const float* __restrict__ bias, int relu,
                                              const bf16* __restrict__ gate) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int i0 = (blockIdx.y * 2 + (w >> 1)) * 16, j0 = (blockIdx.x * 2 + (w & 1)) * 16;
  if (i0 >= M || j0 >= N) return;  // uniform per wave
  const int ai = i0 + (l & 15), bj = j0 + (l & 15), kq = (l >> 4) * 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = k0 + kq + v;
      a[v] = (ai < M && k < K) ? ld_bf(A + ai * sai + k * sak) : (short)0;
      b[v] = (bj < N && k < K) ? ld_bf(B + k * sbk + bj * sbj) : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  const int j = j0 + (l & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + 4 * (l >> 4) + v;
    if (i >= M || j >= N) continue;
    float x = acc[v];
    if (bias) x += bias[j];
    if (relu) x = fmaxf(x, 0.f);
    if (gate && !(bf2f(gate[(size_t)i * ldc + j]) > 0.f)) x = 0.f;
    st_c(C + (size_t)i * ldc + j, x);
  }
}

// ---------------------------------------------------------------------------
// Dense layer with the weight panel resident in LDS (contraction length
// K <= 32*KS <= 256):
//   C[i][j] = epilogue(sum_k A[i][k] W(k,j)),  A row-major [M][K] (FP32 or
//   BF16), W(k,j) = W[k*sbk + j*sbj] (BF16), C row-major with leading
//   dimension ldc (FP32 or BF16); epilogue as in k_gemm.
// blockIdx.y picks a panel of NB output columns; the workgroup (NT/64 waves)
// stages W(k, panel) transposed, Wt[j][k], in LDS once (rows padded to
// 32*KS + 8 values so that the 16-byte fragment reads of 16 lanes hit
// distinct banks) with the panel's bias behind it, then each wave walks
// 16-row tiles of A: the tile's BF16 fragments for all k sit in registers
// (lane l: row l%16, k = 32 s + 8 (l/16) .. +7 of k step s) while the next
// tile's are loaded, and are contracted with the panel's 16-column tiles,
// four at a time with independent accumulators, by v_mfma_f32_16x16x32_bf16
// with the weight tile as the first operand, so the accumulator of lane l
// holds output row l%16, columns 4 (l/16) .. +3: four adjacent values,
// stored with one vector store.
// wmode: how the panel is staged: 1 = 16-byte loads along k (sbk == 1),
// 2 = 16-byte loads along j (sbj == 1), 0 = element by element.
template <typename TA>
struct RawA {  // one k step of a lane's A fragment as loaded
  typedef f32x8 T;
};
template <>
struct RawA<bf16> {
  typedef u32x4 T;
};

template <int KS, typename TA>
__device__ inline void load_a(typename RawA<TA>::T (&r)[KS], const TA* __restrict__ row,
                              bool valid, int K, int vecA, int lq) {
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k0 = 32 * s + 8 * lq;
    if constexpr (sizeof(TA) == 4) {
      f32x8 f = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (valid) {
        if (vecA && k0 + 8 <= K) {
          const float4 lo = *reinterpret_cast<const float4*>(row + k0);
          const float4 hi = *reinterpret_cast<const float4*>(row + k0 + 4);
          f = f32x8{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (k0 + u < K) f[u] = row[k0 + u];
        }
      }
      r[s] = f;
    } else {
      u32x4 q = {0u, 0u, 0u, 0u};
      if (valid) {
        if (vecA && k0 + 8 <= K) {
          const uint4 v = *reinterpret_cast<const uint4*>(row + k0);
          q = u32x4{v.x, v.y, v.z, v.w};
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (k0 + u < K) q[u >> 1] |= (uint32_t)row[k0 + u] << (16 * (u & 1));
        }
      }
      r[s] = q;
    }
  }
}

template <int KS, typename TA>
__device__ inline void to_frag(const typename RawA<TA>::T (&r)[KS], bf16x8 (&a)[KS]) {
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    if constexpr (sizeof(TA) == 4) a[s] = to_bf8(r[s]);
    else a[s] = __builtin_bit_cast(bf16x8, r[s]);
  }
}

template <int KS, typename TA, typename TC, int NT>
__global__ __launch_bounds__(NT) void k_dense(int M, int N, int K, const TA* __restrict__ A,
                                               int vecA, const bf16* __restrict__ W,
                                               long long sbk, long long sbj, int wmode,
                                               TC* __restrict__ C, int ldc, int vecC,
                                               const float* __restrict__ bias, int relu,
                                               const bf16* __restrict__ gate, int vg, int NB) {
  extern __shared__ __align__(16) bf16 wt[];
  constexpr int KP = 32 * KS, S = KP + 8, U = 8;
  const int jb = blockIdx.y * NB;
  const int nbc = min(NB, N - jb);          // columns of this panel
  const int ncp = (nbc + 15) & ~15;         // ... in whole 16-column tiles
  float* bs = reinterpret_cast<float*>(wt + (size_t)((min(NB, N) + 15) & ~15) * S);
  // stage the panel, U 16-byte loads in flight per thread
  if (wmode == 1) {
    constexpr int KV = KP / 8;
    const int n = ncp * KV;
    for (int e0 = threadIdx.x; e0 < n; e0 += NT * U) {
      uint4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + NT * u, j = e / KV, k = (e % KV) * 8;
        v[u] = uint4{0u, 0u, 0u, 0u};
        if (e < n && j < nbc && k < K)
          v[u] = *reinterpret_cast<const uint4*>(W + k + (size_t)(jb + j) * sbj);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + NT * u;
        if (e < n) *reinterpret_cast<uint4*>(wt + (e / KV) * S + (e % KV) * 8) = v[u];
      }
    }
  } else if (wmode == 2) {
    const int jv = ncp / 8, n = KP * jv;
    for (int e0 = threadIdx.x; e0 < n; e0 += NT * U) {
      uint4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + NT * u, k = e / jv, j = (e % jv) * 8;
        v[u] = uint4{0u, 0u, 0u, 0u};
        if (e < n && j < nbc && k < K)
          v[u] = *reinterpret_cast<const uint4*>(W + (size_t)k * sbk + jb + j);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + NT * u, k = e / jv, j = (e % jv) * 8;
        if (e >= n) continue;
        const uint32_t q[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
        for (int h = 0; h < 8; ++h) wt[(j + h) * S + k] = (bf16)(q[h >> 1] >> (16 * (h & 1)));
      }
    }
  } else {
    const int n = ncp * KP;
    for (int e0 = threadIdx.x; e0 < n; e0 += NT * U) {
      bf16 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + NT * u, j = e / KP, k = e % KP;
        v[u] = (e < n && j < nbc && k < K) ? W[(size_t)k * sbk + (size_t)(jb + j) * sbj] : (bf16)0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + NT * u;
        if (e < n) wt[(e / KP) * S + e % KP] = v[u];
      }
    }
  }
  for (int j = threadIdx.x; j < ncp; j += NT) bs[j] = (bias && j < nbc) ? bias[jb + j] : 0.f;
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  const int ntm = (M + 15) / 16, nct = ncp / 16, stride = gridDim.x * (NT / 64);
  int tm = blockIdx.x * (NT / 64) + w;  // uniform per wave
  typename RawA<TA>::T raw[KS];
  if (tm < ntm) load_a<KS, TA>(raw, A + (size_t)(tm * 16 + lr) * K, tm * 16 + lr < M, K, vecA, lq);
  for (; tm < ntm; tm += stride) {
    bf16x8 a[KS];
    to_frag<KS, TA>(raw, a);
    const int i = tm * 16 + lr;
    const int tn = tm + stride;
    if (tn < ntm) load_a<KS, TA>(raw, A + (size_t)(tn * 16 + lr) * K, tn * 16 + lr < M, K, vecA, lq);
    for (int jt = 0; jt < nct; jt += 4) {
      uint2 gv[4];  // gate values of the four tiles (BF16 pairs)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        gv[u] = uint2{0u, 0u};
        const int j = jb + 4 * lq + 16 * (jt + u);
        if (vg && i < M && j + 4 <= N)
          gv[u] = *reinterpret_cast<const uint2*>(gate + (size_t)i * ldc + j);
      }
      f32x4 acc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (jt + u >= nct) continue;
          const bf16x8 b =
              *reinterpret_cast<const bf16x8*>(wt + ((jt + u) * 16 + lr) * S + 32 * s + 8 * lq);
          acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a[s], acc[u], 0, 0, 0);
        }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int jl = 16 * (jt + u) + 4 * lq, j = jb + jl;  // panel column, output column
        if (jt + u >= nct || i >= M || j >= N) continue;
        float x[4] = {acc[u][0], acc[u][1], acc[u][2], acc[u][3]};
        const bool full = j + 4 <= N;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          x[v] += bs[jl + v];
          if (relu) x[v] = fmaxf(x[v], 0.f);
          if (gate) {
            const bf16 gh = (vg && full) ? (bf16)((v < 2 ? gv[u].x : gv[u].y) >> (16 * (v & 1)))
                            : (j + v < N ? gate[(size_t)i * ldc + j + v] : (bf16)0);
            if (!(bf2f(gh) > 0.f)) x[v] = 0.f;
          }
        }
        TC* out = C + (size_t)i * ldc + j;
        if (vecC && full) {
          if constexpr (sizeof(TC) == 4) {
            *reinterpret_cast<float4*>(out) = float4{x[0], x[1], x[2], x[3]};
          } else {
            *reinterpret_cast<uint2*>(out) =
                uint2{(uint32_t)f2bf(x[0]) | ((uint32_t)f2bf(x[1]) << 16),
                      (uint32_t)f2bf(x[2]) | ((uint32_t)f2bf(x[3]) << 16)};
          }
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (j + v < N) st_c(out + v, x[v]);
        }
      }
    }
  }
}

constexpr int kDenseLds = 160 * 1024;  // LDS of one CU

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <int KS, typename TA, typename TC>
void dense_launch(int M, int N, int K, const TA* A, const bf16* W, long long sbk, long long sbj,
                  TC* C, int ldc, const float* bias, int relu, const bf16* gate, hipStream_t st) {
  constexpr int KP = 32 * KS, S = KP + 8;
  const int ncmax = (kDenseLds / (2 * S + 4)) & ~15;
  const int NB = std::min((N + 15) & ~15, ncmax);
  const int ny = (N + NB - 1) / NB;
  const int ncp0 = (std::min(NB, N) + 15) & ~15;
  const int lds = ncp0 * S * 2 + ncp0 * 4;  // panel, then its bias
  int wmode = 0;
  if (sbk == 1 && K % 8 == 0 && sbj % 8 == 0 && aligned16(W)) wmode = 1;
  else if (sbj == 1 && N % 8 == 0 && sbk % 8 == 0 && aligned16(W)) wmode = 2;
  const int vecA = K % 8 == 0 && aligned16(A);
  const int vecC = ldc % 4 == 0 && (reinterpret_cast<uintptr_t>(C) % (4 * sizeof(TC))) == 0;
  const int per_cu = std::max(1, std::min(4, kDenseLds / std::max(lds, 1)));
  const int ntm = (M + 15) / 16;
  // 16 waves a workgroup where the registers stay within 128 a lane (BF16
  // operands, or FP32 ones with K <= 128), else 8
  constexpr int NT = (sizeof(TA) == 2 || KS <= 4) ? 1024 : 512, NW = NT / 64;
  const int nx = std::max(1, std::min((ntm + NW - 1) / NW, 256 * per_cu / ny));
  auto* f = &k_dense<KS, TA, TC, NT>;
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  const int vg = gate && ldc % 4 == 0 && reinterpret_cast<uintptr_t>(gate) % 8 == 0;
  f<<<dim3(nx, ny), NT, lds, st>>>(M, N, K, A, vecA, W, sbk, sbj, wmode, C, ldc, vecC, bias, relu,
                                    gate, vg, NB);
}

// C = epilogue(A W) for A row-major [M][K]; the dense kernel for K <= 256,
// else the fallback GEMM.
template <typename TA, typename TC>
void dense(int M, int N, int K, const TA* A, const bf16* W, long long sbk, long long sbj, TC* C,
           int ldc, const float* bias, int relu, const bf16* gate, hipStream_t st) {
  if (K <= 32) dense_launch<1>(M, N, K, A, W, sbk, sbj, C, ldc, bias, relu, gate, st);
  else if (K <= 64) dense_launch<2>(M, N, K, A, W, sbk, sbj, C, ldc, bias, relu, gate, st);
  else if (K <= 128) dense_launch<4>(M, N, K, A, W, sbk, sbj, C, ldc, bias, relu, gate, st);
  else if (K <= 256) dense_launch<8>(M, N, K, A, W, sbk, sbj, C, ldc, bias, relu, gate, st);
  else {
    dim3 grid((N + 31) / 32, (M + 31) / 32);
    k_gemm<TA, TC><<<grid, 256, 0, st>>>(M, N, K, A, K, 1, W, sbk, sbj, C, ldc, bias, relu, gate);
  }
}

// ---------------------------------------------------------------------------
// Weight gradient, split over the rows r (the batch):
//   part[c][i][j] = sum_{r in chunk c} D[r][i] X[r][j]   (i < M, j < N)
// with D [R][M] FP32 and X [R][N] (FP32 or BF16), and, in the workgroups of
// the first column tile, cpart[c][i] = sum_{r in chunk c} D[r][i] in FP32
// (the bias gradient).  A workgroup (4 waves) owns a 64x64 tile of the
// output and a chunk of rows; per stage of 64 rows each thread loads column
// t%64 of rows 8 g .. 8 g + 7 of two row groups g (coalesced along the
// columns), converts them to BF16 and writes them as one 16-byte row segment
// of the transposed tiles Dt[i][r], Xt[j][r] in LDS; each wave then
// contracts a 32x32 quarter of the tile with v_mfma_f32_16x16x32_bf16.  The
// next stage's loads are issued before the current stage's products.
template <typename TX>
__global__ __launch_bounds__(256) void k_wgrad(int R, int M, int N, const float* __restrict__ D,
                                               const TX* __restrict__ X, int rows_per_chunk,
                                               float* __restrict__ part,
                                               float* __restrict__ cpart) {
  constexpr int S = 72;  // 64 rows + 8: 16-byte row segments on distinct banks
  __shared__ __align__(16) bf16 dt[64 * S], xt[64 * S];
  __shared__ float cs[4][64];
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64, c = blockIdx.z;
  const int rb = c * rows_per_chunk, re = min(R, rb + rows_per_chunk);
  const int t = threadIdx.x, col = t & 63, g = t >> 6;
  const int l = t & 63, lr = l & 15, lq = l >> 4;
  const int wi = (g >> 1) * 32, wj = (g & 1) * 32;
  const bool di = i0 + col < M, xj = j0 + col < N;
  float dv[16], xv[16];
  auto load = [&](int r0) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = r0 + 8 * (g + 4 * (u >> 3)) + (u & 7);
      dv[u] = (di && r < re) ? D[(size_t)r * M + i0 + col] : 0.f;
      xv[u] = (xj && r < re) ? ld_f(X + (size_t)r * N + j0 + col) : 0.f;
    }
  };
  f32x4 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
  float csum = 0.f;
  if (rb < re) load(rb);
  for (int r0 = rb; r0 < re; r0 += 64) {
#pragma unroll
    for (int u = 0; u < 16; ++u) csum += dv[u];
    __syncthreads();  // the previous stage's fragment reads are done
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int rr = 8 * (g + 4 * h);
      *reinterpret_cast<bf16x8*>(dt + col * S + rr) =
          to_bf8(f32x8{dv[8 * h], dv[8 * h + 1], dv[8 * h + 2], dv[8 * h + 3], dv[8 * h + 4],
                       dv[8 * h + 5], dv[8 * h + 6], dv[8 * h + 7]});
      *reinterpret_cast<bf16x8*>(xt + col * S + rr) =
          to_bf8(f32x8{xv[8 * h], xv[8 * h + 1], xv[8 * h + 2], xv[8 * h + 3], xv[8 * h + 4],
                       xv[8 * h + 5], xv[8 * h + 6], xv[8 * h + 7]});
    }
    __syncthreads();
    if (r0 + 64 < re) load(r0 + 64);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        a[p] = *reinterpret_cast<const bf16x8*>(dt + (wi + 16 * p + lr) * S + 32 * s + 8 * lq);
        b[p] = *reinterpret_cast<const bf16x8*>(xt + (wj + 16 * p + lr) * S + 32 * s + 8 * lq);
      }
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[p], b[q], acc[p][q], 0, 0, 0);
    }
  }
  // lane l holds rows 4 (l/16) .. +3, column l%16 of each 16x16 product
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int j = j0 + wj + 16 * q + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wi + 16 * p + 4 * lq + v;
        if (i < M && j < N) part[((size_t)c * M + i) * N + j] = acc[p][q][v];
      }
    }
  if (blockIdx.y == 0) {
    cs[g][col] = csum;
    __syncthreads();
    if (t < 64 && i0 + t < M)
      cpart[(size_t)c * M + i0 + t] = ((cs[0][t] + cs[1][t]) + cs[2][t]) + cs[3][t];
  }
}

// out[e] = sum_{c < nc} part[c n + e], summed in the order of c
__global__ void k_sum_parts(long long n, int nc, const float* __restrict__ part,
                            float* __restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float s = 0.f;
  int c = 0;
  for (; c + 8 <= nc; c += 8) {  // eight loads in flight, added in order
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(c + u) * n + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; c < nc; ++c) s += part[(size_t)c * n + e];
  out[e] = s;
}

// chunks of the weight-gradient split for R rows and an M x N output: about
// 1024 workgroups, at least 64 rows per chunk
void wgrad_split(int R, int M, int N, int* nchunk, int* rows) {
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int nc = std::max(1, std::min((1024 + tiles - 1) / tiles, (R + 63) / 64));
  int rc = (((R + nc - 1) / nc) + 63) / 64 * 64;
  *rows = rc;
  *nchunk = (R + rc - 1) / rc;
}

// partial-sum floats of wgrad for R rows: products, then column sums
long long wgrad_part_floats(int R, int M, int N) {
  int nc, rc;
  wgrad_split(R, M, N, &nc, &rc);
  return (long long)nc * M * N + (long long)nc * M;
}

// dW[i][j] = sum_r D[r][i] X[r][j] and db[i] = sum_r D[r][i], through the
// partial-sum buffer part
template <typename TX>
void wgrad(int R, int M, int N, const float* D, const TX* X, float* dW, float* db, float* part,
           hipStream_t st) {
  int nc, rc;
  wgrad_split(R, M, N, &nc, &rc);
  float* cpart = part + (size_t)nc * M * N;
  k_wgrad<TX><<<dim3((M + 63) / 64, (N + 63) / 64, nc), 256, 0, st>>>(R, M, N, D, X, rc, part,
                                                                    cpart);
  const long long n = (long long)M * N;
  k_sum_parts<<<(int)((n + 255) / 256), 256, 0, st>>>(n, nc, part, dW);
  k_sum_parts<<<(M + 255) / 256, 256, 0, st>>>(M, nc, cpart, db);
}

// dy = 2 (y - t) / n and the block's share of loss = mean((y - t)^2),
// n = rows * cols: part[b] = sum over the elements b*256 + t + q*gridDim*256
// of (y - t)^2 / n (fixed reduction order); k_sum_parts adds the shares.
__global__ __launch_bounds__(256) void k_mse(int n, const float* y, const float* t, float* dy,
                                             float* part) {
  __shared__ float sh[256];
  float s = 0.f;
  const float inv = 1.f / (float)n;
  for (int q = blockIdx.x * 256 + threadIdx.x; q < n; q += gridDim.x * 256) {
    const float e = y[q] - t[q];
    dy[q] = 2.f * e * inv;
    s += e * e;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] * inv;
}
constexpr int kMseBlocks = 256;

// Adam (Kingma & Ba, 2015) on the FP32 master parameters, then the BF16 copy.
__global__ void k_adam(long long n, float* w, unsigned short* wb, const float* g, float* m,
                       float* v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.f - b1) * gq;
  const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  const float wq = w[q] - lr * (mq / c1) / (sqrtf(vq / c2) + eps);
  w[q] = wq;
  wb[q] = f2bf(wq);
}

__global__ void k_to_bf16(long long n, const float* w, unsigned short* wb) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) wb[q] = f2bf(w[q]);
}

// rows perm[b0 + r] of X (cols wide) -> row r of Xb
__global__ void k_gather(int nb, int cols, const int* perm, int b0, const float* X, float* Xb) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)nb * cols) return;
  const int r = (int)(q / cols), c = (int)(q % cols);
  Xb[q] = X[(size_t)perm[b0 + r] * cols + c];
}

void* malloc_dev(sgw_mlp* m, size_t bytes) {
  bytes = std::max<size_t>(bytes, 256);
  void* p = nullptr;
  if (m->has_al) p = m->al.alloc(bytes, m->al.user);
  else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
  if (p) {
    m->mem.push_back(p);
    if (hipMemset(p, 0, bytes) != hipSuccess) return nullptr;
  }
  return p;
}
template <class T>
T* dalloc(sgw_mlp* m, size_t n) {
  return reinterpret_cast<T*>(malloc_dev(m, n * sizeof(T)));
}

uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
double unif(uint64_t& s) { return (splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

int ensure_cap(sgw_mlp* m, int nb) {
  if (nb <= m->cap) return 0;
  const int c = std::max(nb, 256);
  const int H = m->H, ni = m->nin, ng = m->ng;
  const long long np = std::max({wgrad_part_floats(c, ng, H), wgrad_part_floats(c, H, H),
                                 wgrad_part_floats(c, H, ni), (long long)kMseBlocks});
  m->xb = dalloc<float>(m, (size_t)c * ni);
  m->tb = dalloc<float>(m, (size_t)c * ng);
  m->h1 = dalloc<bf16>(m, (size_t)c * H);
  m->h2 = dalloc<bf16>(m, (size_t)c * H);
  m->y = dalloc<float>(m, (size_t)c * ng);
  m->dy = dalloc<float>(m, (size_t)c * ng);
  m->d2 = dalloc<float>(m, (size_t)c * H);
  m->d1 = dalloc<float>(m, (size_t)c * H);
  m->part = dalloc<float>(m, (size_t)np);
  if (!m->xb || !m->tb || !m->h1 || !m->h2 || !m->y || !m->dy || !m->d2 || !m->d1 || !m->part) {
    m->err = "device allocation failed (MLP work space)";
    return SGW_ENOMEM;
  }
  m->cap = c;
  return 0;
}

// forward on rows x[nb][nin] with the hidden activations (BF16, the operands
// of the next layer's products) in h1, h2 ([nb][H] each; the work space's
// unless given)
void forward(sgw_mlp* m, const float* x, float* y, int nb, hipStream_t st, bf16* h1 = nullptr,
             bf16* h2 = nullptr) {
  const int H = m->H, ni = m->nin, ng = m->ng;
  const bf16* wb = m->wb;
  const float* w = m->w;
  if (!h1) h1 = m->h1;
  if (!h2) h2 = m->h2;
  // h = relu(x W^T + b): W(k,j) = W[j][k]
  dense<float, bf16>(nb, H, ni, x, wb + m->off[0], 1, ni, h1, H, w + m->off[1], 1, nullptr, st);
  dense<bf16, bf16>(nb, H, H, h1, wb + m->off[2], 1, H, h2, H, w + m->off[3], 1, nullptr, st);
  dense<bf16, float>(nb, ng, H, h2, wb + m->off[4], 1, H, y, ng, w + m->off[5], 0, nullptr, st);
}

// Scratch of the allocation-free forward pass (sgw_mlp_forward_noalloc):
// the two hidden activations, nb x H BF16 values each (nb x 2 x H is limited
// to 4 Mi, the array's length in floats).  Every GPU that runs the library
// holds its own copy until the process ends; host code reaches it
// only through the per-device address from hipGetSymbolAddress.
#define SGW_MLP_SCRATCH_FLOATS (4 << 20)  // 16 MiB
static __device__ __align__(256) float scratch[SGW_MLP_SCRATCH_FLOATS];
#define SGW_MAX_DEVICES 64
static float* scratch_ptr[SGW_MAX_DEVICES] = {};
static std::mutex scratch_mu;

// device address of this device's scratch (looked up once per device, with
// that device current); nullptr on a HIP error
float* scratch_address(int dev) {
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    scratch_ptr[dev] = reinterpret_cast<float*>(p);
  }
  return scratch_ptr[dev];
}

// loss and gradient of the mean squared error of rows xb -> tb (work space)
void backward(sgw_mlp* m, const float* x, const float* t, int nb, hipStream_t st) {
  const int H = m->H, ni = m->nin, ng = m->ng;
  float* g = m->g;
  const bf16* wb = m->wb;
  forward(m, x, m->y, nb, st);
  const int n = nb * ng;
  const int nmb = std::max(1, std::min(kMseBlocks, (n + 1023) / 1024));
  k_mse<<<nmb, 256, 0, st>>>(n, m->y, t, m->dy, m->part);
  k_sum_parts<<<1, 256, 0, st>>>(1, nmb, m->part, m->loss);
  // layer 3: dW3 = dy^T h2, db3 = colsum(dy), d2 = (dy W3) * [h2 > 0]
  wgrad<bf16>(nb, ng, H, m->dy, m->h2, g + m->off[4], g + m->off[5], m->part, st);
  dense<float, float>(nb, H, ng, m->dy, wb + m->off[4], H, 1, m->d2, H, nullptr, 0, m->h2, st);
  // layer 2
  wgrad<bf16>(nb, H, H, m->d2, m->h1, g + m->off[2], g + m->off[3], m->part, st);
  dense<float, float>(nb, H, H, m->d2, wb + m->off[2], H, 1, m->d1, H, nullptr, 0, m->h1, st);
  // layer 1
  wgrad<float>(nb, H, ni, m->d1, x, g + m->off[0], g + m->off[1], m->part, st);
}

int launch_check(sgw_mlp* m) {
  if (hipGetLastError() != hipSuccess) {
    m->err = "kernel launch failed";
    return SGW_EHIP;
  }
  return 0;
}

}  // namespace

namespace sgw {
int mlp_forward(sgw_mlp* m, const float* x, float* y, int nb, hipStream_t st) {
  if (!m || !x || !y || nb <= 0) return SGW_EINVAL;
  int rc = ensure_cap(m, nb);
  if (rc) return rc;
  forward(m, x, y, nb, st);
  return launch_check(m);
}
}  // namespace sgw

extern "C" {

int sgw_mlp_create(int n_in, int n_out, int hidden, unsigned long long seed,
                   const sgw_allocator* al, sgw_mlp** out) {
  if (!out) return SGW_EINVAL;
  *out = nullptr;
  if (n_in <= 0 || n_out <= 0 || hidden <= 0 || hidden > 4096 || n_in > (1 << 22) ||
      n_out > (1 << 20))
    return SGW_EINVAL;
  sgw_mlp* m = new sgw_mlp();
  if (al && al->alloc && al->free) {
    m->al = *al;
    m->has_al = true;
  }
  m->ng = n_out;
  m->nin = n_in;
  m->H = hidden;
  const long long H = hidden, ni = m->nin, ng = n_out;
  const long long sizes[6] = {H * ni, H, H * H, H, ng * H, ng};
  long long o = 0;
  for (int q = 0; q < 6; ++q) {
    m->off[q] = o;
    o += sizes[q];
  }
  m->np = o;
  // He-uniform weights (ReLU), last layer scaled by 0.1 so the initial
  // correction is small; zero biases.
  std::vector<float> w((size_t)o, 0.f);
  uint64_t s = seed;
  const long long fan[3] = {ni, H, H};
  for (int layer = 0; layer < 3; ++layer) {
    const double a = std::sqrt(6.0 / fan[layer]) * (layer == 2 ? 0.1 : 1.0);
    for (long long q = 0; q < sizes[2 * layer]; ++q)
      w[(size_t)(m->off[2 * layer] + q)] = (float)((2.0 * unif(s) - 1.0) * a);
  }
  m->w = dalloc<float>(m, (size_t)o);
  m->wb = dalloc<unsigned short>(m, (size_t)o);
  m->g = dalloc<float>(m, (size_t)o);
  m->m = dalloc<float>(m, (size_t)o);
  m->v = dalloc<float>(m, (size_t)o);
  m->loss = dalloc<float>(m, 1);
  if (!m->w || !m->wb || !m->g || !m->m || !m->v || !m->loss ||
      hipHostMalloc((void**)&m->hloss, sizeof(float)) != hipSuccess) {
    m->err = "allocation failed";
    *out = m;
    return SGW_ENOMEM;
  }
  if (hipMemcpy(m->w, w.data(), (size_t)o * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    m->err = "upload failed";
    *out = m;
    return SGW_EHIP;
  }
  k_to_bf16<<<(int)((o + 255) / 256), 256>>>(o, m->w, m->wb);
  if (hipDeviceSynchronize() != hipSuccess) {
    m->err = "device error during set-up";
    *out = m;
    return SGW_EHIP;
  }
  *out = m;
  return 0;
}

int sgw_mlp_destroy(sgw_mlp* m) {
  if (!m) return 0;
  (void)hipDeviceSynchronize();
  for (void* p : m->mem) {
    if (m->has_al) m->al.free(p, m->al.user);
    else (void)hipFree(p);
  }
  if (m->hloss) (void)hipHostFree(m->hloss);
  delete m;
  return 0;
}

long long sgw_mlp_num_params(const sgw_mlp* m) { return m ? m->np : -1; }

const char* sgw_mlp_last_error(const sgw_mlp* m) { return m ? m->err.c_str() : "null model"; }

int sgw_mlp_params(sgw_mlp* m, float* w, int set, int where, void* stream) {
  if (!m || !w || (where != SGW_HOST && where != SGW_DEVICE)) return SGW_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const size_t bytes = (size_t)m->np * sizeof(float);
  hipMemcpyKind kind = set ? (where == SGW_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice)
                           : (where == SGW_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice);
  hipError_t e = set ? hipMemcpyAsync(m->w, w, bytes, kind, st)
                     : hipMemcpyAsync(w, m->w, bytes, kind, st);
  if (e != hipSuccess) {
    m->err = "copy failed";
    return SGW_EHIP;
  }
  if (set) {
    k_to_bf16<<<(int)((m->np + 255) / 256), 256, 0, st>>>(m->np, m->w, m->wb);
    m->adam_t = 0;  // new parameters: fresh Adam moments
    (void)hipMemsetAsync(m->m, 0, bytes, st);
    (void)hipMemsetAsync(m->v, 0, bytes, st);
  }
  if (hipStreamSynchronize(st) != hipSuccess) {
    m->err = "device error";
    return SGW_EHIP;
  }
  return 0;
}

int sgw_mlp_forward(sgw_mlp* m, const float* x, float* y, int nb, void* stream) {
  int rc = sgw::mlp_forward(m, x, y, nb, (hipStream_t)stream);
  if (rc) return rc;
  return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? 0 : SGW_EHIP;
}

int sgw_mlp_forward_noalloc(sgw_mlp* m, const float* x, float* y, int nb, void* stream) {
  if (!m || !x || !y || nb <= 0) return SGW_EINVAL;
  if ((long long)nb * 2 * m->H > SGW_MLP_SCRATCH_FLOATS) {
    m->err = "batch too large for the static scratch (nb x 2 x hidden above 4 Mi floats)";
    return SGW_EINVAL;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SGW_MAX_DEVICES) {
    m->err = "no usable HIP device";
    return SGW_EHIP;
  }
  float* p = scratch_address(dev);
  if (!p) {
    m->err = "hipGetSymbolAddress failed for the scratch array";
    return SGW_EHIP;
  }
  bf16* h1 = reinterpret_cast<bf16*>(p);  // two BF16 activations, the second 16-byte aligned
  forward(m, x, y, nb, (hipStream_t)stream, h1, h1 + (((size_t)nb * m->H + 7) & ~(size_t)7));
  return launch_check(m);
}

int sgw_mlp_loss_grad(sgw_mlp* m, const float* x, const float* t, int nb, float* grad,
                      float* loss, void* stream) {
  if (!m || !x || !t || nb <= 0) return SGW_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int rc = ensure_cap(m, nb);
  if (rc) return rc;
  backward(m, x, t, nb, st);
  if ((rc = launch_check(m))) return rc;
  if (grad &&
      hipMemcpyAsync(grad, m->g, (size_t)m->np * sizeof(float), hipMemcpyDeviceToDevice, st) !=
          hipSuccess)
    return SGW_EHIP;
  if (hipMemcpyAsync(m->hloss, m->loss, sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    m->err = "device error";
    return SGW_EHIP;
  }
  if (loss) *loss = *m->hloss;
  return 0;
}

int sgw_mlp_train(sgw_mlp* m, const float* x, const float* t, int nsamples, int epochs,
                  int batch, double lr, unsigned long long seed, void* stream,
                  float* final_loss) {
  if (!m || !x || !t || nsamples <= 0 || epochs <= 0 || batch <= 0 || !(lr > 0)) return SGW_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  batch = std::min(batch, nsamples);
  int rc = ensure_cap(m, batch);
  if (rc) return rc;
  if (nsamples > m->perm_cap) {
    m->perm = dalloc<int>(m, (size_t)nsamples);
    if (!m->perm) {
      m->err = "device allocation failed (permutation)";
      return SGW_ENOMEM;
    }
    m->perm_cap = nsamples;
  }
  std::vector<int> perm((size_t)nsamples);
  uint64_t s = seed;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  double last = 0.0;
  for (int e = 0; e < epochs; ++e) {
    for (int q = 0; q < nsamples; ++q) perm[q] = q;
    for (int q = nsamples - 1; q > 0; --q) {
      const int r = (int)(splitmix64(s) % (uint64_t)(q + 1));
      std::swap(perm[q], perm[r]);
    }
    if (hipMemcpyAsync(m->perm, perm.data(), (size_t)nsamples * sizeof(int),
                       hipMemcpyHostToDevice, st) != hipSuccess)
      return SGW_EHIP;
    double sum = 0.0;
    int nbat = 0;
    for (int b0 = 0; b0 + batch <= nsamples; b0 += batch) {
      const long long nx = (long long)batch * m->nin, nt = (long long)batch * m->ng;
      k_gather<<<(int)((nx + 255) / 256), 256, 0, st>>>(batch, m->nin, m->perm, b0, x, m->xb);
      k_gather<<<(int)((nt + 255) / 256), 256, 0, st>>>(batch, m->ng, m->perm, b0, t, m->tb);
      backward(m, m->xb, m->tb, batch, st);
      ++m->adam_t;
      const float c1 = 1.f - (float)std::pow(b1, (double)m->adam_t);
      const float c2 = 1.f - (float)std::pow(b2, (double)m->adam_t);
      k_adam<<<(int)((m->np + 255) / 256), 256, 0, st>>>(m->np, m->w, m->wb, m->g, m->m, m->v,
                                                         (float)lr, b1, b2, eps, c1, c2);
      if (e + 1 == epochs) {  // loss of the last epoch (one read per batch)
        if (hipMemcpyAsync(m->hloss, m->loss, sizeof(float), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
          return SGW_EHIP;
        sum += *m->hloss;
        ++nbat;
      }
    }
    if ((rc = launch_check(m))) return rc;
    if (e + 1 == epochs) last = nbat ? sum / nbat : 0.0;
  }
  if (hipStreamSynchronize(st) != hipSuccess) return SGW_EHIP;
  if (final_loss) *final_loss = (float)last;
  return 0;
}

}  // extern "C"
