// Learned initial guess: the MLP, its training (Adam) and inference kernels.
// Matrix products run on MFMA (v_mfma_f32_16x16x16_bf16: BF16 operands, FP32
// accumulation); everything else is FP32 elementwise or reduction work.
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
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite inputs).
__host__ __device__ inline unsigned short f2bf(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline short ld_bf(const float* p) { return (short)f2bf(*p); }
__device__ inline short ld_bf(const unsigned short* p) { return (short)*p; }

// C[i][j] = epilogue(sum_k A(i,k) B(k,j)) with A(i,k) = A[i*sai + k*sak] and
// B(k,j) = B[k*sbk + j*sbj] (so transposed operands are plain strides).
// Epilogue: + bias[j] (if bias), ReLU (if relu), times [gate[i][j] > 0] (if
// gate).  A workgroup = 4 waves = a 32x32 tile of C, one 16x16 tile per wave;
// each lane loads its 4-value slices of A and B for every 16-wide k step
// (lane l: A rows l%16, B columns l%16, k = 4*(l/16) .. +3), out-of-range
// entries read as zero.  Result of the MFMA: lane l holds rows 4*(l/16) ..
// +3 of column l%16.
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const TA* __restrict__ A,
                                              long long sai, long long sak,
                                              const TB* __restrict__ B, long long sbk,
                                              long long sbj, float* __restrict__ C, int ldc,
                                              const float* __restrict__ bias, int relu,
                                              const float* __restrict__ gate) {
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
    if (gate && !(gate[(size_t)i * ldc + j] > 0.f)) x = 0.f;
    C[(size_t)i * ldc + j] = x;
  }
}

template <typename TA, typename TB>
void gemm(int M, int N, int K, const TA* A, long long sai, long long sak, const TB* B,
          long long sbk, long long sbj, float* C, int ldc, const float* bias, int relu,
          const float* gate, hipStream_t st) {
  dim3 grid((N + 31) / 32, (M + 31) / 32);
  k_gemm<TA, TB><<<grid, 256, 0, st>>>(M, N, K, A, sai, sak, B, sbk, sbj, C, ldc, bias, relu,
                                       gate);
}

// out[j] = sum_i X[i][j] (column sums, fixed order)
__global__ void k_colsum(int rows, int cols, const float* X, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int i = 0; i < rows; ++i) s += X[(size_t)i * cols + j];
  out[j] = s;
}

// dy = 2 (y - t) / n and loss = mean((y - t)^2), n = rows * cols; one
// workgroup, fixed reduction order.
__global__ __launch_bounds__(256) void k_mse(int n, const float* y, const float* t, float* dy,
                                             float* loss) {
  __shared__ float sh[256];
  float s = 0.f;
  const float inv = 1.f / (float)n;
  for (int q = threadIdx.x; q < n; q += 256) {
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
  if (threadIdx.x == 0) *loss = sh[0] * inv;
}

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
  m->xb = dalloc<float>(m, (size_t)c * m->nin);
  m->tb = dalloc<float>(m, (size_t)c * m->ng);
  m->h1 = dalloc<float>(m, (size_t)c * m->H);
  m->h2 = dalloc<float>(m, (size_t)c * m->H);
  m->y = dalloc<float>(m, (size_t)c * m->ng);
  m->dy = dalloc<float>(m, (size_t)c * m->ng);
  m->d2 = dalloc<float>(m, (size_t)c * m->H);
  m->d1 = dalloc<float>(m, (size_t)c * m->H);
  if (!m->xb || !m->tb || !m->h1 || !m->h2 || !m->y || !m->dy || !m->d2 || !m->d1) {
    m->err = "device allocation failed (MLP work space)";
    return SGW_ENOMEM;
  }
  m->cap = c;
  return 0;
}

// forward on rows x[nb][nin] with the hidden activations in h1, h2
// ([nb][H] each; the work space's unless given)
void forward(sgw_mlp* m, const float* x, float* y, int nb, hipStream_t st,
             float* h1 = nullptr, float* h2 = nullptr) {
  const int H = m->H, ni = m->nin, ng = m->ng;
  const unsigned short* wb = m->wb;
  const float* w = m->w;
  if (!h1) h1 = m->h1;
  if (!h2) h2 = m->h2;
  // h = relu(x W^T + b): A(i,k) = x[i][k], B(k,j) = W[j][k]
  gemm<float, unsigned short>(nb, H, ni, x, ni, 1, wb + m->off[0], 1, ni, h1, H,
                              w + m->off[1], 1, nullptr, st);
  gemm<float, unsigned short>(nb, H, H, h1, H, 1, wb + m->off[2], 1, H, h2, H,
                              w + m->off[3], 1, nullptr, st);
  gemm<float, unsigned short>(nb, ng, H, h2, H, 1, wb + m->off[4], 1, H, y, ng,
                              w + m->off[5], 0, nullptr, st);
}

// Scratch of the allocation-free forward pass (sgw_mlp_forward_noalloc):
// the two hidden activations, nb x H floats each.  Every GPU that runs the
// library holds its own copy until the process ends; host code reaches it
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
  const unsigned short* wb = m->wb;
  forward(m, x, m->y, nb, st);
  k_mse<<<1, 256, 0, st>>>(nb * ng, m->y, t, m->dy, m->loss);
  // layer 3: dW3 = dy^T h2, db3 = colsum(dy), d2 = (dy W3) * [h2 > 0]
  gemm<float, float>(ng, H, nb, m->dy, 1, ng, m->h2, H, 1, g + m->off[4], H, nullptr, 0, nullptr,
                     st);
  k_colsum<<<(ng + 255) / 256, 256, 0, st>>>(nb, ng, m->dy, g + m->off[5]);
  gemm<float, unsigned short>(nb, H, ng, m->dy, ng, 1, wb + m->off[4], H, 1, m->d2, H, nullptr, 0,
                              m->h2, st);
  // layer 2
  gemm<float, float>(H, H, nb, m->d2, 1, H, m->h1, H, 1, g + m->off[2], H, nullptr, 0, nullptr, st);
  k_colsum<<<(H + 255) / 256, 256, 0, st>>>(nb, H, m->d2, g + m->off[3]);
  gemm<float, unsigned short>(nb, H, H, m->d2, H, 1, wb + m->off[2], H, 1, m->d1, H, nullptr, 0,
                              m->h1, st);
  // layer 1
  gemm<float, float>(H, ni, nb, m->d1, 1, H, x, ni, 1, g + m->off[0], ni, nullptr, 0, nullptr, st);
  k_colsum<<<(H + 255) / 256, 256, 0, st>>>(nb, H, m->d1, g + m->off[1]);
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
  forward(m, x, y, nb, (hipStream_t)stream, p, p + (size_t)nb * m->H);
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
