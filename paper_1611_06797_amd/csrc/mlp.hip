// Learned Laplace quadrature: a small MLP proposes the minimax exponents and
// weights, a few Remez steps polish them, and the plain fit is both the arbiter
// (certification by equioscillation) and the fallback.
//
// Network: 3 -> 64 (tanh) -> 64 (tanh) -> 24, FP32.
//   input   (log x_min, log R / log 1e4, N / 12),   R = x_max / x_min
//   output  slots 0..11: log alpha_n, slots 12..23: log beta_n of the
//           unit-interval fit (y = x / x_min in [1, R]); the first N of each
//           half are used, the rest are masked out of the loss.
// Loss: mean squared error over the unmasked outputs.
// Training: Adam on the GPU with the kernels below (forward, backward, Adam);
// every reduction is a fixed-order loop, so runs are reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ltmp2.h"
#include "quadrature.h"

namespace ltmp2 {

constexpr int kIn = 3, kH = 64, kOut = 24;
constexpr int kP = kH * kIn + kH + kH * kH + kH + kOut * kH + kOut;
static_assert(kP == LTMP2_MLP_NPARAM, "parameter count");

struct Net {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
};
inline Net unpack(const float* p) {
  Net n;
  n.W1 = p;
  n.b1 = n.W1 + kH * kIn;
  n.W2 = n.b1 + kH;
  n.b2 = n.W2 + kH * kH;
  n.W3 = n.b2 + kH;
  n.b3 = n.W3 + kOut * kH;
  return n;
}

// Y[b][o] = act(sum_i X[b][i] W[o][i] + bias[o]); act 1 = tanh
__global__ void k_lin_fwd(const float* __restrict__ X, int B, int I, const float* __restrict__ W,
                          const float* __restrict__ bias, int O, int act, float* __restrict__ Y) {
  const long t = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= long(B) * O) return;
  const int b = int(t / O), o = int(t - long(b) * O);
  float s = bias[o];
  for (int i = 0; i < I; ++i) s += X[long(b) * I + i] * W[o * I + i];
  Y[t] = act ? tanhf(s) : s;
}

// dX[b][i] = (sum_o dY[b][o] W[o][i]) * (1 - A[b][i]^2)   (A = tanh output feeding W)
__global__ void k_lin_bwd_x(const float* __restrict__ dY, int B, int O, const float* __restrict__ W,
                            int I, const float* __restrict__ A, float* __restrict__ dX) {
  const long t = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= long(B) * I) return;
  const int b = int(t / I), i = int(t - long(b) * I);
  float s = 0.f;
  for (int o = 0; o < O; ++o) s += dY[long(b) * O + o] * W[o * I + i];
  const float a = A[t];
  dX[t] = s * (1.f - a * a);
}

// dW[o][i] = sum_b dY[b][o] X[b][i] (threads o*I + i), db[o] = sum_b dY[b][o]
__global__ void k_lin_bwd_w(const float* __restrict__ dY, const float* __restrict__ X, int B,
                            int O, int I, float* __restrict__ dW, float* __restrict__ db) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < O * I) {
    const int o = t / I, i = t - o * I;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += dY[long(b) * O + o] * X[long(b) * I + i];
    dW[t] = s;
  } else if (t < O * I + O) {
    const int o = t - O * I;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += dY[long(b) * O + o];
    db[o] = s;
  }
}

// masked squared error: dOut = 2 (out - y) m / count, lossb[b] = sum_k m (out - y)^2
__global__ void k_mse(const float* __restrict__ out, const float* __restrict__ y,
                      const float* __restrict__ m, int B, int K, float inv_count,
                      float* __restrict__ dout, float* __restrict__ lossb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float s = 0.f;
  for (int k = 0; k < K; ++k) {
    const long q = long(b) * K + k;
    const float d = (out[q] - y[q]) * m[q];
    dout[q] = 2.f * d * inv_count;
    s += d * d;
  }
  lossb[b] = s;
}

__global__ void k_sum(const float* __restrict__ x, int n, float* __restrict__ out) {
  __shared__ float red[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] += red[0];
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void k_gather(const float* __restrict__ src, const int* __restrict__ idx, int B, int K,
                         float* __restrict__ dst) {
  const long t = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= long(B) * K) return;
  const int b = int(t / K), k = int(t - long(b) * K);
  dst[t] = src[long(idx[b]) * K + k];
}

namespace {

inline unsigned nblk(long n) { return unsigned((n + 255) / 256); }

// splitmix64 (Steele, Lea, Flood 2014): counter-based 64-bit generator
inline uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline double uniform01(uint64_t& s) { return double(splitmix64(s) >> 11) * 0x1.0p-53; }

// Device workspace of one forward/backward pass over a batch.
struct Work {
  float *P, *G, *X, *Y, *M, *H1, *H2, *O, *dO, *dH2, *dH1, *lossb, *loss;
  std::vector<void*> owned;
  ~Work() {
    for (void* p : owned) (void)hipFree(p);
  }
  bool alloc(float** p, size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(float)) != hipSuccess) return false;
    owned.push_back(q);
    *p = static_cast<float*>(q);
    return true;
  }
  bool init(int B) {
    return alloc(&P, kP) && alloc(&G, kP) && alloc(&X, size_t(B) * kIn) &&
           alloc(&Y, size_t(B) * kOut) && alloc(&M, size_t(B) * kOut) &&
           alloc(&H1, size_t(B) * kH) && alloc(&H2, size_t(B) * kH) &&
           alloc(&O, size_t(B) * kOut) && alloc(&dO, size_t(B) * kOut) &&
           alloc(&dH2, size_t(B) * kH) && alloc(&dH1, size_t(B) * kH) && alloc(&lossb, B) &&
           alloc(&loss, 1);
  }
};

void forward(const Work& w, int B, hipStream_t st) {
  Net n = unpack(w.P);
  hipLaunchKernelGGL(k_lin_fwd, dim3(nblk(long(B) * kH)), dim3(256), 0, st, w.X, B, kIn, n.W1,
                     n.b1, kH, 1, w.H1);
  hipLaunchKernelGGL(k_lin_fwd, dim3(nblk(long(B) * kH)), dim3(256), 0, st, w.H1, B, kH, n.W2,
                     n.b2, kH, 1, w.H2);
  hipLaunchKernelGGL(k_lin_fwd, dim3(nblk(long(B) * kOut)), dim3(256), 0, st, w.H2, B, kH, n.W3,
                     n.b3, kOut, 0, w.O);
}

// gradient of the masked MSE into w.G; loss (mean) accumulated into w.loss
void backward(const Work& w, int B, float inv_count, hipStream_t st) {
  Net n = unpack(w.P);
  float* gW1 = w.G;
  float* gb1 = gW1 + kH * kIn;
  float* gW2 = gb1 + kH;
  float* gb2 = gW2 + kH * kH;
  float* gW3 = gb2 + kH;
  float* gb3 = gW3 + kOut * kH;
  hipLaunchKernelGGL(k_mse, dim3(nblk(B)), dim3(256), 0, st, w.O, w.Y, w.M, B, kOut, inv_count,
                     w.dO, w.lossb);
  hipLaunchKernelGGL(k_lin_bwd_w, dim3(nblk(kOut * kH + kOut)), dim3(256), 0, st, w.dO, w.H2, B,
                     kOut, kH, gW3, gb3);
  hipLaunchKernelGGL(k_lin_bwd_x, dim3(nblk(long(B) * kH)), dim3(256), 0, st, w.dO, B, kOut, n.W3,
                     kH, w.H2, w.dH2);
  hipLaunchKernelGGL(k_lin_bwd_w, dim3(nblk(kH * kH + kH)), dim3(256), 0, st, w.dH2, w.H1, B, kH,
                     kH, gW2, gb2);
  hipLaunchKernelGGL(k_lin_bwd_x, dim3(nblk(long(B) * kH)), dim3(256), 0, st, w.dH2, B, kH, n.W2,
                     kH, w.H1, w.dH1);
  hipLaunchKernelGGL(k_lin_bwd_w, dim3(nblk(kH * kIn + kH)), dim3(256), 0, st, w.dH1, w.X, B, kH,
                     kIn, gW1, gb1);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, w.lossb, B, w.loss);
}

float mask_count(const float* M, long n) {
  double c = 0.0;
  for (long i = 0; i < n; ++i) c += M[i];
  return float(c);
}

thread_local std::string g_mlp_error;

ltmp2_status mfail(ltmp2_status s, const std::string& m) {
  g_mlp_error = m;
  return s;
}

}  // namespace

void mlp_features(double x_min, double x_max, int n_tau, float* f) {
  f[0] = float(std::log(x_min));
  f[1] = float(std::log(x_max / x_min) / std::log(1e4));
  f[2] = float(n_tau) / 12.0f;
}

const char* mlp_last_error() { return g_mlp_error.c_str(); }

}  // namespace ltmp2

using namespace ltmp2;

extern "C" ltmp2_status ltmp2_mlp_init(uint64_t seed, float* params) {
  if (!params) return mfail(LTMP2_EINVAL, "params is NULL");
  uint64_t s = seed;
  auto fill = [&](float* p, int fan_in, int fan_out, int count) {
    const double a = std::sqrt(6.0 / (fan_in + fan_out));  // Glorot uniform
    for (int k = 0; k < count; ++k) p[k] = float((2.0 * uniform01(s) - 1.0) * a);
  };
  Net n = unpack(params);
  fill(const_cast<float*>(n.W1), kIn, kH, kH * kIn);
  std::fill(const_cast<float*>(n.b1), const_cast<float*>(n.b1) + kH, 0.f);
  fill(const_cast<float*>(n.W2), kH, kH, kH * kH);
  std::fill(const_cast<float*>(n.b2), const_cast<float*>(n.b2) + kH, 0.f);
  fill(const_cast<float*>(n.W3), kH, kOut, kOut * kH);
  std::fill(const_cast<float*>(n.b3), const_cast<float*>(n.b3) + kOut, 0.f);
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_quadrature_table(int n_tau, int count, const double* R,
                                               double* alpha, double* beta, double* delta) {
  if ((count > 0) && (!R || !alpha || !beta)) return mfail(LTMP2_EINVAL, "NULL array");
  const int r = quadrature_table(n_tau, count, R, alpha, beta, delta);
  if (r == 1) return mfail(LTMP2_EINVAL, "need ascending R > 1 and 1 <= n_tau <= 16");
  if (r != 0) return mfail(LTMP2_ENUMERIC, "continuation failed");
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_mlp_dataset(int count, uint64_t seed, double dmin_lo, double dmin_hi,
                                          double ratio_lo, double ratio_hi, const int* n_taus,
                                          int n_choices, float* X, float* Y, float* M,
                                          double* xrange) {
  if (count < 1 || !n_taus || n_choices < 1 || !X || !Y || !M)
    return mfail(LTMP2_EINVAL, "bad dataset arguments");
  if (!(0 < dmin_lo && dmin_lo <= dmin_hi) || !(1 < ratio_lo && ratio_lo <= ratio_hi))
    return mfail(LTMP2_EINVAL, "bad sampling ranges");
  for (int c = 0; c < n_choices; ++c)
    if (n_taus[c] < 1 || n_taus[c] > 12) return mfail(LTMP2_EINVAL, "n_tau choices must be 1..12");
  uint64_t s = seed;
  std::vector<double> xmin(count), ratio(count);
  std::vector<int> nt(count);
  for (int k = 0; k < count; ++k) {
    nt[k] = n_taus[std::min<int>(n_choices - 1, int(uniform01(s) * n_choices))];
    xmin[k] = std::exp(std::log(dmin_lo) + uniform01(s) * std::log(dmin_hi / dmin_lo));
    ratio[k] = std::exp(std::log(ratio_lo) + uniform01(s) * std::log(ratio_hi / ratio_lo));
  }
  std::fill(Y, Y + size_t(count) * kOut, 0.f);
  std::fill(M, M + size_t(count) * kOut, 0.f);
  // one continuation sweep per n_tau choice, sweeps in parallel threads
  std::vector<int> status(n_choices, 0);
  std::vector<std::thread> pool;
  for (int c = 0; c < n_choices; ++c) {
    pool.emplace_back([&, c]() {
      const int n = n_taus[c];
      for (int c2 = 0; c2 < c; ++c2)
        if (n_taus[c2] == n) return;  // repeated choice: handled once
      std::vector<int> idx;
      for (int k = 0; k < count; ++k)
        if (nt[k] == n) idx.push_back(k);
      if (idx.empty()) return;
      std::sort(idx.begin(), idx.end(), [&](int a, int b) { return ratio[a] < ratio[b]; });
      std::vector<double> R(idx.size()), al(idx.size() * n), be(idx.size() * n);
      for (size_t q = 0; q < idx.size(); ++q) R[q] = ratio[idx[q]];
      if (quadrature_table(n, (int)idx.size(), R.data(), al.data(), be.data(), nullptr) != 0) {
        status[c] = 1;
        return;
      }
      for (size_t q = 0; q < idx.size(); ++q) {
        const int k = idx[q];
        for (int t = 0; t < n; ++t) {
          Y[size_t(k) * kOut + t] = float(std::log(al[q * n + t]));
          Y[size_t(k) * kOut + 12 + t] = float(std::log(be[q * n + t]));
          M[size_t(k) * kOut + t] = 1.f;
          M[size_t(k) * kOut + 12 + t] = 1.f;
        }
      }
    });
  }
  for (auto& t : pool) t.join();
  for (int c = 0; c < n_choices; ++c)
    if (status[c]) return mfail(LTMP2_ENUMERIC, "minimax table failed");
  for (int k = 0; k < count; ++k) {
    mlp_features(xmin[k], xmin[k] * ratio[k], nt[k], X + size_t(k) * kIn);
    if (xrange) {
      xrange[2 * k] = xmin[k];
      xrange[2 * k + 1] = xmin[k] * ratio[k];
    }
  }
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_mlp_forward(const float* params, const float* X, int n, float* Yout,
                                          void* stream) {
  if (!params || !X || !Yout || n < 1) return mfail(LTMP2_EINVAL, "bad arguments");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Work w;
  if (!w.init(n)) return mfail(LTMP2_ENOMEM, "device allocation failed");
  if (hipMemcpyAsync(w.P, params, kP * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(w.X, X, size_t(n) * kIn * sizeof(float), hipMemcpyHostToDevice, st) !=
          hipSuccess)
    return mfail(LTMP2_EDEVICE, "copy failed");
  forward(w, n, st);
  if (hipGetLastError() != hipSuccess) return mfail(LTMP2_EDEVICE, "launch failed");
  if (hipMemcpyAsync(Yout, w.O, size_t(n) * kOut * sizeof(float), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return mfail(LTMP2_EDEVICE, "copy back failed");
  return LTMP2_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free forward pass.  The hidden activations of up to
// LTMP2_MLP_NOALLOC_MAX_ROWS rows live in `scratch`, a device array of this
// file that every GPU running the library holds for the life of the process
// (8 MiB).  Host code never passes the array's name to a kernel: each
// device's own address of it comes from hipGetSymbolAddress, taken once per
// device (with that device current) on the entry point's first call there.
// Both hidden layers are written in full before they are read, so nothing
// needs clearing between calls; calls that overlap on one GPU share the
// array and race.
namespace {
constexpr int kNoAllocRows = LTMP2_MLP_NOALLOC_MAX_ROWS;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) float scratch[2 * size_t(kNoAllocRows) * kH];

namespace {
// Device address of this GPU's scratch array (nullptr on failure).
float* scratch_on_current_device(std::string& err) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    err = "no usable current device";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<float*>(ptr);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" ltmp2_status ltmp2_mlp_forward_noalloc(const float* params_dev, const float* X_dev,
                                                  int n, float* Y_dev, void* hip_stream) {
  if (!params_dev || !X_dev || !Y_dev) return mfail(LTMP2_EINVAL, "NULL device pointer");
  if (n < 1 || n > kNoAllocRows)
    return mfail(LTMP2_EINVAL, "n must be in [1, " + std::to_string(kNoAllocRows) +
                                   "] for the allocation-free forward pass");
  std::string err;
  float* h = scratch_on_current_device(err);
  if (!h) return mfail(LTMP2_EDEVICE, err);
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  Net net = unpack(params_dev);
  float* h1 = h;
  float* h2 = h + size_t(kNoAllocRows) * kH;
  hipLaunchKernelGGL(k_lin_fwd, dim3(nblk(long(n) * kH)), dim3(256), 0, st, X_dev, n, kIn,
                     net.W1, net.b1, kH, 1, h1);
  hipLaunchKernelGGL(k_lin_fwd, dim3(nblk(long(n) * kH)), dim3(256), 0, st, h1, n, kH, net.W2,
                     net.b2, kH, 1, h2);
  hipLaunchKernelGGL(k_lin_fwd, dim3(nblk(long(n) * kOut)), dim3(256), 0, st, h2, n, kH, net.W3,
                     net.b3, kOut, 0, Y_dev);
  if (hipGetLastError() != hipSuccess) return mfail(LTMP2_EDEVICE, "launch failed");
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_mlp_grad(const float* params, const float* X, const float* Y,
                                       const float* M, int n, float* grad, float* loss,
                                       void* stream) {
  if (!params || !X || !Y || !M || !grad || n < 1) return mfail(LTMP2_EINVAL, "bad arguments");
  const float cnt = mask_count(M, long(n) * kOut);
  if (!(cnt > 0)) return mfail(LTMP2_EINVAL, "empty mask");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Work w;
  if (!w.init(n)) return mfail(LTMP2_ENOMEM, "device allocation failed");
  const size_t bo = size_t(n) * kOut * sizeof(float);
  if (hipMemcpyAsync(w.P, params, kP * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(w.X, X, size_t(n) * kIn * sizeof(float), hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(w.Y, Y, bo, hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(w.M, M, bo, hipMemcpyHostToDevice, st) ||
      hipMemsetAsync(w.loss, 0, sizeof(float), st))
    return mfail(LTMP2_EDEVICE, "copy failed");
  forward(w, n, st);
  backward(w, n, 1.f / cnt, st);
  if (hipGetLastError() != hipSuccess) return mfail(LTMP2_EDEVICE, "launch failed");
  float l = 0.f;
  if (hipMemcpyAsync(grad, w.G, kP * sizeof(float), hipMemcpyDeviceToHost, st) ||
      hipMemcpyAsync(&l, w.loss, sizeof(float), hipMemcpyDeviceToHost, st) ||
      hipStreamSynchronize(st))
    return mfail(LTMP2_EDEVICE, "copy back failed");
  if (loss) *loss = l / cnt;
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_mlp_train(float* params, const float* X, const float* Y,
                                        const float* M, int n, int epochs, int batch, float lr,
                                        uint64_t seed, float* loss_hist, void* stream) {
  if (!params || !X || !Y || !M || n < 1 || epochs < 1 || batch < 1 || !(lr > 0))
    return mfail(LTMP2_EINVAL, "bad arguments");
  batch = std::min(batch, n);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Work w;
  float *dX = nullptr, *dY = nullptr, *dM = nullptr, *m1 = nullptr, *m2 = nullptr;
  int* didx = nullptr;
  if (!w.init(batch) || !w.alloc(&dX, size_t(n) * kIn) || !w.alloc(&dY, size_t(n) * kOut) ||
      !w.alloc(&dM, size_t(n) * kOut) || !w.alloc(&m1, kP) || !w.alloc(&m2, kP) ||
      !w.alloc(reinterpret_cast<float**>(&didx), batch))
    return mfail(LTMP2_ENOMEM, "device allocation failed");
  if (hipMemcpyAsync(w.P, params, kP * sizeof(float), hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(dX, X, size_t(n) * kIn * sizeof(float), hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(dY, Y, size_t(n) * kOut * sizeof(float), hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(dM, M, size_t(n) * kOut * sizeof(float), hipMemcpyHostToDevice, st) ||
      hipMemsetAsync(m1, 0, kP * sizeof(float), st) || hipMemsetAsync(m2, 0, kP * sizeof(float), st))
    return mfail(LTMP2_EDEVICE, "copy failed");
  uint64_t s = seed;
  std::vector<int> perm(n);
  std::vector<float> mrow(size_t(batch) * kOut);
  long step = 0;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int k = 0; k < n; ++k) perm[k] = k;
    for (int k = n - 1; k > 0; --k) std::swap(perm[k], perm[int(uniform01(s) * (k + 1))]);
    // cosine learning-rate schedule
    const float lre = lr * 0.5f * (1.f + std::cos(float(M_PI) * ep / epochs));
    if (hipMemsetAsync(w.loss, 0, sizeof(float), st)) return mfail(LTMP2_EDEVICE, "memset");
    double epoch_count = 0.0;
    for (int b0 = 0; b0 + batch <= n; b0 += batch) {
      if (hipMemcpyAsync(didx, perm.data() + b0, batch * sizeof(int), hipMemcpyHostToDevice, st))
        return mfail(LTMP2_EDEVICE, "copy failed");
      double cnt = 0.0;
      for (int b = 0; b < batch; ++b)
        for (int k = 0; k < kOut; ++k) cnt += M[size_t(perm[b0 + b]) * kOut + k];
      epoch_count += cnt;
      hipLaunchKernelGGL(k_gather, dim3(nblk(long(batch) * kIn)), dim3(256), 0, st, dX, didx, batch,
                         kIn, w.X);
      hipLaunchKernelGGL(k_gather, dim3(nblk(long(batch) * kOut)), dim3(256), 0, st, dY, didx, batch,
                         kOut, w.Y);
      hipLaunchKernelGGL(k_gather, dim3(nblk(long(batch) * kOut)), dim3(256), 0, st, dM, didx, batch,
                         kOut, w.M);
      forward(w, batch, st);
      backward(w, batch, float(1.0 / cnt), st);
      ++step;
      const float bc1 = 1.f - std::pow(b1, float(step)), bc2 = 1.f - std::pow(b2, float(step));
      hipLaunchKernelGGL(k_adam, dim3(nblk(kP)), dim3(256), 0, st, w.P, w.G, m1, m2, kP, lre, b1,
                         b2, eps, bc1, bc2);
      // hipMemcpyAsync of the index list above reads host memory that the next
      // iteration overwrites; keep the stream ordered with the host
      if (hipStreamSynchronize(st)) return mfail(LTMP2_EDEVICE, "training step failed");
    }
    float l = 0.f;
    if (hipMemcpyAsync(&l, w.loss, sizeof(float), hipMemcpyDeviceToHost, st) ||
        hipStreamSynchronize(st))
      return mfail(LTMP2_EDEVICE, "copy back failed");
    if (loss_hist) loss_hist[ep] = float(l / epoch_count);
  }
  if (hipGetLastError() != hipSuccess) return mfail(LTMP2_EDEVICE, "launch failed");
  if (hipMemcpyAsync(params, w.P, kP * sizeof(float), hipMemcpyDeviceToHost, st) ||
      hipStreamSynchronize(st))
    return mfail(LTMP2_EDEVICE, "copy back failed");
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_learned_quadrature(const float* params, double x_min, double x_max,
                                                 int n_tau, int polish_steps, double cert_tol,
                                                 double* tau, double* w, double* delta,
                                                 int* flags, void* stream) {
  if (!params || !tau || !w || n_tau < 1 || n_tau > 12 || !(x_min > 0) || !(x_max > x_min))
    return mfail(LTMP2_EINVAL, "bad arguments");
  float f[kIn], out[kOut];
  mlp_features(x_min, x_max, n_tau, f);
  ltmp2_status s = ltmp2_mlp_forward(params, f, 1, out, stream);
  if (s) return s;
  bool finite = true;
  for (int t = 0; t < n_tau; ++t) {
    tau[t] = std::exp(double(out[t])) / x_min;
    w[t] = std::exp(double(out[12 + t])) / x_min;
    finite = finite && std::isfinite(tau[t]) && std::isfinite(w[t]) && tau[t] > 0 && w[t] > 0;
  }
  int cert = 0;
  double d = 0.0;
  if (finite && remez_polish(x_min, x_max, n_tau, polish_steps, cert_tol, tau, w, &d, &cert) != 0)
    cert = 0;
  int fl = cert ? 1 : 0;
  if (!cert) {
    const int r = minimax_quadrature(x_min, x_max, n_tau, tau, w, &d);
    if (r != 0) return mfail(LTMP2_ENUMERIC, "fallback minimax fit failed");
    fl |= 2;
  }
  if (delta) *delta = d;
  if (flags) *flags = fl;
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_remez_polish(double x_min, double x_max, int n_tau, int steps,
                                           double cert_tol, double* tau, double* w, double* delta,
                                           int* certified) {
  if (!tau || !w) return mfail(LTMP2_EINVAL, "NULL array");
  if (remez_polish(x_min, x_max, n_tau, steps, cert_tol, tau, w, delta, certified) != 0)
    return mfail(LTMP2_EINVAL, "bad arguments");
  return LTMP2_OK;
}

extern "C" const char* ltmp2_mlp_last_error(void) { return mlp_last_error(); }
