// Surrogate MLP kernels (gfx950): 7 -> 256 -> 256 -> 256 -> 3 with SiLU,
// BF16 weights and activations feeding MFMA (v_mfma_f32_16x16x16_bf16) with FP32
// accumulation; FP32 pre-activations, gradients of the biases and Adam master
// weights.  Layer k computes z_k = a_{k-1} W_k + b_k (W_k stored [fan_in][fan_out]),
// a_k = silu(z_k) for the hidden layers; the output layer is linear.  Loss
// L = 1/(3B) sum (y - t)^2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>

#include "ftlm_internal.hpp"

namespace ftlm {

namespace {

constexpr int kIn = 7, kHid = 256, kOut = 3;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// C[m][n] = sum_k A(m,k) B(k,n), A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn]
// (bf16), FP32 accumulation.  Block = 4 waves on a 64x64 tile of C; each wave owns
// 32x32 = 2x2 MFMA 16x16 tiles; K advances 16 at a time through LDS.
// Epilogue modes:
//   0: hidden forward:  Z = C + bias -> zf (fp32, ld N) and a = silu(Z) -> ob (bf16, ld N)
//   1: output forward:  Y = C + bias -> zf (fp32, ld N)
//   2: plain:           zf = C (fp32, ld N)
//   3: backward:        g = C * silu'(zin[m][n]) -> zf (fp32) and ob (bf16)
struct GemmArgs {
  int M, N, K;
  int ksplit;  // mode 2: K split over blockIdx.z, partial products at zf + z*M*N (0 or 1: none)
  const uint16_t *A;
  long sam, sak;
  const uint16_t *B;
  long sbk, sbn;
  int mode;
  const float *bias;
  const float *zin;
  float *zf;
  uint16_t *ob;
};

__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
  __shared__ uint16_t As[64][16 + 4];
  __shared__ uint16_t Bs[16][64 + 4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  // K range of this block (all of K unless split)
  const int ks = g.ksplit > 1 ? g.ksplit : 1;
  const int kchunk = ((g.K + ks - 1) / ks + 15) & ~15;
  const int kb = (int)blockIdx.z * kchunk, ke = min(g.K, kb + kchunk);
  float *zf = g.zf + (ks > 1 ? (long)blockIdx.z * g.M * g.N : 0L);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += 16) {
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int idx = t + 256 * e;  // 0..1023
      {
        const int r = idx >> 4, c = idx & 15;
        const int m = m0 + r, k = k0 + c;
        As[r][c] = (m < g.M && k < ke) ? g.A[(long)m * g.sam + (long)k * g.sak] : (uint16_t)0;
      }
      {
        const int r = idx >> 6, c = idx & 63;
        const int k = k0 + r, n = n0 + c;
        Bs[r][c] = (k < ke && n < g.N) ? g.B[(long)k * g.sbk + (long)n * g.sbn] : (uint16_t)0;
      }
    }
    __syncthreads();
    const int kq = 4 * (lane >> 4), rl = lane & 15;
#pragma unroll
    for (int i = 0; i < 2; i++) {
      bf16x4 a;
#pragma unroll
      for (int j = 0; j < 4; j++) a[j] = (short)As[wm + 16 * i + rl][kq + j];
#pragma unroll
      for (int jj = 0; jj < 2; jj++) {
        bf16x4 b;
#pragma unroll
        for (int j = 0; j < 4; j++) b[j] = (short)Bs[kq + j][wn + 16 * jj + rl];
        acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[i][jj], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // D[row = 4*(lane/16) + j][col = lane % 16] of each 16x16 tile
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int jj = 0; jj < 2; jj++)
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + j;
        const int n = n0 + wn + 16 * jj + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float c = acc[i][jj][j];
        const long o = (long)m * g.N + n;
        if (g.mode == 0) {
          c += g.bias[n];
          g.zf[o] = c;
          g.ob[o] = f2bf(silu(c));
        } else if (g.mode == 1) {
          g.zf[o] = c + g.bias[n];
        } else if (g.mode == 2) {
          zf[o] = c;
        } else {
          c *= dsilu(g.zin[o]);
          g.zf[o] = c;
          g.ob[o] = f2bf(c);
        }
      }
}

// out[i] = sum_z part[z][i] in split order
__global__ void splitk_sum_kernel(const float *part, int splits, long n, float *out) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < splits; z++) s += part[(long)z * n + i];
    out[i] = s;
  }
}

void gemm(const GemmArgs &a, hipStream_t s) {
  dim3 grid((a.N + 63) / 64, (a.M + 63) / 64, a.ksplit > 1 ? a.ksplit : 1);
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, s, a);
}

// Plain GEMM (mode 2) with a long K and few output tiles (the weight gradients:
// K = batch): K is split over up to kMaxSplit blocks per tile, the partial
// products go to scratch and are summed in split order.
constexpr int kMaxSplit = 16;
void gemm_splitk(GemmArgs a, float *scratch, hipStream_t s) {
  const int tiles = ((a.N + 63) / 64) * ((a.M + 63) / 64);
  int splits = std::min(kMaxSplit, std::max(1, (a.K + 255) / 256));
  if (tiles >= 256) splits = 1;
  if (splits <= 1) {
    a.ksplit = 1;
    gemm(a, s);
    return;
  }
  float *out = a.zf;
  a.ksplit = splits;
  a.zf = scratch;
  gemm(a, s);
  const long n = (long)a.M * a.N;
  hipLaunchKernelGGL(splitk_sum_kernel, dim3((unsigned)std::min<long>((n + 255) / 256, 1024)), dim3(256), 0, s,
                     scratch, splits, n, out);
}

__global__ void to_bf16_kernel(const float *x, uint16_t *y, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = f2bf(x[i]);
}

// dY = 2 (y - t) / (3B) (fp32 and bf16) and the loss, summed by one block in a
// fixed order.
__global__ void loss_kernel(const float *y, const float *tg, int n, float *dyf, uint16_t *dyb,
                            float *loss) {
  __shared__ float red[256];
  float s = 0.f;
  const float sc = 2.0f / (float)n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const float d = y[i] - tg[i];
    s += d * d;
    const float g = sc * d;
    dyf[i] = g;
    dyb[i] = f2bf(g);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = red[0] / (float)n;
}

// db[n] = sum_b g[b][n].  A block of 256 threads takes 16 columns: thread t sums
// rows t/16, t/16 + 16, ... of column t % 16 (16 lanes read 64 contiguous bytes),
// then the 16 row phases are added in order -- a fixed summation order, and
// rows/16 independent loads per thread instead of one serial chain over rows.
__global__ __launch_bounds__(256) void colsum_kernel(const float *g, int rows, int cols, float *db) {
  __shared__ float part[16][16];
  const int c = threadIdx.x & 15, ph = threadIdx.x >> 4;
  const int n = blockIdx.x * 16 + c;
  float s = 0.f;
  if (n < cols)
    for (int b = ph; b < rows; b += 16) s += g[(long)b * cols + n];
  part[ph][c] = s;
  __syncthreads();
  if (threadIdx.x < 16 && n < cols) {
    float t = 0.f;
    for (int q = 0; q < 16; q++) t += part[q][c];
    db[n] = t;
  }
}

__global__ void adam_kernel(long n, float *p, const float *g, float *m, float *v, uint16_t *pb,
                            float lr, float b1, float b2, float eps, float c1, float c2) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (pb) pb[i] = f2bf(pi);
  }
}

struct MlpWs {
  uint16_t *xb;          // [B][7]
  float *z[3];           // [B][256] pre-activations
  uint16_t *a[3];        // [B][256] activations (bf16)
  float *y;              // [B][3] output copy
  float *gf;             // [B][256] gradient (fp32)
  uint16_t *gb[2];       // [B][256] gradient (bf16), ping-pong
  float *dyf;            // [B][3]
  uint16_t *dyb;         // [B][3]
  float *splitk;         // [kMaxSplit][256][256] partial weight gradients
  size_t bytes;
};

MlpWs layout(int B, void *base) {
  MlpWs w{};
  size_t off = 0;
  auto take = [&](size_t n) {
    const size_t o = (off + 255) & ~size_t(255);
    off = o + n;
    return reinterpret_cast<unsigned char *>(base) + o;
  };
  w.xb = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * B * kIn));
  for (int k = 0; k < 3; k++) w.z[k] = reinterpret_cast<float *>(take(sizeof(float) * B * kHid));
  for (int k = 0; k < 3; k++) w.a[k] = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * B * kHid));
  w.y = reinterpret_cast<float *>(take(sizeof(float) * B * kOut));
  w.gf = reinterpret_cast<float *>(take(sizeof(float) * B * kHid));
  for (int k = 0; k < 2; k++) w.gb[k] = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * B * kHid));
  w.dyf = reinterpret_cast<float *>(take(sizeof(float) * B * kOut));
  w.dyb = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * B * kOut));
  w.splitk = reinterpret_cast<float *>(take(sizeof(float) * kMaxSplit * kHid * kHid));
  w.bytes = (off + 255) & ~size_t(255);
  return w;
}

const int kFanIn[4] = {kIn, kHid, kHid, kHid};
const int kFanOut[4] = {kHid, kHid, kHid, kOut};

}  // namespace
}  // namespace ftlm

using namespace ftlm;

extern "C" {

int ftlm_mlp_workspace_size(int32_t batch, size_t *bytes) {
  if (batch < 1 || !bytes) {
    set_error("batch must be >= 1 and bytes non-NULL");
    return FTLM_EINVAL;
  }
  *bytes = layout(batch, nullptr).bytes;
  return FTLM_OK;
}

int ftlm_mlp_forward(const ftlm_mlp_weights *w, int32_t B, const float *x, float *y, void *ws,
                     size_t bytes, void *stream) {
  if (!w || !x || !y || !ws || B < 1) {
    set_error("NULL argument or bad batch");
    return FTLM_EINVAL;
  }
  MlpWs L = layout(B, ws);
  if (bytes < L.bytes) {
    set_error("MLP workspace too small");
    return FTLM_ENOMEM;
  }
  for (int k = 0; k < 4; k++)
    if (!w->W[k] || !w->b[k]) {
      set_error("NULL weight");
      return FTLM_EINVAL;
    }
  hipStream_t s = (hipStream_t)stream;
  const long nx = (long)B * kIn;
  hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((nx + 255) / 256 < 4096 ? (nx + 255) / 256 : 4096)),
                     dim3(256), 0, s, x, L.xb, nx);
  const uint16_t *in = L.xb;
  for (int k = 0; k < 4; k++) {
    GemmArgs g{};
    g.M = B;
    g.N = kFanOut[k];
    g.K = kFanIn[k];
    g.A = in;
    g.sam = kFanIn[k];
    g.sak = 1;
    g.B = w->W[k];
    g.sbk = kFanOut[k];
    g.sbn = 1;
    g.bias = w->b[k];
    if (k < 3) {
      g.mode = 0;
      g.zf = L.z[k];
      g.ob = L.a[k];
      in = L.a[k];
    } else {
      g.mode = 1;
      g.zf = L.y;
    }
    gemm(g, s);
  }
  if (hipMemcpyAsync(y, L.y, sizeof(float) * B * kOut, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipGetLastError() != hipSuccess) {
    set_error("MLP forward launch failed");
    return FTLM_EHIP;
  }
  return FTLM_OK;
}

int ftlm_mlp_backward(const ftlm_mlp_weights *w, int32_t B, const float *t, float *loss,
                      float *const dW[4], float *const db[4], void *ws, size_t bytes, void *stream) {
  if (!w || !t || !dW || !db || !ws || B < 1) {
    set_error("NULL argument or bad batch");
    return FTLM_EINVAL;
  }
  MlpWs L = layout(B, ws);
  if (bytes < L.bytes) {
    set_error("MLP workspace too small");
    return FTLM_ENOMEM;
  }
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, s, L.y, t, B * kOut, L.dyf, L.dyb, loss);
  // output layer
  const uint16_t *gin = L.dyb;  // gradient w.r.t. z of the current layer (bf16)
  const float *gin_f = L.dyf;
  int cur = 0;
  for (int k = 3; k >= 0; k--) {
    const uint16_t *act_prev = k > 0 ? L.a[k - 1] : L.xb;
    // dW_k = a_{k-1}^T g  ([fan_in][fan_out])
    GemmArgs gw{};
    gw.M = kFanIn[k];
    gw.N = kFanOut[k];
    gw.K = B;
    gw.A = act_prev;
    gw.sam = 1;
    gw.sak = kFanIn[k];
    gw.B = gin;
    gw.sbk = kFanOut[k];
    gw.sbn = 1;
    gw.mode = 2;
    gw.zf = dW[k];
    gemm_splitk(gw, L.splitk, s);
    hipLaunchKernelGGL(colsum_kernel, dim3((kFanOut[k] + 15) / 16), dim3(256), 0, s, gin_f, B, kFanOut[k],
                       db[k]);
    if (k == 0) break;
    // g_{k-1} = (g W_k^T) * silu'(z_{k-1})
    GemmArgs ga{};
    ga.M = B;
    ga.N = kFanIn[k];
    ga.K = kFanOut[k];
    ga.A = gin;
    ga.sam = kFanOut[k];
    ga.sak = 1;
    ga.B = w->W[k];
    ga.sbk = 1;
    ga.sbn = kFanOut[k];
    ga.mode = 3;
    ga.zin = L.z[k - 1];
    ga.zf = L.gf;
    ga.ob = L.gb[cur];
    gemm(ga, s);
    gin = L.gb[cur];
    gin_f = L.gf;
    cur ^= 1;
  }
  if (hipGetLastError() != hipSuccess) {
    set_error("MLP backward launch failed");
    return FTLM_EHIP;
  }
  return FTLM_OK;
}

int ftlm_adam_step(int64_t n, float *p, const float *grad, float *m, float *v, uint16_t *pb, float lr,
                   float beta1, float beta2, float eps, int32_t step, void *stream) {
  if (n < 1 || !p || !grad || !m || !v || step < 1) {
    set_error("bad Adam arguments");
    return FTLM_EINVAL;
  }
  const float c1 = 1.0f - std::pow(beta1, (float)step), c2 = 1.0f - std::pow(beta2, (float)step);
  const long blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (long)n, p, grad,
                     m, v, pb, lr, beta1, beta2, eps, c1, c2);
  if (hipGetLastError() != hipSuccess) {
    set_error("Adam launch failed");
    return FTLM_EHIP;
  }
  return FTLM_OK;
}

}  // extern "C"
