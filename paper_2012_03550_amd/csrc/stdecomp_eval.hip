// gfx950 kernels of libstdecomp, evaluation side: model values x_hat for
// a set of entries (Definition "Sparse Tucker Decomposition") and the FP64
// RMSE / MAE sums of Section "Experimental Settings"; reductions used by the
// runtime (sums of squares, non-finite checks) and FP32 -> BF16 copies.
#include "stdecomp_device.h"

namespace stdk {

static int grid_for(int64_t n, int threads, int cap = 65536) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

int chain_variant(const Shape& s) {
  const int j0 = s.J[0];
  for (int k = 1; k < s.N; ++k)
    if (s.J[k] != j0) return 0;
  switch (j0) {
    case 2: case 3: case 4: case 5: case 6: case 8: case 10: case 12: case 16: case 20: return j0;
    default: return 0;
  }
}

// ---------------------------------------------------------------------------
// Model values and FP64 error sums over a set of records.
// ---------------------------------------------------------------------------
template <int JU>
__global__ __launch_bounds__(256) void k_eval(Shape s, const uint32_t* __restrict__ rec, int64_t n, FactorPtrs Aptr,
                                              const float* __restrict__ G, float* __restrict__ out,
                                              double* __restrict__ block_out) {
  constexpr int JR = JU ? JU : kMaxRank;
  constexpr bool EXACT = JU != 0;
  extern __shared__ float lds[];
  const int tid = threadIdx.x, BT = blockDim.x;
  const int gts = EXACT ? pad4(JR) : pad4(s.J[0]);
  const int K0 = s.P / s.J[0];
  float* Gs = lds;
  float* GT = Gs + ((s.P + 3) & ~3);
  float* rowbuf = GT + ((K0 * gts + 3) & ~3);
  double* red = reinterpret_cast<double*>(rowbuf + ((BT * s.rs + 3) & ~3));
  float* A[kMaxOrder];
#pragma unroll
  for (int k = 0; k < kMaxOrder; ++k) A[k] = (k < s.N) ? const_cast<float*>(Aptr.A[k]) : nullptr;
  for (int lin = tid; lin < s.P; lin += BT) Gs[lin] = G[lin];
  __syncthreads();
  build_gt(s, 0, Gs, GT, gts);
  __syncthreads();
  const int J0 = EXACT ? JR : s.J[0];
  double sse = 0.0, sae = 0.0, bad = 0.0;
  float* rb = rowbuf + tid * s.rs;
  for (int64_t t = (int64_t)blockIdx.x * BT + tid; t < n; t += (int64_t)gridDim.x * BT) {
    int idx[kMaxOrder];
    const float x = load_record(rec + t * s.R, s.R, s.N, idx);
    gather_rows(s, A, idx, rb, -1, nullptr, 0, 0);
    float E[JR];
    compute_E<JR, EXACT>(s, 0, GT, gts, rb, E);
    float xh = 0.f;
#pragma unroll
    for (int j = 0; j < JR; ++j)
      if (EXACT || j < J0) xh = fmaf(rb[s.rs_off[0] + j], E[j], xh);
    if (out) out[t] = xh;
    const double r = (double)x - (double)xh;
    if (!isfinite(r)) bad += 1.0;
    sse += r * r;
    sae += fabs(r);
  }
  if (block_out) {
    red[tid] = sse;
    red[BT + tid] = sae;
    red[2 * BT + tid] = bad;
    __syncthreads();
    for (int st = BT / 2; st > 0; st >>= 1) {
      if (tid < st) {
        red[tid] += red[tid + st];
        red[BT + tid] += red[BT + tid + st];
        red[2 * BT + tid] += red[2 * BT + tid + st];
      }
      __syncthreads();
    }
    if (tid == 0) {
      block_out[blockIdx.x * 3 + 0] = red[0];
      block_out[blockIdx.x * 3 + 1] = red[BT];
      block_out[blockIdx.x * 3 + 2] = red[2 * BT];
    }
  }
}

__global__ void k_sum_blocks(const double* __restrict__ block_out, int nblocks, double* __restrict__ out3) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = 0; i < nblocks; ++i) {
    a += block_out[i * 3 + 0];
    b += block_out[i * 3 + 1];
    c += block_out[i * 3 + 2];
  }
  out3[0] = a;
  out3[1] = b;
  out3[2] = c;
}

static size_t eval_lds_bytes(const Shape& s, int threads) {
  const int JU = chain_variant(s);
  const int gts = JU ? pad4(JU) : pad4(s.J[0]);
  auto al = [](size_t f) { return (f + 3) & ~(size_t)3; };
  size_t f = al(s.P) + al((size_t)(s.P / s.J[0]) * gts) + al((size_t)threads * s.rs);
  return f * 4 + (size_t)threads * 3 * 8;
}

static hipError_t launch_eval(const Shape& s, const uint32_t* rec, int64_t n, FactorPtrs A, const float* G,
                              float* out, double* block_out, int nblocks, hipStream_t st) {
  const int threads = 256;
  const size_t bytes = eval_lds_bytes(s, threads);
  hipError_t e = hipSuccess;
  STDK_FOR_VARIANT(chain_variant(s), {
    e = hipFuncSetAttribute((const void*)k_eval<JU>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_eval<JU>, dim3(nblocks), dim3(threads), bytes, st, s, rec, n, A, G, out, block_out);
      e = hipGetLastError();
    }
  });
  return e;
}

hipError_t launch_predict(const Shape& s, const uint32_t* rec, int64_t n, FactorPtrs A, const float* G, float* out,
                          int nblocks, hipStream_t st) {
  return launch_eval(s, rec, n, A, G, out, nullptr, nblocks, st);
}

hipError_t launch_loss(const Shape& s, const uint32_t* rec, int64_t n, FactorPtrs A, const float* G,
                       double* block_out, int nblocks, double* out3, hipStream_t st) {
  hipError_t e = launch_eval(s, rec, n, A, G, nullptr, block_out, nblocks, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_blocks, dim3(1), dim3(64), 0, st, block_out, nblocks, out3);
  return hipGetLastError();
}

// Per-block FP64 sums of squares (fixed tree order), for the L2 terms of the objective.
__global__ __launch_bounds__(256) void k_sumsq(const float* __restrict__ p, int64_t n, double* __restrict__ block_out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += (double)p[i] * (double)p[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_out[blockIdx.x] = red[0];
}

hipError_t launch_sumsq(const float* p, int64_t n, double* block_out, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(k_sumsq, dim3(nblocks), dim3(256), 0, st, p, n, block_out);
  return hipGetLastError();
}

__global__ void k_nonfinite(const float* __restrict__ p, int64_t n, int* flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(p[i])) *flag = 1;
}

// p[0..n) = v (a kernel, not a memset node, so that captured graphs replay it).
__global__ void k_fill_i32(int* p, int v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_i32(int* p, int v, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256, 1024)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_count_nonfinite(const float* p, int64_t n, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_nonfinite, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, p, n, flag);
  return hipGetLastError();
}

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t to_bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
  const uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

__global__ void k_to_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = to_bf16_rne(src[i]);
}

__global__ void k_rows_to_bf16(const float* __restrict__ src, int sstride, uint16_t* __restrict__ dst, int dstride,
                               int64_t rows, int cols) {
  const int64_t n = rows * dstride;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / dstride;
    const int c = (int)(i - r * dstride);
    dst[i] = c < cols ? to_bf16_rne(src[r * sstride + c]) : (uint16_t)0;
  }
}

hipError_t launch_rows_to_bf16(const float* src, int sstride, uint16_t* dst, int dstride, int64_t rows, int cols,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_rows_to_bf16, dim3(grid_for(rows * dstride, 256, 8192)), dim3(256), 0, st, src, sstride, dst,
                     dstride, rows, cols);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* src, uint16_t* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace stdk
