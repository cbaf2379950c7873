// gfx950 kernels of libstdecomp: the SGD_Tucker minibatch update
// (arXiv 2012.03550) for sparse Tucker decomposition on one MI355X.
//
//   k_perm_gather  epoch order pi_e of the training entries (sampler) and the
//                  gather of the COO records into that order
//   k_sort         per minibatch and mode, the positions sorted by (row, position),
//                  i.e. the row sets (Psi_M^(n))_{i_n} of Eq. SGD_factor_matrix
//   k_chain        persistent cooperative kernel: for every minibatch the core
//                  sub-step and the N factor sub-steps of Algorithm 1, separated
//                  by grid barriers (each sub-step needs the previous one's result)
//   k_loss/predict model values x_hat and FP64 RMSE/MAE sums (Section
//                  "Experimental Settings")
//
// Layout: factor matrices A(n) are FP32 row-major I_n x Jp_n (rows padded to
// 16 bytes); the core G is flat with j_0 fastest (the vectorisation of the
// mode-1 unfolding); COO records are N int32 indices followed by the float
// value.  No kernel uses floating-point atomics: every reduction has a fixed
// order, so results are bit-reproducible run to run.
#include "stdecomp_internal.h"

namespace stdk {

// ---------------------------------------------------------------------------
// Sampler: a keyed permutation of [0, T) per epoch.  A 4-round balanced
// Feistel network on 2h-bit words (Luby-Rackoff) whose round function is the
// SplitMix64 output function (Steele, Lea and Flood 2014) of the right half
// xor the round key, restricted to [0, T) by cycle walking (Black and Rogaway
// 2002).  Round key r of epoch e: mix(seed ^ mix(4e + r)).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct FeistelKey {
  uint64_t k[4];
  int h;
};

__device__ __forceinline__ FeistelKey make_key(uint64_t seed, int64_t epoch, int64_t T) {
  FeistelKey fk;
  int h = 1;
  while (h < 31 && (1ull << (2 * h)) < (uint64_t)T) ++h;
  fk.h = h;
#pragma unroll
  for (int r = 0; r < 4; ++r) fk.k[r] = mix64(seed ^ mix64((uint64_t)(4 * epoch + r)));
  return fk;
}

__device__ __forceinline__ uint64_t feistel_encrypt(uint64_t x, const FeistelKey& fk) {
  const uint64_t mask = (1ull << fk.h) - 1;
  uint64_t left = x >> fk.h, right = x & mask;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint64_t f = mix64(right ^ fk.k[r]) & mask;
    const uint64_t nr = left ^ f;
    left = right;
    right = nr;
  }
  return (left << fk.h) | right;
}

__device__ __forceinline__ uint64_t epoch_entry(uint64_t q, uint64_t T, const FeistelKey& fk) {
  uint64_t y = feistel_encrypt(q, fk);
  while (y >= T) y = feistel_encrypt(y, fk);  // cycle walk: ends, the map is a bijection
  return y;
}

__global__ void k_perm_gather(const uint32_t* __restrict__ coo, uint32_t* __restrict__ out, int64_t T, int R,
                              uint64_t seed, int64_t epoch) {
  const FeistelKey fk = make_key(seed, epoch, T);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < T; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = (int64_t)epoch_entry((uint64_t)q, (uint64_t)T, fk);
    const uint32_t* src = coo + t * R;
    uint32_t* dst = out + q * R;
    for (int w = 0; w < R; ++w) dst[w] = src[w];
  }
}

__global__ void k_perm_only(int64_t* __restrict__ out, int64_t T, uint64_t seed, int64_t epoch) {
  const FeistelKey fk = make_key(seed, epoch, T);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < T; q += (int64_t)gridDim.x * blockDim.x)
    out[q] = (int64_t)epoch_entry((uint64_t)q, (uint64_t)T, fk);
}

static int grid_for(int64_t n, int threads, int cap = 65536) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

hipError_t launch_perm_gather(const Shape& s, const uint32_t* coo, uint32_t* coo_perm, int64_t T, uint64_t seed,
                              int64_t epoch, hipStream_t st) {
  hipLaunchKernelGGL(k_perm_gather, dim3(grid_for(T, 256)), dim3(256), 0, st, coo, coo_perm, T, s.R, seed, epoch);
  return hipGetLastError();
}

hipError_t launch_perm_only(int64_t T, uint64_t seed, int64_t epoch, int64_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_perm_only, dim3(grid_for(T, 256)), dim3(256), 0, st, out, T, seed, epoch);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Row sets of a minibatch: positions sorted by the key (row i_n, position).
// The key is unique, so the order is unique.  One workgroup per (minibatch,
// mode): keys sorted in registers (bitonic network), then merged pairwise in
// LDS along merge paths.  Output sigma[n*T + b*M + q] = q-th position.
// ---------------------------------------------------------------------------
template <int ITEMS>
__global__ __launch_bounds__(kSortThreads) void k_sort(const uint32_t* __restrict__ coo, uint16_t* __restrict__ sigma,
                                                       int* __restrict__ xrow, int* __restrict__ nseg, int64_t T,
                                                       int64_t M, int64_t b_begin, int R, int N, int W, int chunk) {
  extern __shared__ unsigned long long keys[];
  __shared__ int heads;
  const int64_t b = b_begin + blockIdx.x;
  const int n = blockIdx.y;
  const int64_t base = b * M;
  const int m = (int)((T - base < M) ? (T - base) : M);
  constexpr int CAP = kSortThreads * ITEMS;
  const int tid = threadIdx.x;
  unsigned long long k[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const int pos = tid * ITEMS + i;
    k[i] = (pos < m) ? (((unsigned long long)coo[(base + pos) * R + n] << 16) | (unsigned)pos) : ~0ull;
  }
#pragma unroll
  for (int kk = 2; kk <= ITEMS; kk <<= 1) {
#pragma unroll
    for (int j = kk >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & kk) == 0;
          const unsigned long long x = k[i], y = k[l];
          if ((x > y) == up) {
            k[i] = y;
            k[l] = x;
          }
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) keys[tid * ITEMS + i] = k[i];
  __syncthreads();
  for (int w = ITEMS; w < CAP; w <<= 1) {
    const int out0 = tid * ITEMS;
    const int base2 = out0 & ~(2 * w - 1);
    const int diag = out0 - base2;
    const unsigned long long* pa = keys + base2;
    const unsigned long long* pb = keys + base2 + w;
    int lo = diag - w > 0 ? diag - w : 0;
    int hi = diag < w ? diag : w;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (pa[mid] < pb[diag - 1 - mid]) lo = mid + 1;
      else hi = mid;
    }
    int ai = lo, bi = diag - lo;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const bool take_a = (ai < w) && (bi >= w || pa[ai] < pb[bi]);
      if (take_a) k[i] = pa[ai++];
      else k[i] = pb[bi++];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) keys[out0 + i] = k[i];
    __syncthreads();
  }
  uint16_t* out = sigma + (int64_t)n * T + base;
  if (tid == 0) heads = 0;
  __syncthreads();
  int my_heads = 0;
  for (int q = tid; q < m; q += kSortThreads) {
    out[q] = (uint16_t)(keys[q] & 0xFFFFull);
    my_heads += (q == 0 || (keys[q] >> 16) != (keys[q - 1] >> 16)) ? 1 : 0;
  }
  atomicAdd(&heads, my_heads);  // integer count: order does not matter
  __syncthreads();
  if (tid == 0) nseg[b * N + n] = heads;
  // Chunk boundaries of the chain: the row that straddles boundary bw (the
  // positions bw*chunk - 1 and bw*chunk share it), or -1.
  if (W > 1) {
    int* xr = xrow + ((size_t)b * N + n) * W;
    for (int bw = tid; bw < W; bw += kSortThreads) {
      const int q = bw * chunk;
      int v = -1;
      if (bw > 0 && q < m) {
        const unsigned long long r0 = keys[q - 1] >> 16, r1 = keys[q] >> 16;
        if (r0 == r1) v = (int)r1;
      }
      xr[bw] = v;
    }
  }
}

hipError_t launch_sort(const Shape& s, const uint32_t* coo_perm, uint16_t* sigma, int* xrow, int* nseg, int W,
                       int chunk, int64_t T, int64_t M, int64_t b_begin, int64_t b_end, hipStream_t st) {
  const int64_t nb = b_end - b_begin;
  if (nb <= 0) return hipSuccess;
  for (int64_t b0 = 0; b0 < nb; b0 += 65535) {
    const int g = (int)((nb - b0 < 65535) ? nb - b0 : 65535);
    dim3 grid(g, s.N);
    if (M <= 1024) {
      hipLaunchKernelGGL(k_sort<4>, grid, dim3(kSortThreads), 1024 * 8, st, coo_perm, sigma, xrow, nseg, T, M, b_begin + b0, s.R, s.N, W, chunk);
    } else if (M <= 4096) {
      hipLaunchKernelGGL(k_sort<16>, grid, dim3(kSortThreads), 4096 * 8, st, coo_perm, sigma, xrow, nseg, T, M, b_begin + b0, s.R, s.N, W, chunk);
    } else {
      hipError_t e = hipFuncSetAttribute((const void*)k_sort<64>, hipFuncAttributeMaxDynamicSharedMemorySize, 16384 * 8);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_sort<64>, grid, dim3(kSortThreads), 16384 * 8, st, coo_perm, sigma, xrow, nseg, T, M, b_begin + b0, s.R, s.N, W, chunk);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Row of the q-th position of minibatch b in the (row, position) order of mode n.
__device__ __forceinline__ int sorted_row(const uint32_t* coo, const uint16_t* sigma, int64_t T, int64_t base, int R,
                                          int n, int q) {
  const int p = sigma[(int64_t)n * T + base + q];
  return (int)coo[(base + p) * R + n];
}

// Segment starts of one (minibatch, mode): where the row changes along the
// sorted order.  Debug export for the bit-exactness tests; the chain kernel
// applies the same rule on the fly.
__global__ void k_debug_segments(const uint32_t* coo, const uint16_t* sigma, int64_t T, int64_t M, int64_t b, int n,
                                 int R, int32_t* seg_off, int32_t* seg_row, int32_t* nseg) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const int64_t base = b * M;
  const int m = (int)((T - base < M) ? (T - base) : M);
  int d = 0, prev = -1;
  for (int q = 0; q < m; ++q) {
    const int row = sorted_row(coo, sigma, T, base, R, n, q);
    if (q == 0 || row != prev) {
      seg_off[d] = q;
      seg_row[d] = row;
      ++d;
    }
    prev = row;
  }
  seg_off[d] = m;
  *nseg = d;
}

hipError_t launch_debug_segments(const Shape& s, const uint32_t* coo_perm, const uint16_t* sigma, int64_t T, int64_t M,
                                 int64_t b, int mode, int32_t* seg_off, int32_t* seg_row, int32_t* nseg,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_debug_segments, dim3(1), dim3(64), 0, st, coo_perm, sigma, T, M, b, mode, s.R, seg_off, seg_row,
                     nseg);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Shared per-sample machinery: one lane per sample.  The sample's N factor
// rows sit in an LDS row buffer (stride s.rs, odd); the mode-n unfolded core
// G_(n)^T sits in LDS as a [K_n][gts] table (the columns of S(n) in the order
// of Eq. optimization_for_factor: lowest other mode fastest).
// ---------------------------------------------------------------------------
struct ModeTab {  // per-mode column decomposition: lowest other mode, then the rest
  int lo;               // lowest mode != n
  int nhi;              // number of remaining modes
  int hi[kMaxOrder - 2];
  int khi;              // prod of J over the remaining modes
};

__device__ __forceinline__ ModeTab mode_tab(const Shape& s, int n) {
  ModeTab t;
  t.lo = (n == 0) ? 1 : 0;
  t.nhi = 0;
  t.khi = 1;
#pragma unroll
  for (int i = 0; i < kMaxOrder - 2; ++i) t.hi[i] = 0;
#pragma unroll
  for (int k = 0; k < kMaxOrder; ++k) {
    if (k < s.N && k != n && k != t.lo) {
#pragma unroll
      for (int i = 0; i < kMaxOrder - 2; ++i)
        if (i == t.nhi) t.hi[i] = k;
      t.nhi++;
      t.khi *= s.J[k];
    }
  }
  return t;
}

// GT[col * gts + j] = G_(n)[j, col] (zero for j >= J_n), built from the core Gs.
__device__ void build_gt(const Shape& s, int n, const float* Gs, float* GT, int gts) {
  const ModeTab t = mode_tab(s, n);
  const int Jn = s.J[n];
  const int Jlo = s.J[t.lo];
  const int K = s.P / Jn;
  int lstride[kMaxOrder];
  int acc = 1;
#pragma unroll
  for (int k = 0; k < kMaxOrder; ++k) {
    lstride[k] = acc;
    if (k < s.N) acc *= s.J[k];
  }
  for (int e = threadIdx.x; e < K * gts; e += blockDim.x) {
    const int col = e / gts, j = e - col * gts;
    float v = 0.f;
    if (j < Jn) {
      int c = col;
      int lin = j * lstride[n] + (c % Jlo) * lstride[t.lo];
      c /= Jlo;
#pragma unroll
      for (int i = 0; i < kMaxOrder - 2; ++i) {
        if (i < t.nhi) {
          const int Jk = s.J[t.hi[i]];
          lin += (c % Jk) * lstride[t.hi[i]];
          c /= Jk;
        }
      }
      v = Gs[lin];
    }
    GT[e] = v;
  }
}

// E[j] = sum_col G_(n)[j, col] * s[col]: the row E_p of E(n) = G_(n) S(n)^T
// for one sample, with s built on the fly as a Kronecker product of the
// sample's rows of the other modes (Algorithm 1, factor loop: cache_S, cache_E).
template <int JR, bool EXACT>
__device__ __forceinline__ void compute_E(const Shape& s, int n, const float* GT, int gts, const float* rb,
                                          float (&E)[JR]) {
  const ModeTab t = mode_tab(s, n);
  const int Jn = s.J[n];
  const int Jlo = s.J[t.lo];
  const int lo_off = s.rs_off[t.lo];
#pragma unroll
  for (int j = 0; j < JR; ++j) E[j] = 0.f;
  int jh[kMaxOrder - 2];
#pragma unroll
  for (int i = 0; i < kMaxOrder - 2; ++i) jh[i] = 0;
  const float* gt = GT;
  for (int h = 0; h < t.khi; ++h) {
    float hp = 1.f;
#pragma unroll
    for (int i = 0; i < kMaxOrder - 2; ++i)
      if (i < t.nhi) hp *= rb[s.rs_off[t.hi[i]] + jh[i]];
    for (int jl = 0; jl < Jlo; ++jl) {
      const float sv = hp * rb[lo_off + jl];
#pragma unroll
      for (int j = 0; j < JR; ++j)
        if (EXACT || j < Jn) E[j] = fmaf(gt[j], sv, E[j]);
      gt += gts;
    }
#pragma unroll
    for (int i = 0; i < kMaxOrder - 2; ++i) {
      if (i < t.nhi) {
        if (++jh[i] < s.J[t.hi[i]]) break;
        jh[i] = 0;
      }
    }
  }
}

// Record of entry e: N indices then the value.
__device__ __forceinline__ float load_record(const uint32_t* rec, int R, int N, int (&idx)[kMaxOrder]) {
#pragma unroll
  for (int k = 0; k < kMaxOrder; ++k) idx[k] = (k < N) ? (int)rec[k] : 0;
  return __uint_as_float(rec[R - 1]);
}

// Copy the N rows of a sample into its LDS row buffer.  Rows of mode `pm`
// listed in the split table (rows finalised at the start of this phase) are
// taken from the table instead of global memory.
__device__ __forceinline__ void gather_rows(const Shape& s, float* const* A, const int (&idx)[kMaxOrder], float* rb,
                                            int pm, const float* split, int nsplit, int sstride) {
#pragma unroll
  for (int k = 0; k < kMaxOrder; ++k) {
    if (k >= s.N) break;
    const float* src = A[k] + (int64_t)idx[k] * s.Jp[k];
    if (k == pm) {
      for (int e = 0; e < nsplit; ++e) {
        if (__float_as_int(split[e * sstride]) == idx[k]) {
          src = split + e * sstride + 4;
          break;
        }
      }
    }
    const int J = s.J[k];
    float* dst = rb + s.rs_off[k];
    for (int j4 = 0; j4 < J; j4 += 4) {
      const float4 v = *reinterpret_cast<const float4*>(src + j4);
      dst[j4] = v.x;
      if (j4 + 1 < J) dst[j4 + 1] = v.y;
      if (j4 + 2 < J) dst[j4 + 2] = v.z;
      if (j4 + 3 < J) dst[j4 + 3] = v.w;
    }
  }
}

// ---------------------------------------------------------------------------
// Grid barrier of the chain: a monotonically increasing arrival counter.
// Every thread fences its global writes (agent scope) before arrival; thread 0
// waits for all W workgroups, with a give-up bound so that a lost workgroup
// can never hang the device (the error flag then stops every workgroup).
// ---------------------------------------------------------------------------
__device__ bool grid_sync(const ChainArgs& a, unsigned& passed, int* flag_lds) {
  passed += 1;
  const unsigned target = passed * (unsigned)a.W;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    int good = 1;
    __hip_atomic_fetch_add(a.bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    long long spins = 0;
    while (__hip_atomic_load(a.bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        good = 0;
        break;
      }
      if (++spins > a.spin_limit) {
        __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    *flag_lds = good;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *flag_lds != 0;
}

// ---------------------------------------------------------------------------
// The chain.  Workgroup w owns positions [w*chunk, (w+1)*chunk) of every
// minibatch: in minibatch order for the core sub-step, in (row, position)
// order for the factor sub-steps.  Each sub-step ends with a grid barrier.
//
// Core sub-step (dense core; once per minibatch):
//   r_p = x_p - a(0)_p . (G_(0) s_p);  partial_w = sum_{p in chunk} r_p h_p
//   next phase, in every workgroup (same data, same order, same result):
//   G <- G - gG * ( -(1/m) sum_w partial_w + lG * G )
// Mode-n sub-step:
//   E_p = G_(n) s_p,  r_p = x_p - a(n)_p . E_p,  u_p = -r_p E_p;
//   F_i = sum of u_p over row i's positions (segmented scan, fixed order);
//   a_i <- a_i - gA * ( F_i / c_i + lA * a_i ).
//   A row whose positions straddle chunk boundaries is finished at the start
//   of the next phase from the chunks' carried partial sums and the carried
//   old row (every workgroup computes it identically into an LDS table;
//   workgroup 0 stores it).  Until the following barrier nobody else reads
//   that row from global memory.
// Carry slot: [0] row, [1] count, [2, 2+J) partial sum, [2+J, 2+2J) old row.
// ---------------------------------------------------------------------------

// Finish the rows that straddled chunk boundaries in the previous factor
// sub-step (mode pm).  xr[bw] is the straddling row at boundary bw or -1.
// Fills the LDS table `split` (row, then the new row values at +4) and
// returns the number of entries.  If `store`, also writes the rows.
template <int JR, bool EXACT>
__device__ int finish_split_rows(const ChainArgs& a, int pm, const int* xr, const float* carry_par, float* split,
                                 int sstride, int* sfirst, int* misc, bool store) {
  const int tid = threadIdx.x, BT = blockDim.x;
  const int pJ = a.s.J[pm];
  if (tid < 64) {  // number the first boundary of every straddling row (wave 0, ballots)
    int ns = 0;
    for (int b0 = 0; b0 < a.W; b0 += 64) {
      const int bw = b0 + tid;
      const bool first = bw >= 1 && bw < a.W && xr[bw] >= 0 && xr[bw - 1] != xr[bw];
      const unsigned long long mask = __ballot(first);
      const int before = __popcll(mask & ((1ull << tid) - 1ull));
      if (bw < a.W) sfirst[bw] = first ? ns + before : -1;
      ns += __popcll(mask);
    }
    if (tid == 0) misc[0] = ns;
  }
  __syncthreads();
  const int nsplit = misc[0];
  for (int bw = tid + 1; bw < a.W; bw += BT) {
    const int e = sfirst[bw];
    if (e < 0) continue;
    const int row = xr[bw];
    const float* slotB = carry_par + ((size_t)(bw - 1) * 2 + 1) * a.carry_stride;
    float F[JR];
    int c = __float_as_int(slotB[1]);
#pragma unroll
    for (int j = 0; j < JR; ++j) F[j] = (EXACT || j < pJ) ? slotB[2 + j] : 0.f;
    for (int v = bw; v < a.W && xr[v] == row; ++v) {
      const float* slotA = carry_par + ((size_t)v * 2 + 0) * a.carry_stride;
      c += __float_as_int(slotA[1]);
#pragma unroll
      for (int j = 0; j < JR; ++j)
        if (EXACT || j < pJ) F[j] += slotA[2 + j];
    }
    float* ent = split + e * sstride;
    ent[0] = __int_as_float(row);
    const float inv_c = 1.0f / (float)c;
#pragma unroll
    for (int j = 0; j < JR; ++j) {
      if (EXACT || j < pJ) {
        const float old = slotB[2 + pJ + j];
        ent[4 + j] = old - a.gA * (F[j] * inv_c + a.lA * old);
      }
    }
  }
  __syncthreads();
  if (store) {
    for (int e = tid; e < nsplit * pJ; e += BT) {
      const int en = e / pJ, j = e - en * pJ;
      const int row = __float_as_int(split[en * sstride]);
      a.A[pm][(int64_t)row * a.s.Jp[pm] + j] = split[en * sstride + 4 + j];
    }
  }
  return nsplit;
}

__device__ __forceinline__ int align4(int f) { return (f + 3) & ~3; }

template <int JU>
__global__ __launch_bounds__(kChainThreads) void k_chain(ChainArgs a) {
  constexpr int JR = JU ? JU : kMaxRank;
  constexpr bool EXACT = JU != 0;
  extern __shared__ float lds[];
  const Shape& s = a.s;
  const int N = s.N;
  const int P = s.P;
  const int tid = threadIdx.x;
  const int BT = blockDim.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int nwaves = BT >> 6;
  const int w = blockIdx.x;

  // ---- LDS carve-up (floats; every region starts on 16 bytes) ----
  const int ras = pad4(JR) + 1;
  const int sstride = 4 + pad4(JR);
  const int wstride = pad4(JR) + 4;
  float* Gs = lds;
  float* GT = Gs + align4(P);
  float* rowbuf = GT + align4(a.gt_floats);
  float* rabuf = rowbuf + align4(BT * s.rs);
  float* gscr = rabuf + align4(BT * ras);
  float* split = gscr + align4(a.grad_groups * P);
  float* wscr = split + align4(a.split_cap * sstride);
  int* ints = reinterpret_cast<int*>(wscr + align4(nwaves * wstride));
  int* rowids = ints;           // BT
  int* segmax = rowids + BT;    // nwaves
  int* xa = segmax + nwaves;    // W   crossing rows, two buffers swapped per phase
  int* xb = xa + a.W;           // W
  int* sfirst = xb + a.W;       // W
  int* misc = sfirst + a.W;     // 8

  for (int lin = tid; lin < P; lin += BT) Gs[lin] = a.G[lin];
  __syncthreads();

  unsigned passed = 0;
  int pm = -1;   // mode of the previous phase (-1: core sub-step or none)
  int ppar = 0;  // carry parity written by the previous phase
  int par = 0;   // carry parity of the current phase
  int* xprev = xa;
  int* xcur = xb;
  const int64_t T = a.T, M = a.M;
  const int R = s.R;
  const size_t carry_par_stride = (size_t)a.W * 2 * a.carry_stride;

  for (int64_t b = a.b_begin; b < a.b_end; ++b) {
    const int64_t base = b * M;
    const int m = (int)((T - base < M) ? (T - base) : M);
    const int lo = w * a.chunk;
    const int cnt = max(0, min(a.chunk, m - lo));

    for (int ph = 0; ph <= N; ++ph) {
      // ---- 1. finish the rows of the previous factor sub-step that straddled chunks
      int nsplit = 0;
      if (pm >= 0 && a.W > 1)
        nsplit = finish_split_rows<JR, EXACT>(a, pm, xprev, a.carry + (size_t)ppar * carry_par_stride, split,
                                              sstride, sfirst, misc, w == 0);

      if (ph == 0) {
        // ================= core sub-step =================
        const int J0 = EXACT ? JR : s.J[0];
        const int gts = pad4(J0);
        build_gt(s, 0, Gs, GT, gts);
        __syncthreads();
        if (tid < cnt) {
          const int p = lo + tid;
          int idx[kMaxOrder];
          const float x = load_record(a.coo + (base + p) * R, R, N, idx);
          float* rb = rowbuf + tid * s.rs;
          gather_rows(s, a.A, idx, rb, pm, split, nsplit, sstride);
          float E[JR];
          compute_E<JR, EXACT>(s, 0, GT, gts, rb, E);
          float xh = 0.f;
#pragma unroll
          for (int j = 0; j < JR; ++j)
            if (EXACT || j < J0) xh = fmaf(rb[s.rs_off[0] + j], E[j], xh);
          const float r = x - xh;
#pragma unroll
          for (int j = 0; j < JR; ++j)
            if (EXACT || j < J0) rabuf[tid * ras + j] = r * rb[s.rs_off[0] + j];
        }
        __syncthreads();
        // partial_w[lin] = sum_{p in chunk} r_p h_p[lin], lin = j0 + J0 * col
        {
          const ModeTab t = mode_tab(s, 0);
          const int K0 = P / J0;
          const int G = a.grad_groups;
          const int per = (cnt + G - 1) / G;
          const int Jlo = s.J[t.lo];
          for (int item = tid; item < K0 * G; item += BT) {
            const int col = item % K0, g = item / K0;
            int c = col;
            const int offlo = s.rs_off[t.lo] + c % Jlo;
            c /= Jlo;
            int offhi[kMaxOrder - 2];
#pragma unroll
            for (int i = 0; i < kMaxOrder - 2; ++i) {
              offhi[i] = 0;
              if (i < t.nhi) {
                const int Jk = s.J[t.hi[i]];
                offhi[i] = s.rs_off[t.hi[i]] + c % Jk;
                c /= Jk;
              }
            }
            float acc[JR];
#pragma unroll
            for (int j = 0; j < JR; ++j) acc[j] = 0.f;
            const int q0 = g * per, q1 = min(cnt, q0 + per);
            for (int q = q0; q < q1; ++q) {
              const float* rbq = rowbuf + q * s.rs;
              float sv = rbq[offlo];
#pragma unroll
              for (int i = 0; i < kMaxOrder - 2; ++i)
                if (i < t.nhi) sv *= rbq[offhi[i]];
              const float* ra = rabuf + q * ras;
#pragma unroll
              for (int j = 0; j < JR; ++j)
                if (EXACT || j < J0) acc[j] = fmaf(ra[j], sv, acc[j]);
            }
            float* dst = gscr + g * P + col * J0;
#pragma unroll
            for (int j = 0; j < JR; ++j)
              if (EXACT || j < J0) dst[j] = acc[j];
          }
          __syncthreads();
          float* out = a.partial + (size_t)w * P;
          for (int lin = tid; lin < P; lin += BT) {
            float v = 0.f;
            for (int g = 0; g < G; ++g) v += gscr[g * P + lin];
            out[lin] = v;
          }
        }
      } else {
        // ================= mode-n sub-step =================
        const int n = ph - 1;
        const int Jn = EXACT ? JR : s.J[n];
        const int gts = pad4(Jn);
        if (n == 0) {  // finish the core step of this minibatch (same in every workgroup)
          const float inv_m = 1.0f / (float)m;
          for (int lin = tid; lin < P; lin += BT) {
            float sum = 0.f;
            for (int v = 0; v < a.W; ++v) sum += a.partial[(size_t)v * P + lin];
            const float g = Gs[lin];
            Gs[lin] = g - a.gG * (-sum * inv_m + a.lG * g);
          }
          __syncthreads();
        }
        build_gt(s, n, Gs, GT, gts);
        if (a.W > 1)
          for (int bw = tid; bw < a.W; bw += BT) xcur[bw] = a.xrow[((size_t)b * N + n) * a.W + bw];
        __syncthreads();
        const bool active = tid < cnt;
        float u[JR], an[JR];
#pragma unroll
        for (int j = 0; j < JR; ++j) {
          u[j] = 0.f;
          an[j] = 0.f;
        }
        int row = -1;
        if (active) {
          const int p = a.sigma[(int64_t)n * T + base + lo + tid];
          int idx[kMaxOrder];
          const float x = load_record(a.coo + (base + p) * R, R, N, idx);
          float* rb = rowbuf + tid * s.rs;
          gather_rows(s, a.A, idx, rb, pm, split, nsplit, sstride);
          float E[JR];
          compute_E<JR, EXACT>(s, n, GT, gts, rb, E);
          float xh = 0.f;
#pragma unroll
          for (int j = 0; j < JR; ++j) {
            if (EXACT || j < Jn) {
              an[j] = rb[s.rs_off[n] + j];
              xh = fmaf(an[j], E[j], xh);
            }
          }
          const float r = x - xh;
#pragma unroll
          for (int j = 0; j < JR; ++j)
            if (EXACT || j < Jn) u[j] = -r * E[j];
          row = idx[n];
          rowids[tid] = row;
        }
        __syncthreads();
        // chunk-local segment heads; sf = first chunk position of my row's run
        const bool head = active && (tid == 0 || rowids[tid - 1] != row);
        int sf = head ? tid : 0;
        for (int d = 1; d < 64; d <<= 1) {
          const int o = __shfl_up(sf, d);
          if (lane >= d) sf = max(sf, o);
        }
        if (lane == 63) segmax[wv] = sf;
        __syncthreads();
        for (int v = 0; v < wv; ++v) sf = max(sf, segmax[v]);
        // wave-level segmented inclusive scan of u (Hillis-Steele, fixed order)
        const int wstart = max(sf, wv * 64) - wv * 64;
        for (int d = 1; d < 64; d <<= 1) {
          const bool take = (lane - d) >= wstart;
#pragma unroll
          for (int j = 0; j < JR; ++j) {
            if (EXACT || j < Jn) {
              const float o = __shfl_up(u[j], d);
              if (take) u[j] += o;
            }
          }
        }
        if (lane == 63) {
#pragma unroll
          for (int j = 0; j < JR; ++j)
            if (EXACT || j < Jn) wscr[wv * wstride + j] = u[j];
        }
        __syncthreads();
        // the tails of earlier waves that my run covers
        for (int v = wv - 1; v >= 0 && v * 64 + 63 >= sf; --v) {
#pragma unroll
          for (int j = 0; j < JR; ++j)
            if (EXACT || j < Jn) u[j] += wscr[v * wstride + j];
        }
        const bool tail = active && (tid == cnt - 1 || rowids[tid + 1] != row);
        if (tail) {
          const int c = tid - sf + 1;
          const bool before = (sf == 0) && a.W > 1 && xcur[w] >= 0;              // run began in an earlier chunk
          const bool after = (tid == cnt - 1) && a.W > 1 && w + 1 < a.W && xcur[w + 1] >= 0;  // run goes on
          if (!before && !after) {
            float* arow = a.A[n] + (int64_t)row * s.Jp[n];
            const float inv_c = 1.0f / (float)c;
#pragma unroll
            for (int j = 0; j < JR; ++j)
              if (EXACT || j < Jn) arow[j] = an[j] - a.gA * (u[j] * inv_c + a.lA * an[j]);
          } else {
            float* slot = a.carry + (size_t)par * carry_par_stride + ((size_t)w * 2 + (before ? 0 : 1)) * a.carry_stride;
            slot[0] = __int_as_float(row);
            slot[1] = __int_as_float(c);
#pragma unroll
            for (int j = 0; j < JR; ++j) {
              if (EXACT || j < Jn) {
                slot[2 + j] = u[j];
                slot[2 + Jn + j] = an[j];
              }
            }
          }
        }
      }
      // ---- 3. barrier: the next sub-step needs this one's result
      if (!grid_sync(a, passed, misc + 7)) return;
      pm = ph - 1;  // -1 after the core sub-step
      ppar = par;
      par ^= 1;
      int* tmp = xprev;
      xprev = xcur;
      xcur = tmp;
    }
  }
  // ---- flush: rows of the last factor sub-step that straddled chunks
  if (pm >= 0 && a.W > 1 && w == 0)
    finish_split_rows<JR, EXACT>(a, pm, xprev, a.carry + (size_t)ppar * carry_par_stride, split, sstride, sfirst,
                                 misc, true);
  if (w == 0)
    for (int lin = tid; lin < P; lin += BT) a.G[lin] = Gs[lin];
}

#define STDK_FOR_VARIANT(JUV, CALL)                 \
  switch (JUV) {                                    \
    case 2: { constexpr int JU = 2; CALL; } break;  \
    case 3: { constexpr int JU = 3; CALL; } break;  \
    case 4: { constexpr int JU = 4; CALL; } break;  \
    case 5: { constexpr int JU = 5; CALL; } break;  \
    case 6: { constexpr int JU = 6; CALL; } break;  \
    case 8: { constexpr int JU = 8; CALL; } break;  \
    case 10: { constexpr int JU = 10; CALL; } break; \
    case 12: { constexpr int JU = 12; CALL; } break; \
    case 16: { constexpr int JU = 16; CALL; } break; \
    default: { constexpr int JU = 0; CALL; } break; \
  }

int chain_variant(const Shape& s) {
  const int j0 = s.J[0];
  for (int k = 1; k < s.N; ++k)
    if (s.J[k] != j0) return 0;
  switch (j0) {
    case 2: case 3: case 4: case 5: case 6: case 8: case 10: case 12: case 16: return j0;
    default: return 0;
  }
}

static size_t chain_lds_floats(const ChainArgs& a, int threads, int JU) {
  const int JR = JU ? JU : kMaxRank;
  const int nwaves = threads / 64;
  auto al = [](size_t f) { return (f + 3) & ~(size_t)3; };
  size_t f = 0;
  f += al(a.s.P);
  f += al(a.gt_floats);
  f += al((size_t)threads * a.s.rs);
  f += al((size_t)threads * (pad4(JR) + 1));
  f += al((size_t)a.grad_groups * a.s.P);
  f += al((size_t)a.split_cap * (4 + pad4(JR)));
  f += al((size_t)nwaves * (pad4(JR) + 4));
  f += threads + nwaves + 3 * a.W + 8;  // ints
  return f;
}

size_t chain_lds_bytes(const ChainArgs& a, int threads) {
  return chain_lds_floats(a, threads, chain_variant(a.s)) * 4;
}

hipError_t launch_chain(const ChainArgs& a, int threads, hipStream_t st) {
  const int var = chain_variant(a.s);
  const size_t bytes = chain_lds_floats(a, threads, var) * 4;
  hipError_t e = hipSuccess;
  ChainArgs args = a;
  void* params[] = {&args};
  STDK_FOR_VARIANT(var, {
    e = hipFuncSetAttribute((const void*)k_chain<JU>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess)
      e = hipLaunchCooperativeKernel((const void*)k_chain<JU>, dim3(a.W), dim3(threads), params, (unsigned)bytes, st);
  });
  return e;
}

// ---------------------------------------------------------------------------
// COO packing of caller-supplied entries (SoA indices + values) into records,
// with an index range check (bad -> *bad = 1).
// ---------------------------------------------------------------------------
__global__ void k_pack(Shape s, const int32_t* __restrict__ idx, const float* __restrict__ vals, int64_t n,
                       uint32_t* __restrict__ rec, int* bad) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    for (int k = 0; k < s.N; ++k) {
      const int32_t v = idx[(int64_t)k * n + t];
      if (v < 0 || (int64_t)v >= s.I[k]) *bad = 1;
      rec[t * s.R + k] = (uint32_t)v;
    }
    rec[t * s.R + s.N] = vals ? __float_as_uint(vals[t]) : 0u;
  }
}

hipError_t launch_pack_records(const Shape& s, const int32_t* idx, const float* vals, int64_t n, uint32_t* rec,
                               int* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_pack, dim3(grid_for(n, 256)), dim3(256), 0, st, s, idx, vals, n, rec, bad);
  return hipGetLastError();
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

hipError_t launch_to_bf16(const float* src, uint16_t* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace stdk
