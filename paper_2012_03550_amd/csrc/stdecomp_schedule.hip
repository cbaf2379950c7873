// gfx950 kernels of libstdecomp, schedule side: the epoch sample order
// (sampler), the per-minibatch row sets of every mode (sort), and packing of
// COO entries into device records.  All integer work; results are
// bit-identical to the definitions they implement.
#include "stdecomp_device.h"

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
                                                       int* __restrict__ xrow, int* __restrict__ nseg,
                                                       uint32_t* __restrict__ rec_sorted, uint32_t* __restrict__ meta,
                                                       int64_t T, int64_t M, int64_t b_begin, int R, int N, int W,
                                                       int chunk) {
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
  // Run metadata for the chain (thread tid holds the sorted positions
  // [tid*ITEMS, (tid+1)*ITEMS) in k[]): the start of each position's row run
  // is the last head at or before it, a block-wide max-scan.
  {
    __shared__ int wtot[kSortThreads / 64];
    const int out0 = tid * ITEMS;
    const int lane = tid & 63, wv = tid >> 6;
    const unsigned long long before_key = out0 > 0 ? keys[out0 - 1] : ~0ull;
    const unsigned long long after_key = out0 + ITEMS < CAP ? keys[out0 + ITEMS] : ~0ull;
    int last = -1;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int pos = out0 + i;
      const unsigned long long pk = (i == 0) ? before_key : k[i - 1];
      if (pos < m && (pos == 0 || (pk >> 16) != (k[i] >> 16))) last = pos;
    }
    int incl = last;
    for (int d = 1; d < 64; d <<= 1) {
      const int o = __shfl_up(incl, d);
      if (lane >= d) incl = max(incl, o);
    }
    if (lane == 63) wtot[wv] = incl;
    __syncthreads();
    int st = __shfl_up(incl, 1);
    if (lane == 0) st = -1;
    for (int v = 0; v < wv; ++v) st = max(st, wtot[v]);
    uint32_t* mt = meta + (int64_t)(n + 1) * T + base;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int pos = out0 + i;
      if (pos < m) {
        const unsigned long long pk = (i == 0) ? before_key : k[i - 1];
        const unsigned long long nk = (i + 1 < ITEMS) ? k[i + 1] : after_key;
        if (pos == 0 || (pk >> 16) != (k[i] >> 16)) st = pos;
        const int qlo = (pos / chunk) * chunk;
        const int sf = max(st, qlo) - qlo;
        const bool next_same = pos + 1 < m && (nk >> 16) == (k[i] >> 16);
        const bool chunk_end = pos + 1 == qlo + chunk;
        int v = sf;
        if (!next_same || chunk_end) v |= kMetaTail;
        if (sf == 0 && st < qlo) v |= kMetaBefore;
        if (chunk_end && next_same) v |= kMetaAfter;
        mt[pos] = (uint32_t)v;
      }
    }
  }
  uint16_t* out = sigma + (int64_t)n * T + base;
  if (tid == 0) heads = 0;
  __syncthreads();
  int my_heads = 0;
  uint32_t* rs_out = rec_sorted + ((int64_t)n * T + base) * R;
  for (int q = tid; q < m; q += kSortThreads) {
    const int p = (int)(keys[q] & 0xFFFFull);
    out[q] = (uint16_t)p;
    my_heads += (q == 0 || (keys[q] >> 16) != (keys[q - 1] >> 16)) ? 1 : 0;
    const uint32_t* src = coo + (base + p) * R;
    for (int w = 0; w < R; ++w) rs_out[(int64_t)q * R + w] = src[w];
  }
  atomicAdd(&heads, my_heads);  // integer count: order does not matter
  __syncthreads();
  if (tid == 0) nseg[b * N + n] = heads;
  // Chunk boundaries of the chain: the row that straddles boundary bw (the
  // positions bw*chunk - 1 and bw*chunk share it) or -1; then, for the first
  // boundary of each straddling row, its entry number; then their count.
  if (W > 1) {
    int* xr = xrow + ((size_t)b * N + n) * xrow_stride(W);
    auto straddle = [&](int bw) {
      const int q = bw * chunk;
      if (bw > 0 && q < m) {
        const unsigned long long r0 = keys[q - 1] >> 16, r1 = keys[q] >> 16;
        if (r0 == r1) return (int)r1;
      }
      return -1;
    };
    for (int bw = tid; bw < W; bw += kSortThreads) xr[bw] = straddle(bw);
    if (tid == 0) {
      int cnt = 0, prev = -1;
      for (int bw = 0; bw < W; ++bw) {
        const int v = straddle(bw);
        xr[W + bw] = (v >= 0 && v != prev) ? cnt++ : -1;
        prev = v;
      }
      xr[2 * W] = cnt;
    }
  }
}

// Which entry of the previous phase's straddling-row table patches each
// position: phase ph finishes the rows of mode pm (updated by the phase
// before it) that straddled chunk boundaries; a position whose mode-pm row is
// one of them gets 1 + its entry number in bits 16-23 of its metadata word.
// One block per (minibatch, phase); runs after the sort of every mode.
__global__ __launch_bounds__(kSortThreads) void k_patch(const uint32_t* __restrict__ coo,
                                                        const uint32_t* __restrict__ rec_sorted,
                                                        const int* __restrict__ xrow, uint32_t* __restrict__ meta,
                                                        int64_t T, int64_t M, int64_t b_begin, int R, int N, int W) {
  __shared__ int ent_row[1024];
  __shared__ int nent;
  const int64_t b = b_begin + blockIdx.x;
  const int ph = blockIdx.y;
  const int64_t base = b * M;
  const int m = (int)((T - base < M) ? (T - base) : M);
  const int pm = ph == 0 ? N - 1 : ph - 2;  // phase 1 follows the core sub-step: nothing to finish
  const int64_t bp = ph == 0 ? b - 1 : b;
  const bool any = W > 1 && pm >= 0 && bp >= 0;
  if (threadIdx.x == 0) nent = 0;
  __syncthreads();
  if (any) {
    const int* xr = xrow + ((size_t)bp * N + pm) * xrow_stride(W);
    for (int bw = threadIdx.x; bw < W; bw += kSortThreads) {
      const int e = xr[W + bw];
      if (e >= 0 && e < 1024) ent_row[e] = xr[bw];
    }
    if (threadIdx.x == 0) nent = min(xr[2 * W], 1024);
  }
  __syncthreads();
  const int ne = nent;
  uint32_t* mt = meta + (int64_t)ph * T + base;
  for (int q = threadIdx.x; q < m; q += kSortThreads) {
    int code = 0;
    if (ne > 0) {
      const uint32_t* rec = ph == 0 ? coo + (base + q) * R : rec_sorted + ((int64_t)(ph - 1) * T + base + q) * R;
      const int row = (int)rec[pm];
      int lo = 0, hi = ne;  // entries follow the boundaries, so their rows increase
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ent_row[mid] < row) lo = mid + 1;
        else hi = mid;
      }
      if (lo < ne && ent_row[lo] == row) code = (lo + 1) << kMetaPatchShift;
    }
    if (ph == 0) mt[q] = (uint32_t)code;  // the core phase has no run metadata
    else if (ph >= 2) mt[q] |= (uint32_t)code;
  }
}

hipError_t launch_sort(const Shape& s, const uint32_t* coo_perm, uint16_t* sigma, int* xrow, int* nseg,
                       uint32_t* rec_sorted, uint32_t* meta, int W, int chunk, int64_t T, int64_t M,
                       int64_t b_begin, int64_t b_end, hipStream_t st) {
  const int64_t nb = b_end - b_begin;
  if (nb <= 0) return hipSuccess;
  for (int64_t b0 = 0; b0 < nb; b0 += 65535) {
    const int g = (int)((nb - b0 < 65535) ? nb - b0 : 65535);
    dim3 grid(g, s.N);
    if (M <= 1024) {
      hipLaunchKernelGGL(k_sort<4>, grid, dim3(kSortThreads), 1024 * 8, st, coo_perm, sigma, xrow, nseg, rec_sorted, meta, T, M, b_begin + b0, s.R, s.N, W, chunk);
    } else if (M <= 4096) {
      hipLaunchKernelGGL(k_sort<16>, grid, dim3(kSortThreads), 4096 * 8, st, coo_perm, sigma, xrow, nseg, rec_sorted, meta, T, M, b_begin + b0, s.R, s.N, W, chunk);
    } else {
      hipError_t e = hipFuncSetAttribute((const void*)k_sort<64>, hipFuncAttributeMaxDynamicSharedMemorySize, 16384 * 8);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_sort<64>, grid, dim3(kSortThreads), 16384 * 8, st, coo_perm, sigma, xrow, nseg, rec_sorted, meta, T, M, b_begin + b0, s.R, s.N, W, chunk);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (s.N + 1 > 65535) return hipErrorInvalidValue;
  for (int64_t b0 = 0; b0 < nb; b0 += 65535) {
    const int g = (int)((nb - b0 < 65535) ? nb - b0 : 65535);
    hipLaunchKernelGGL(k_patch, dim3(g, s.N + 1), dim3(kSortThreads), 0, st, coo_perm, rec_sorted, xrow, meta, T, M,
                       b_begin + b0, s.R, s.N, W);
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


}  // namespace stdk
