// Device helpers shared by the gfx950 kernels of libstdecomp.
#pragma once
#include "stdecomp_internal.h"

namespace stdk {

__device__ __forceinline__ int align4(int f) { return (f + 3) & ~3; }

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
__device__ inline void build_gt(const Shape& s, int n, const float* Gs, float* GT, int gts) {
  const ModeTab t = mode_tab(s, n);
  const int Jn = s.J[n];
  const int Jlo = s.J[t.lo];
  const int K = s.P / Jn;
  const int* lstride = s.lstride;
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

// v[i] for a runtime i without indexing a register array dynamically.
template <int L, typename T>
__device__ __forceinline__ T pick(const T (&v)[L], int i) {
  T r = v[0];
#pragma unroll
  for (int k = 1; k < L; ++k)
    if (k == i) r = v[k];
  return r;
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


// Kernel variants: the common rank when every mode has the same J_n (a
// register-resident specialisation), else 0 (generic, J_n <= 32).
#define STDK_FOR_VARIANT(JUV, CALL)                  \
  switch (JUV) {                                     \
    case 2: { constexpr int JU = 2; CALL; } break;   \
    case 3: { constexpr int JU = 3; CALL; } break;   \
    case 4: { constexpr int JU = 4; CALL; } break;   \
    case 5: { constexpr int JU = 5; CALL; } break;   \
    case 6: { constexpr int JU = 6; CALL; } break;   \
    case 8: { constexpr int JU = 8; CALL; } break;   \
    case 10: { constexpr int JU = 10; CALL; } break; \
    case 12: { constexpr int JU = 12; CALL; } break; \
    case 16: { constexpr int JU = 16; CALL; } break; \
    case 20: { constexpr int JU = 20; CALL; } break; \
    default: { constexpr int JU = 0; CALL; } break;  \
  }

}  // namespace stdk
