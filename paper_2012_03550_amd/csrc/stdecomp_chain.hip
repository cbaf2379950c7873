// gfx950 kernels of libstdecomp, the minibatch chain: one persistent
// cooperative launch runs every minibatch of (a range of) an epoch, each as
// the core sub-step followed by the N factor sub-steps of Algorithm 1
// (arXiv 2012.03550), with a grid barrier after every sub-step because each
// needs the previous one's result.
//
// The dense contraction E_p = G_(n) s_p (s_p: the row of S(n) of sample p,
// the Kronecker product of its other modes' rows) runs on MFMA in two stages.
// With lo = the lowest mode != n and the remaining modes' multi-index h:
//   stage 1 (MFMA):  Y_p[h](j_n) = sum_{j_lo} a(lo)_p[j_lo] * G_(n)[j_n, j_lo + J_lo * h]
//                    a GEMM of the gathered lo-mode rows (16 samples per tile)
//                    with the core reshaped [J_lo x J_n] for each h;
//   stage 2 (VALU):  E_p(j_n) = sum_h hp_p[h] * Y_p[h](j_n), hp_p[h] = the
//                    product of the sample's remaining rows at h.
// The core gradient sum_p r_p h_p is the GEMM
//   dG[j_0, j_lo, h] = sum_p (r_p a(0)_p[j_0] hp_p[h]) * a(lo)_p[j_lo]
// over the samples of a workgroup's chunk (MFMA, K = samples).
// FP32 mode uses v_mfma_f32_16x16x4_f32; BF16 mode rounds the operands to
// BF16 (RNE) and uses v_mfma_f32_16x16x16_bf16, accumulating in FP32, with
// BF16 read copies of the factors and FP32 masters receiving the updates.
#include "stdecomp_device.h"

namespace stdk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (unsigned short)((u >> 16) | 0x40u);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_round(float f) { return __uint_as_float((uint32_t)bf16_bits(f) << 16); }
__device__ __forceinline__ float bf16_val(unsigned short b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------------------------------
// Grid barrier: workgroup w publishes how many barriers it has reached in its
// own flag word (bar[w * kFlagStride]); wave 0 of every workgroup polls all W
// flags (one lane per flag) until each has reached the target.  No
// read-modify-write on a shared word, so arrivals do not serialise.  Every
// thread fences its global writes (agent scope) before the arrival; the wait
// has a give-up bound so a lost workgroup can never hang the device (the
// error flag then stops every workgroup).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void barrier_arrive(const ChainArgs& a, unsigned passed) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(a.bar + blockIdx.x * kFlagStride, passed, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool barrier_wait(const ChainArgs& a, unsigned passed, int* flag_lds) {
  if (threadIdx.x < 64) {
    long long spins = 0;
    int good = 1;
    for (;;) {
      bool ok = true;
      for (int v = threadIdx.x; v < a.W; v += 64)
        ok = ok && __hip_atomic_load(a.bar + v * kFlagStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= passed;
      if (__all(ok)) break;
      if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        good = 0;
        break;
      }
      if (++spins > a.spin_limit) {
        if (threadIdx.x == 0) __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0) *flag_lds = good;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *flag_lds != 0;
}

// The record (N indices, value) a lane handles in phase ph of minibatch b:
// minibatch order for the core sub-step, (row, position) order of mode ph-1
// for the factor sub-steps.  Records are read-only during the chain, so they
// are loaded before the barrier that opens the phase.
__device__ __forceinline__ void load_phase_record(const ChainArgs& a, int64_t b, int ph,
                                                  uint32_t (&rec)[kMaxOrder + 1]) {
  const int64_t base = b * a.M;
  const int m = (int)((a.T - base < a.M) ? (a.T - base) : a.M);
  const int q = blockIdx.x * a.chunk + (int)threadIdx.x;
  if ((int)threadIdx.x < a.chunk && q < m) {
    const uint32_t* src = (ph == 0) ? a.coo + (base + q) * a.s.R
                                    : a.rec_sorted + ((int64_t)(ph - 1) * a.T + base + q) * a.s.R;
#pragma unroll
    for (int w = 0; w < kMaxOrder + 1; ++w)
      if (w < a.s.R) rec[w] = src[w];
  }
}

// Copy the N rows of a sample into its LDS row buffer: all loads are issued
// before the first LDS store (the read copies: FP32 masters, or BF16).
template <int JR, bool BF>
__device__ __forceinline__ void gather_sample_rows(const ChainArgs& a, const int (&idx)[kMaxOrder], float* rb) {
  const Shape& s = a.s;
  constexpr int STAGE = JR <= 16 ? 4 : 2;  // modes staged in registers at once
  if constexpr (!BF) {
    constexpr int C4 = (JR + 3) / 4;
    for (int k0 = 0; k0 < s.N; k0 += STAGE) {
      float4 st[STAGE][C4];
#pragma unroll
      for (int kk = 0; kk < STAGE; ++kk) {
        const int k = k0 + kk;
        int row = 0;
#pragma unroll
        for (int t = 0; t < kMaxOrder; ++t)
          if (t == k) row = idx[t];
        if (k < s.N) {
          const float4* src = reinterpret_cast<const float4*>(a.A[k] + (int64_t)row * s.Jp[k]);
#pragma unroll
          for (int c = 0; c < C4; ++c)
            if (4 * c < s.J[k]) st[kk][c] = src[c];
        }
      }
#pragma unroll
      for (int kk = 0; kk < STAGE; ++kk) {
        const int k = k0 + kk;
        if (k < s.N) {
          const int J = s.J[k];
          float* dst = rb + s.rs_off[k];
#pragma unroll
          for (int c = 0; c < C4; ++c) {
            if (4 * c < J) dst[4 * c] = st[kk][c].x;
            if (4 * c + 1 < J) dst[4 * c + 1] = st[kk][c].y;
            if (4 * c + 2 < J) dst[4 * c + 2] = st[kk][c].z;
            if (4 * c + 3 < J) dst[4 * c + 3] = st[kk][c].w;
          }
        }
      }
    }
  } else {
    constexpr int C8 = (JR + 7) / 8;
    for (int k0 = 0; k0 < s.N; k0 += STAGE) {
      uint4 st[STAGE][C8];
#pragma unroll
      for (int kk = 0; kk < STAGE; ++kk) {
        const int k = k0 + kk;
        int row = 0;
#pragma unroll
        for (int t = 0; t < kMaxOrder; ++t)
          if (t == k) row = idx[t];
        if (k < s.N) {
          const uint4* src = reinterpret_cast<const uint4*>(a.Ab[k] + (int64_t)row * a.Jb[k]);
#pragma unroll
          for (int c = 0; c < C8; ++c)
            if (8 * c < s.J[k]) st[kk][c] = src[c];
        }
      }
#pragma unroll
      for (int kk = 0; kk < STAGE; ++kk) {
        const int k = k0 + kk;
        if (k < s.N) {
          const int J = s.J[k];
          float* dst = rb + s.rs_off[k];
#pragma unroll
          for (int c = 0; c < C8; ++c) {
            const uint32_t w4[4] = {st[kk][c].x, st[kk][c].y, st[kk][c].z, st[kk][c].w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int j = 8 * c + e;
              if (j < J) dst[j] = bf16_val((unsigned short)((e & 1) ? (w4[e >> 1] >> 16) : (w4[e >> 1] & 0xFFFFu)));
            }
          }
        }
      }
    }
  }
}

// Finish the rows that straddled chunk boundaries in the previous factor
// sub-step (mode pm): xr[bw] is the straddling row at boundary bw or -1;
// carry slots hold [row, count, partial sum (J), old master row (J)].
// carry_par is the LDS copy of those slots.  Fills the LDS table `split`
// (row, then the new master row at +4) and
// returns the number of entries.  If `store`, also writes the rows (master,
// and BF16 copy in BF16 mode).
template <int JR, bool EXACT, bool BF>
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
      const float v = split[en * sstride + 4 + j];
      a.A[pm][(int64_t)row * a.s.Jp[pm] + j] = v;
      if (BF) a.Ab[pm][(int64_t)row * a.Jb[pm] + j] = bf16_bits(v);
    }
  }
  return nsplit;
}

// Per-mode tiling of the two-stage contraction.
struct Tiling {
  int lo, nhi, khi;       // lowest other mode, count and product of the remaining ones
  int hi[kMaxOrder - 2];
  int hJ[kMaxOrder - 2];  // J of each remaining mode
  int hls[kMaxOrder - 2]; // its stride in the flat core
  int hrs[kMaxOrder - 2]; // its offset in an LDS row buffer
  int jlo, kp, nt;        // J_lo, J_lo padded to the MFMA K step, 16-wide j_n tiles
  int ls_n, ls_lo, rs_lo; // core strides of j_n and j_lo, row-buffer offset of the lo row
};

__device__ __forceinline__ Tiling tiling(const Shape& s, int n, bool bf) {
  const ModeTab t = mode_tab(s, n);
  Tiling g;
  g.lo = t.lo;
  g.nhi = t.nhi;
  g.khi = t.khi;
#pragma unroll
  for (int i = 0; i < kMaxOrder - 2; ++i) {
    g.hi[i] = t.hi[i];
    g.hJ[i] = i < t.nhi ? s.J[t.hi[i]] : 1;
    g.hls[i] = i < t.nhi ? s.lstride[t.hi[i]] : 0;
    g.hrs[i] = i < t.nhi ? s.rs_off[t.hi[i]] : 0;
  }
  g.ls_n = s.lstride[n];
  g.ls_lo = s.lstride[t.lo];
  g.rs_lo = s.rs_off[t.lo];
  g.jlo = s.J[t.lo];
  g.kp = bf ? ((g.jlo + 15) & ~15) : pad4(g.jlo);
  g.nt = (s.J[n] + 15) / 16;
  return g;
}

// Offsets of the remaining modes' multi-index h (mode-lowest first):
//   hmap[h]                  = sum_i digit_i(h) * lstride[hi[i]]  (offset in the flat core)
//   hmap[khi + h * nhi + i]  = rs_off[hi[i]] + digit_i(h)          (offset in a row buffer)
// One thread per h, so the table and hp fills below need no division.
__device__ __forceinline__ void build_hmap(const Tiling& g, int* hmap) {
  for (int h = threadIdx.x; h < g.khi; h += blockDim.x) {
    int hh = h, off = 0;
#pragma unroll
    for (int i = 0; i < kMaxOrder - 2; ++i) {
      if (i < g.nhi) {
        const int d = hh % g.hJ[i];
        hh /= g.hJ[i];
        off += d * g.hls[i];
        hmap[g.khi + h * g.nhi + i] = g.hrs[i] + d;
      }
    }
    hmap[h] = off;
  }
}

// B-operand table of mode n, built from the core Gs:
//   FP32: TB[((h * nt + t) * kp + k) * 16 + c]   = G_(n)[16t + c, k + J_lo h]
//   BF16: TB16[((h * nt + t) * 16 + c) * kp + k] = bf16(same)
// (zero outside j_n < J_n, k < J_lo).  A flat loop over table elements;
// each thread issues its four core reads before its four table writes (the
// two LDS arrays could alias as far as the compiler knows).
template <bool BF>
__device__ void build_tables(const Shape& s, int n, const Tiling& g, const float* Gs, const int* hmap, float* TB) {
  const int Jn = s.J[n];
  const int total = g.khi * g.nt * g.kp * 16;
  unsigned short* TB16 = reinterpret_cast<unsigned short*>(TB);
  const int BT = blockDim.x;
  for (int e0 = threadIdx.x; e0 < total; e0 += 4 * BT) {
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * BT;
      v[u] = 0.f;
      if (e < total) {
        int k, c, ht;
        if (BF) {  // e = (ht * 16 + c) * kp + k
          k = e % g.kp;
          const int r = e / g.kp;
          c = r & 15;
          ht = r >> 4;
        } else {   // e = (ht * kp + k) * 16 + c
          c = e & 15;
          const int r = e >> 4;
          k = r % g.kp;
          ht = r / g.kp;
        }
        const int h = g.nt == 1 ? ht : ht / g.nt;
        const int t = ht - h * g.nt;
        const int jn = 16 * t + c;
        if (k < g.jlo && jn < Jn) v[u] = Gs[hmap[h] + k * g.ls_lo + jn * g.ls_n];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * BT;
      if (e < total) {
        if (BF) TB16[e] = bf16_bits(v[u]);
        else TB[e] = v[u];
      }
    }
  }
}

// hp[h * chp + p] = prod over the remaining modes of the sample's rows at h
// (1 when there are none); zero for positions p >= cnt.  Reads are batched
// ahead of the writes, four h at a time.
__device__ __forceinline__ void build_hp(const Shape& s, const Tiling& g, const float* rowbuf, const int* hmap,
                                         int cnt, int chp, float* hp) {
  const int p = threadIdx.x;
  if (p >= chp) return;
  const float* rb = rowbuf + p * s.rs;
  const int* ro = hmap + g.khi;
  if (p >= cnt) {
    for (int h = 0; h < g.khi; ++h) hp[h * chp + p] = 0.f;
    return;
  }
  if (g.nhi == 0) {
    hp[p] = 1.f;
    return;
  }
  for (int h0 = 0; h0 < g.khi; h0 += 4) {
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int h = h0 + u;
      v[u] = 1.f;
      if (h < g.khi)
        for (int i = 0; i < g.nhi; ++i) v[u] *= rb[ro[h * g.nhi + i]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (h0 + u < g.khi) hp[(h0 + u) * chp + p] = v[u];
  }
}

// E_p for the chunk's samples into ebuf[p * es + j_n] (MFMA, see the file
// header).  Each wave carries two 16-sample tiles at once so that two
// independent MFMA chains overlap.
template <int JR, bool BF>
__device__ void mfma_E(const Shape& s, int n, const Tiling& g, const float* TB, const float* rowbuf,
                       const float* hp, int cnt, int chp, float* ebuf, int es) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int Jn = s.J[n];
  const int MT = (cnt + 15) >> 4;
  const int lo_off = g.rs_lo;
  const int jobs = ((MT + 1) >> 1) * g.nt;  // job = (tile pair, j_n tile)
  for (int job = wv; job < jobs; job += nwaves) {
    const int mp = job / g.nt, t = job - mp * g.nt;
    const int mt0 = 2 * mp, mt1 = 2 * mp + 1;
    const int prow0 = mt0 * 16 + r16, prow1 = mt1 * 16 + r16;
    f32x4 e0 = {0.f, 0.f, 0.f, 0.f}, e1 = {0.f, 0.f, 0.f, 0.f};
    const float* hp0 = hp + mt0 * 16 + 4 * kq;
    const float* hp1 = hp + mt1 * 16 + 4 * kq;  // within chp: chp is a multiple of 16 and covers mt1 when used
    const bool has1 = mt1 < MT;
    if constexpr (!BF) {
      constexpr int KS = (JR + 3) / 4;
      float a0[KS], a1[KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int k = 4 * ks + kq;
        a0[ks] = (prow0 < cnt && k < g.jlo) ? rowbuf[prow0 * s.rs + lo_off + k] : 0.f;
        a1[ks] = (prow1 < cnt && k < g.jlo) ? rowbuf[prow1 * s.rs + lo_off + k] : 0.f;
      }
      const int nks = g.kp >> 2;
      const float* tb = TB + (t * g.kp + kq) * 16 + r16;
      const int hstride = g.nt * g.kp * 16;
      int h = 0;
      for (; h + 1 < g.khi; h += 2) {  // two h per iteration: four independent MFMA chains
        f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
        f32x4 d0 = {0.f, 0.f, 0.f, 0.f}, d1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          if (ks < nks) {
            const float bv = tb[h * hstride + ks * 64];
            const float bw = tb[(h + 1) * hstride + ks * 64];
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[ks], bv, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[ks], bv, c1, 0, 0, 0);
            d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[ks], bw, d0, 0, 0, 0);
            d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[ks], bw, d1, 0, 0, 0);
          }
        }
        const float4 h0 = *reinterpret_cast<const float4*>(hp0 + h * chp);
        const float4 g0 = *reinterpret_cast<const float4*>(hp0 + (h + 1) * chp);
        const float4 h1 = has1 ? *reinterpret_cast<const float4*>(hp1 + h * chp) : make_float4(0.f, 0.f, 0.f, 0.f);
        const float4 g1 = has1 ? *reinterpret_cast<const float4*>(hp1 + (h + 1) * chp) : make_float4(0.f, 0.f, 0.f, 0.f);
        e0[0] = fmaf(c0[0], h0.x, e0[0]);
        e0[1] = fmaf(c0[1], h0.y, e0[1]);
        e0[2] = fmaf(c0[2], h0.z, e0[2]);
        e0[3] = fmaf(c0[3], h0.w, e0[3]);
        e1[0] = fmaf(c1[0], h1.x, e1[0]);
        e1[1] = fmaf(c1[1], h1.y, e1[1]);
        e1[2] = fmaf(c1[2], h1.z, e1[2]);
        e1[3] = fmaf(c1[3], h1.w, e1[3]);
        e0[0] = fmaf(d0[0], g0.x, e0[0]);
        e0[1] = fmaf(d0[1], g0.y, e0[1]);
        e0[2] = fmaf(d0[2], g0.z, e0[2]);
        e0[3] = fmaf(d0[3], g0.w, e0[3]);
        e1[0] = fmaf(d1[0], g1.x, e1[0]);
        e1[1] = fmaf(d1[1], g1.y, e1[1]);
        e1[2] = fmaf(d1[2], g1.z, e1[2]);
        e1[3] = fmaf(d1[3], g1.w, e1[3]);
      }
      for (; h < g.khi; ++h) {
        f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          if (ks < nks) {
            const float bv = tb[h * hstride + ks * 64];
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[ks], bv, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[ks], bv, c1, 0, 0, 0);
          }
        }
        const float4 h0 = *reinterpret_cast<const float4*>(hp0 + h * chp);
        const float4 h1 = has1 ? *reinterpret_cast<const float4*>(hp1 + h * chp) : make_float4(0.f, 0.f, 0.f, 0.f);
        e0[0] = fmaf(c0[0], h0.x, e0[0]);
        e0[1] = fmaf(c0[1], h0.y, e0[1]);
        e0[2] = fmaf(c0[2], h0.z, e0[2]);
        e0[3] = fmaf(c0[3], h0.w, e0[3]);
        e1[0] = fmaf(c1[0], h1.x, e1[0]);
        e1[1] = fmaf(c1[1], h1.y, e1[1]);
        e1[2] = fmaf(c1[2], h1.z, e1[2]);
        e1[3] = fmaf(c1[3], h1.w, e1[3]);
      }
    } else {
      constexpr int KS = (JR + 15) / 16;
      s16x4 a0[KS], a1[KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = 16 * ks + 4 * kq + e;
          a0[ks][e] = (short)bf16_bits((prow0 < cnt && k < g.jlo) ? rowbuf[prow0 * s.rs + lo_off + k] : 0.f);
          a1[ks][e] = (short)bf16_bits((prow1 < cnt && k < g.jlo) ? rowbuf[prow1 * s.rs + lo_off + k] : 0.f);
        }
      }
      const int nks = g.kp >> 4;
      const unsigned short* tb = reinterpret_cast<const unsigned short*>(TB) + (t * 16 + r16) * g.kp + 4 * kq;
      const int hstride = g.nt * 16 * g.kp;
for (int h = 0; h < g.khi; ++h) {
        f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          if (ks < nks) {
            const s16x4 bv = *reinterpret_cast<const s16x4*>(tb + h * hstride + 16 * ks);
            c0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0[ks], bv, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[ks], bv, c1, 0, 0, 0);
          }
        }
        const float4 h0 = *reinterpret_cast<const float4*>(hp0 + h * chp);
        const float4 h1 = has1 ? *reinterpret_cast<const float4*>(hp1 + h * chp) : make_float4(0.f, 0.f, 0.f, 0.f);
        e0[0] = fmaf(c0[0], h0.x, e0[0]);
        e0[1] = fmaf(c0[1], h0.y, e0[1]);
        e0[2] = fmaf(c0[2], h0.z, e0[2]);
        e0[3] = fmaf(c0[3], h0.w, e0[3]);
        e1[0] = fmaf(c1[0], h1.x, e1[0]);
        e1[1] = fmaf(c1[1], h1.y, e1[1]);
        e1[2] = fmaf(c1[2], h1.z, e1[2]);
        e1[3] = fmaf(c1[3], h1.w, e1[3]);
      }
    }
    const int jn = 16 * t + r16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p0 = mt0 * 16 + 4 * kq + i, p1 = mt1 * 16 + 4 * kq + i;
      if (p0 < cnt && jn < Jn) ebuf[p0 * es + jn] = e0[i];
      if (p1 < cnt && jn < Jn) ebuf[p1 * es + jn] = e1[i];
    }
  }
}

// partial[lin] = sum over the chunk of r_p h_p[lin], lin = j0 + J0 (j_lo + J_lo h)
// (MFMA over samples; ra[p * ras + j0] = r_p a(0)_p[j0], hp rows zero for
// p >= cnt).  Jobs are (h, j0 tile, j_lo tile); a wave carries up to three
// jobs with the same tiles and consecutive h at once, which share the A row
// and B column loads and keep three independent MFMA chains in flight.
template <bool BF>
__device__ void mfma_core_grad(const Shape& s, const Tiling& g, const float* rowbuf, const float* ra, int ras,
                               const float* hp, int cnt, int chp, float* out) {
  constexpr int JG = 3;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int J0 = s.J[0];
  const int MT0 = (J0 + 15) >> 4, NT1 = (g.jlo + 15) >> 4;
  const int lo_off = g.rs_lo;
  const int hgroups = (g.khi + JG - 1) / JG;
  const int jobs = hgroups * MT0 * NT1;
  constexpr int KSTEP = BF ? 16 : 4;
  const int nsteps = (cnt + KSTEP - 1) / KSTEP;
  for (int job = wv; job < jobs; job += nwaves) {
    const int hg = job / (MT0 * NT1);
    const int rem = job - hg * MT0 * NT1;
    const int t0 = rem / NT1, t1 = rem - t0 * NT1;
    const int j0 = 16 * t0 + r16;  // A row
    const int jl = 16 * t1 + r16;  // B column
    const bool arow = j0 < J0, bcol = jl < g.jlo;
    const int h0 = hg * JG;
    const float* hph[JG];
    bool hok[JG];
#pragma unroll
    for (int q = 0; q < JG; ++q) {
      hok[q] = h0 + q < g.khi;
      hph[q] = hp + (hok[q] ? h0 + q : h0) * chp;
    }
    f32x4 c[JG];
#pragma unroll
    for (int q = 0; q < JG; ++q) c[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (!BF) {
      // operands of step st+1 are read before the MFMAs of step st
      auto load = [&](int st, float& rav, float& bv, float (&hv)[JG]) {
        const int p = st * 4 + kq;
        rav = (arow && p < chp) ? ra[p * ras + j0] : 0.f;
        bv = (bcol && p < cnt) ? rowbuf[p * s.rs + lo_off + jl] : 0.f;
#pragma unroll
        for (int q = 0; q < JG; ++q) hv[q] = (p < chp) ? hph[q][p] : 0.f;
      };
      float rav, bv, hv[JG];
      if (nsteps > 0) load(0, rav, bv, hv);
      for (int st = 0; st < nsteps; ++st) {
        float rav2 = 0.f, bv2 = 0.f, hv2[JG];
#pragma unroll
        for (int q = 0; q < JG; ++q) hv2[q] = 0.f;
        if (st + 1 < nsteps) load(st + 1, rav2, bv2, hv2);
#pragma unroll
        for (int q = 0; q < JG; ++q) c[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(rav * hv[q], bv, c[q], 0, 0, 0);
        rav = rav2;
        bv = bv2;
#pragma unroll
        for (int q = 0; q < JG; ++q) hv[q] = hv2[q];
      }
    } else {
      for (int st = 0; st < nsteps; ++st) {
        float rav[4];
        s16x4 bv;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int p = st * 16 + 4 * kq + e;
          rav[e] = (arow && p < chp) ? ra[p * ras + j0] : 0.f;
          bv[e] = (short)bf16_bits((bcol && p < cnt) ? rowbuf[p * s.rs + lo_off + jl] : 0.f);
        }
#pragma unroll
        for (int q = 0; q < JG; ++q) {
          s16x4 av;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int p = st * 16 + 4 * kq + e;
            av[e] = (short)bf16_bits(p < chp ? rav[e] * hph[q][p] : 0.f);
          }
          c[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, c[q], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < JG; ++q) {
      if (!hok[q]) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int jr = 16 * t0 + 4 * kq + i;
        if (jr < J0 && bcol) out[jr + J0 * (jl + g.jlo * (h0 + q))] = c[q][i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The chain kernel.  Workgroup w owns positions [w*chunk, (w+1)*chunk) of
// every minibatch: in minibatch order for the core sub-step, in (row,
// position) order for the factor sub-steps.
//
// Core sub-step (dense core, once per minibatch):
//   r_p = x_p - a(0)_p . E_p;  partial_w = sum_{p in chunk} r_p h_p;
//   at the start of the next sub-step every workgroup forms the same
//   G <- G - gG * ( -(1/m) sum_w partial_w + lG * G ) (fixed order over w).
// Mode-n sub-step:
//   r_p = x_p - a(n)_p . E_p,  u_p = -r_p E_p;  F_i = sum of u_p over row i's
//   positions (segmented scan in (row, position) order, fixed tree);
//   a_i <- a_i - gA * ( F_i / c_i + lA * a_i ).
//   A row whose positions straddle chunk boundaries is finished at the start
//   of the next sub-step from the chunks' carried partial sums and the
//   carried old row (every workgroup computes it identically into an LDS
//   table; workgroup 0 stores it; until the next barrier nobody else reads it
//   from global memory).
// Carry slot: [0] row, [1] count, [2, 2+J) partial sum, [2+J, 2+2J) old row.
// ---------------------------------------------------------------------------
template <int JU, int BFI>
__global__ __launch_bounds__(kChainThreads) void k_chain(ChainArgs a) {
  constexpr int JR = JU ? JU : kMaxRank;
  constexpr bool EXACT = JU != 0;
  constexpr bool BF = BFI != 0;
  extern __shared__ float lds[];
  const Shape& s = a.s;
  const int N = s.N;
  const int P = s.P;
  const int Pp = pad4(P);
  const int tid = threadIdx.x;
  const int BT = blockDim.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int w = blockIdx.x;
  const ChainLayout& L = a.lay;

  float* Gs = lds + L.gs;
  float* TB = lds + L.tb;
  float* rowbuf = lds + L.row;
  float* hp = lds + L.hp;
  float* ebuf = lds + L.ebuf;
  float* rabuf = lds + L.ra;
  float* split = lds + L.split;
  float* cbuf = lds + L.cbuf;  // the previous phase's carry slots, copied at phase start
  int* hmap = reinterpret_cast<int*>(lds + L.hmap);
  float* wscr = lds + L.wscr;
  int* ints = reinterpret_cast<int*>(lds + L.ints);
  int* rowids = ints;                // BT
  int* segmax = rowids + BT;         // BT / 64
  int* xa = segmax + (BT >> 6);      // W   crossing rows, buffers rotated per phase
  int* xb = xa + a.W;                // W
  int* sfirst = xb + a.W;            // W
  int* misc = sfirst + a.W;          // 8
  const int chp = L.chp, es = L.es, ras = L.ras, sstride = L.sstride, wstride = L.wstride;

  for (int lin = tid; lin < P; lin += BT) Gs[lin] = a.G[lin];
  __syncthreads();

  unsigned passed = 0;
  int pm = -1;   // mode of the previous phase (-1: core sub-step or none)
  int ppar = 0;  // carry parity written by the previous phase
  int par = 0;   // carry parity of the current phase
  int* xprev = xa;
  int* xcur = xb;
  const int64_t T = a.T, M = a.M;
  const size_t carry_par_stride = (size_t)a.W * 2 * a.carry_stride;

  uint32_t rec[kMaxOrder + 1];
#pragma unroll
  for (int i = 0; i < kMaxOrder + 1; ++i) rec[i] = 0;
  if (a.b_begin < a.b_end) load_phase_record(a, a.b_begin, 0, rec);

  for (int64_t b = a.b_begin; b < a.b_end; ++b) {
    const int64_t base = b * M;
    const int m = (int)((T - base < M) ? (T - base) : M);
    const int lo = w * a.chunk;
    const int cnt = max(0, min(a.chunk, m - lo));

    for (int ph = 0; ph <= N; ++ph) {
      const int n = ph == 0 ? 0 : ph - 1;  // the mode whose unfolding this phase contracts with
      const int Jn = EXACT ? JR : s.J[n];
      const bool active = tid < cnt;
      const Tiling g = tiling(s, n, BF);

      // ---- 1. this lane's sample: record and rows (issued first: longest latency)
      int idx[kMaxOrder];
#pragma unroll
      for (int k = 0; k < kMaxOrder; ++k) idx[k] = (k < N) ? (int)rec[k] : 0;
      const float x = __uint_as_float(pick(rec, s.R - 1));
      float* rb = rowbuf + tid * s.rs;
      if (active) gather_sample_rows<JR, BF>(a, idx, rb);
      float an[JR];  // own-mode FP32 master row (the row the update starts from)
#pragma unroll
      for (int j = 0; j < JR; ++j) an[j] = 0.f;
      if (BF && active && ph > 0) {
        const float* src = a.A[n] + (int64_t)pick(idx, n) * s.Jp[n];
#pragma unroll
        for (int j = 0; j < JR; ++j)
          if (EXACT || j < Jn) an[j] = src[j];
      }
      if (ph > 0 && a.W > 1)
        for (int bw = tid; bw < a.W; bw += BT) xcur[bw] = a.xrow[((size_t)b * N + n) * a.W + bw];
      if (pm >= 0 && a.W > 1) {
        const float4* src = reinterpret_cast<const float4*>(a.carry + (size_t)ppar * carry_par_stride);
        float4* dst = reinterpret_cast<float4*>(cbuf);
        for (int i = tid; i < (int)(carry_par_stride >> 2); i += BT) dst[i] = src[i];
      }

      // ---- 2. core: finish the core step of this minibatch (same in every workgroup)
      if (ph == 1) {
        const float inv_m = 1.0f / (float)m;
        const int P4 = Pp >> 2;
        const float4* src = reinterpret_cast<const float4*>(a.partial);
        for (int l4 = tid; l4 < P4; l4 += BT) {
          float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 16
          for (int v = 0; v < a.W; ++v) {
            const float4 t4 = src[(size_t)v * P4 + l4];
            sum.x += t4.x;
            sum.y += t4.y;
            sum.z += t4.z;
            sum.w += t4.w;
          }
          const float sv[4] = {sum.x, sum.y, sum.z, sum.w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int lin = 4 * l4 + i;
            if (lin < P) {
              const float gv = Gs[lin];
              Gs[lin] = gv - a.gG * (-sv[i] * inv_m + a.lG * gv);
            }
          }
        }
        __syncthreads();
      }

      // ---- 3. rows of the previous factor sub-step that straddled chunks
      if (pm >= 0 && a.W > 1) {
        const int nsplit = finish_split_rows<JR, EXACT, BF>(a, pm, xprev, cbuf, split, sstride, sfirst, misc, w == 0);
        if (active && nsplit > 0) {
          // the table follows the chunk boundaries, so its rows are increasing
          const int pJ = s.J[pm];
          const int prow = pick(idx, pm);
          int lo2 = 0, hi2 = nsplit;
          while (lo2 < hi2) {
            const int mid = (lo2 + hi2) >> 1;
            if (__float_as_int(split[mid * sstride]) < prow) lo2 = mid + 1;
            else hi2 = mid;
          }
          if (lo2 < nsplit && __float_as_int(split[lo2 * sstride]) == prow) {
            for (int j = 0; j < pJ; ++j) {
              const float v = split[lo2 * sstride + 4 + j];
              rb[s.rs_off[pm] + j] = BF ? bf16_round(v) : v;
            }
          }
        }
      }
      // own-mode master row in FP32 mode is the gathered row
      __syncthreads();
      // ---- 4. contraction tables of this phase's mode, E_p for every sample
      build_hmap(g, hmap);
      __syncthreads();
      build_tables<BF>(s, n, g, Gs, hmap, TB);
      build_hp(s, g, rowbuf, hmap, cnt, chp, hp);
      __syncthreads();
      mfma_E<JR, BF>(s, n, g, TB, rowbuf, hp, cnt, chp, ebuf, es);
      {  // the next phase's record (read-only; its load overlaps the rest of this phase)
        int64_t nbb = b;
        int nph = ph + 1;
        if (nph > N) {
          nph = 0;
          ++nbb;
        }
        if (nbb < a.b_end) load_phase_record(a, nbb, nph, rec);
      }
      __syncthreads();

      if (ph == 0) {
        // ================= core sub-step =================
        if (tid < chp) {
          float r = 0.f;
          if (active) {
            float xh = 0.f;
#pragma unroll
            for (int j = 0; j < JR; ++j)
              if (EXACT || j < Jn) xh = fmaf(rb[s.rs_off[0] + j], ebuf[tid * es + j], xh);
            r = x - xh;
          }
#pragma unroll
          for (int j = 0; j < JR; ++j)
            if (EXACT || j < Jn) rabuf[tid * ras + j] = active ? r * rb[s.rs_off[0] + j] : 0.f;
        }
        // (the core-gradient tiles reuse hp of mode 0: the remaining modes of mode 1's columns)
        const Tiling g0 = tiling(s, 0, BF);
        __syncthreads();
        mfma_core_grad<BF>(s, g0, rowbuf, rabuf, ras, hp, cnt, chp, a.partial + (size_t)w * Pp);
      } else {
        // ================= mode-n sub-step =================
        float u[JR];
#pragma unroll
        for (int j = 0; j < JR; ++j) u[j] = 0.f;
        const int row = active ? pick(idx, n) : -1;
        if (active) {
          float xh = 0.f;
#pragma unroll
          for (int j = 0; j < JR; ++j) {
            if (EXACT || j < Jn) {
              const float e = ebuf[tid * es + j];
              if (!BF) an[j] = rb[s.rs_off[n] + j];
              xh = fmaf(rb[s.rs_off[n] + j], e, xh);
              u[j] = e;
            }
          }
          const float r = x - xh;
#pragma unroll
          for (int j = 0; j < JR; ++j)
            if (EXACT || j < Jn) u[j] = -r * u[j];
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
          const bool before = (sf == 0) && a.W > 1 && xcur[w] >= 0;                          // run began earlier
          const bool after = (tid == cnt - 1) && a.W > 1 && w + 1 < a.W && xcur[w + 1] >= 0;  // run goes on
          if (!before && !after) {
            float* arow = a.A[n] + (int64_t)row * s.Jp[n];
            unsigned short* brow = BF ? a.Ab[n] + (int64_t)row * a.Jb[n] : nullptr;
            const float inv_c = 1.0f / (float)c;
#pragma unroll
            for (int j = 0; j < JR; ++j) {
              if (EXACT || j < Jn) {
                const float v = an[j] - a.gA * (u[j] * inv_c + a.lA * an[j]);
                arow[j] = v;
                if (BF) brow[j] = bf16_bits(v);
              }
            }
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
      // ---- 5. barrier: the next sub-step needs this one's result
      passed += 1;
      barrier_arrive(a, passed);
      if (!barrier_wait(a, passed, misc + 7)) return;
      pm = ph - 1;  // -1 after the core sub-step
      ppar = par;
      par ^= 1;
      int* tmp = xprev;
      xprev = xcur;
      xcur = tmp;
    }
  }
  // ---- flush: rows of the last factor sub-step that straddled chunks
  if (pm >= 0 && a.W > 1 && w == 0) {
    const float4* src = reinterpret_cast<const float4*>(a.carry + (size_t)ppar * carry_par_stride);
    float4* dst = reinterpret_cast<float4*>(cbuf);
    for (int i = tid; i < (int)(carry_par_stride >> 2); i += BT) dst[i] = src[i];
    __syncthreads();
    finish_split_rows<JR, EXACT, BF>(a, pm, xprev, cbuf, split, sstride, sfirst, misc, true);
  }
  if (w == 0)
    for (int lin = tid; lin < P; lin += BT) a.G[lin] = Gs[lin];
}

// LDS plan of the chain (floats; every region starts on 16 bytes).
size_t plan_chain_lds(ChainArgs& a, int threads, bool bf) {
  const Shape& s = a.s;
  // every region below is sized from these: refuse an incomplete request
  if (a.W < 1 || a.chunk < 1 || a.chunk > threads || (a.W > 1 && (a.carry_stride < 4 || a.split_cap < a.W - 1)))
    return 0;
  const int JU = chain_variant(s);
  const int JR = JU ? JU : kMaxRank;
  auto al = [](size_t f) { return (f + 3) & ~(size_t)3; };
  ChainLayout& L = a.lay;
  int jmax = 0;
  size_t tb = 0, khimax = 1;
  for (int n = 0; n < s.N; ++n) {
    jmax = s.J[n] > jmax ? s.J[n] : jmax;
    const int lo = n == 0 ? 1 : 0;
    const int jlo = s.J[lo];
    const size_t khi = (size_t)s.P / s.J[n] / jlo;
    const int nt = (s.J[n] + 15) / 16;
    const size_t kp = bf ? (size_t)((jlo + 15) & ~15) : (size_t)pad4(jlo);
    const size_t f = bf ? (khi * nt * 16 * kp + 1) / 2 : khi * nt * kp * 16;
    tb = f > tb ? f : tb;
    khimax = khi > khimax ? khi : khimax;
  }
  L.chp = (a.chunk + 15) & ~15;
  L.es = 16 * ((jmax + 15) / 16) + 1;
  L.ras = pad4(JR) + 1;
  L.sstride = 4 + pad4(JR);
  L.wstride = pad4(JR) + 4;
  size_t off = 0;
  L.gs = (int)off;    off += al(s.P);
  L.tb = (int)off;    off += al(tb);
  L.row = (int)off;   off += al((size_t)threads * s.rs);
  L.hp = (int)off;    off += al(khimax * L.chp);
  L.ebuf = (int)off;  off += al((size_t)L.chp * L.es);
  L.ra = (int)off;    off += al((size_t)L.chp * L.ras);
  L.split = (int)off; off += al((size_t)a.split_cap * L.sstride);
  L.cbuf = (int)off;  off += al(a.W > 1 ? (size_t)a.W * 2 * a.carry_stride : 0);
  L.hmap = (int)off;  off += al(khimax * (size_t)(s.N > 2 ? s.N - 1 : 1));
  L.wscr = (int)off;  off += al((size_t)(threads / 64) * L.wstride);
  L.ints = (int)off;  off += threads + threads / 64 + 3 * a.W + 8;
  L.total = (int)off;
  return off * 4;
}

size_t chain_lds_bytes(const ChainArgs& a, int threads) { return (size_t)a.lay.total * 4; }

hipError_t launch_chain(const ChainArgs& a, int threads, hipStream_t st) {
  const int var = chain_variant(a.s);
  const size_t bytes = (size_t)a.lay.total * 4;
  {  // the plan must be the one these arguments produce
    ChainArgs chk = a;
    if (plan_chain_lds(chk, threads, a.bf16 != 0) != bytes || chk.lay.cbuf != a.lay.cbuf || chk.lay.ints != a.lay.ints)
      return hipErrorInvalidValue;
  }
  hipError_t e = hipSuccess;
  ChainArgs args = a;
  void* params[] = {&args};
  if (a.bf16) {
    STDK_FOR_VARIANT(var, {
      e = hipFuncSetAttribute((const void*)k_chain<JU, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      if (e == hipSuccess)
        e = hipLaunchCooperativeKernel((const void*)k_chain<JU, 1>, dim3(a.W), dim3(threads), params, (unsigned)bytes,
                                       st);
    });
  } else {
    STDK_FOR_VARIANT(var, {
      e = hipFuncSetAttribute((const void*)k_chain<JU, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      if (e == hipSuccess)
        e = hipLaunchCooperativeKernel((const void*)k_chain<JU, 0>, dim3(a.W), dim3(threads), params, (unsigned)bytes,
                                       st);
    });
  }
  return e;
}

}  // namespace stdk
