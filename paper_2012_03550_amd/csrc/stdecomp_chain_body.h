// Device code of the minibatch chain, shared by the translation units that
// instantiate its kernels (stdecomp_chain.hip: the plain and Kruskal-core
// kernels and the host planner; stdecomp_chain_mom.hip: the kernels with
// heavy-ball momentum, compiled beside them).
//
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
//
// Latency plan of a sub-step (one workgroup of four waves per chunk, so
// every dependent round trip to memory is exposed):
//   * the rows a sub-step reads are loaded during the previous sub-step and
//     parked in registers, except the rows of the modes updated by the two
//     previous sub-steps; those, the previous sub-step's carried partial sums
//     and the core partials are read in one batch after the barrier;
//   * the B-operand tables of every mode depend only on the core and are
//     rebuilt once per minibatch (right after the core update) when they fit
//     in LDS; the index maps they need are built on the host;
//   * the run structure of the (row, position) order (run starts, last
//     positions, runs crossing chunk boundaries and their numbering) comes
//     with the schedule, so the factor sub-step needs no search for it.
#pragma once
#include <algorithm>
#include <vector>

#include "stdecomp_device.h"

namespace stdk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Zero words after the LDS row buffer: the MFMA K steps of the contraction
// read up to 31 words past a sample's lo-mode row (multiplied by zero table
// rows), so everything they can reach must hold finite values.
constexpr int kRowTail = 32;

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  // round to nearest even (gfx950 converts in hardware, NaN stays NaN)
  return __builtin_bit_cast(unsigned short, (__bf16)f);
}
__device__ __forceinline__ float bf16_val(unsigned short b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------------------------------
// Grid barrier: workgroup w publishes how many barriers it has reached in its
// own flag word; wave 0 of every workgroup polls all W flags (one lane per
// flag, device-scope loads, which miss the L1) until each has reached the
// target.  No read-modify-write on a shared word, so arrivals do not
// serialise.  Each wave waits until its own global writes have completed, the
// workgroup synchronises, and thread 0 publishes them all with one flag
// store; on the other side the polling wave acquires once at agent scope
// (which invalidates the L1) and the workgroup barrier hands that on to the
// other waves.  The wait has a give-up bound so a lost workgroup can never
// hang the device (the error flag then stops every workgroup).  Arrival and
// wait are separate calls so that work which reads nothing the other
// workgroups write can run in between.
//
// Two releases.  Workgroups spread over the XCCs (a.xid < 0; flags kFlagStride
// words apart) publish with an agent-scope release store, which first writes
// this XCC's L2 back to memory so that the other XCCs can read what the
// workgroup wrote.  When every workgroup runs on one XCC (a.xid >= 0; flags
// packed, workgroup w's at bar[w]) they share one L2, where their writes meet:
// a completed store (vmcnt) has reached it, as the L1 writes through, so the
// flag is a plain store and nothing is written back; the chain's data then
// stays in that L2 from one sub-step to the next.  (The acquire cannot be
// narrowed to the L1 alone: `buffer_inv sc0` leaves stale L1 lines outside the
// split-workgroup mode, which the barrier check, k_barrier_check, detects.)
// ---------------------------------------------------------------------------
// s_waitcnt operand (gfx9 encoding) that waits for vmcnt(0) only: vector memory
// counter 0 (bits 3:0 and 15:14), export and LDS/scalar counters at their maxima.
constexpr int kWaitVmcnt0 = 0x0F70;
// On one XCC the flags are packed (workgroup w's at bar[w]) so that one wave's
// poll of all W is one request, and the placement claim of chain_workgroup
// sits in the last word of the flag buffer.
__device__ __forceinline__ constexpr int kClaim(int W) { return W * kFlagStride - 1; }

// XL: the one-XCC form (a compile-time choice, so that the spread kernels
// carry no trace of it).
template <bool XL>
__device__ __forceinline__ void barrier_arrive(const ChainArgs& a, int w, unsigned passed) {
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  __syncthreads();
  if (threadIdx.x == 0) {
    if constexpr (XL)
      __hip_atomic_store(a.bar + w, passed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else
      __hip_atomic_store(a.bar + w * kFlagStride, passed, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <bool XL>
__device__ __forceinline__ bool barrier_wait(const ChainArgs& a, unsigned passed, int* flag_lds) {
  if (threadIdx.x < 64) {
    constexpr int fs = XL ? 1 : kFlagStride;  // flag stride: packed on one XCC
    long long spins = 0;
    int good = 1;
    for (;;) {
      bool ok = true;
      for (int v = threadIdx.x; v < a.W; v += 64)
        ok = ok && __hip_atomic_load(a.bar + v * fs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= passed;
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
  return *flag_lds != 0;
}

// The XCC this wave runs on (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ int xcc_id() {
  unsigned v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return (int)(v & 15u);
}

// Workgroup index of this block in a chain placed by a.xs / a.xid, or -1 for a
// block outside the chain.  Spread: blocks 0..W-1.  One XCC: the grid has W xs
// blocks and the dispatcher deals them to the xs XCCs in turn (from an XCC
// that changes from one dispatch to the next), so XCC xid receives the W
// blocks of one residue b mod xs, and w = b / xs numbers them.  The first wave
// to arrive claims its residue in bar[W kFlagStride - 1] (the last word of the flags, zero at
// launch); a block on XCC xid with another residue would mean the dispatch
// does not deal in turn: it sets the error flag to 2 and leaves, and the
// chain stops at its next barrier.
template <bool XL>
__device__ __forceinline__ int chain_workgroup(const ChainArgs& a) {
  const int b = blockIdx.x;
  if constexpr (!XL) return b;
  if (xcc_id() != a.xid) return -1;
  const unsigned r = (unsigned)(b % a.xs) + 1u;
  int ok = 1;
  if (__lane_id() == 0) {
    unsigned e = 0;
    ok = __hip_atomic_compare_exchange_strong(a.bar + kClaim(a.W), &e, r, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT) || e == r;
    if (!ok) __hip_atomic_store(a.err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (!__builtin_amdgcn_readfirstlane(ok)) return -1;
  return b / a.xs;
}

// Record a non-finite parameter write (integer atomic; the plain load skips
// the atomic once an earlier location is known, so a diverged chain does not
// pay one atomic per write).
__device__ __forceinline__ void report_nonfinite(const ChainArgs& a, unsigned long long key) {
  if (key < *reinterpret_cast<volatile unsigned long long*>(a.nf)) atomicMin(a.nf, key);
}

// ---------------------------------------------------------------------------
// The record a lane handles in one phase: minibatch order for the core
// sub-step, (row, position) order of mode ph-1 for the factor sub-steps.
// Every field is read from memory at a uniform offset, so no register array
// is ever indexed at run time.
// ---------------------------------------------------------------------------
template <int NM>
struct LaneRec {
  int idx[NM];         // the N indices (only read at compile-time positions)
  float x;             // the value
  int rown;            // index in the phase's mode n
  int meta;            // run metadata and split-row patch entry (see kMetaPatchShift)
  bool valid;
};

template <int NM>
__device__ __forceinline__ void load_lane_rec(const ChainArgs& a, int w, int N, int64_t b, int ph, LaneRec<NM>& r) {
  const PhaseTab& pt = a.pt[ph];
  const int64_t base = b * a.M;
  const int m = (int)((a.T - base < a.M) ? (a.T - base) : a.M);
  const int q = w * a.chunk + (int)threadIdx.x;
  r.valid = (int)threadIdx.x < a.chunk && q < m;
#pragma unroll
  for (int k = 0; k < NM; ++k) r.idx[k] = 0;
  r.x = 0.f;
  r.rown = 0;
  r.meta = 0;
  if (r.valid) {
    const uint32_t* src = (ph == 0) ? a.coo + (base + q) * a.s.R
                                    : a.rec_sorted + ((int64_t)(ph - 1) * a.T + base + q) * a.s.R;
#pragma unroll
    for (int k = 0; k < NM; ++k)
      if (k < N) r.idx[k] = (int)src[k];
    r.x = __uint_as_float(src[a.s.R - 1]);
    r.rown = (int)src[pt.n];
    r.meta = (int)a.meta[(int64_t)ph * a.T + base + q];
  }
}

// ---------------------------------------------------------------------------
// Row buffers.  Chunk-major: mode k's values [c*V, c*V + V) (one 16-byte chunk;
// V = 4 FP32 or 8 BF16 values of the read copy) of sample p sit at float word
// ((coff[k] + c) * chp + p) * 4, so the 64 lanes of a wave (samples 64 wv + l)
// fill 1 KB of consecutive LDS with one 16-byte transfer each.  The loads go
// from global memory straight into LDS: no registers are held while they are
// in flight, and a wave waits for vmcnt before the rows are read.
// ---------------------------------------------------------------------------
template <int JR, bool BF, bool EXACT, int NM>
__device__ __forceinline__ void issue_rows_lds(const ChainArgs& a, const int (&idx)[NM], unsigned mask, float* buf,
                                               int chp, bool valid) {
  constexpr int V = BF ? 8 : 4;
  constexpr int CM = (JR + V - 1) / V;
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    if ((mask >> k) & 1u) {
      const int J = EXACT ? JR : a.s.J[k];
      const char* src = BF ? reinterpret_cast<const char*>(a.Ab[k] + (int64_t)idx[k] * a.Jb[k])
                           : reinterpret_cast<const char*>(a.A[k] + (int64_t)idx[k] * a.s.Jp[k]);
      float* dst = buf + (a.lay.coff[k] * chp + wv * 64) * 4;
#pragma unroll
      for (int c = 0; c < CM; ++c)
        if ((EXACT || c * V < J) && valid) __builtin_amdgcn_global_load_lds(src + 16 * c, dst + c * chp * 4, 16, 0, 0);
    }
  }
}

// Value j of the mode whose chunks start at ck, for sample p.
template <bool BF>
__device__ __forceinline__ float row_at(const float* buf, int ck, int chp, int p, int j) {
  if constexpr (!BF) {
    return buf[((ck + (j >> 2)) * chp + p) * 4 + (j & 3)];
  } else {
    const unsigned short* b16 = reinterpret_cast<const unsigned short*>(buf);
    return bf16_val(b16[((ck + (j >> 3)) * chp + p) * 8 + (j & 7)]);
  }
}

// Sample p's whole row of a mode (values j >= J read as the zero padding of
// the factor rows, or stay 0).
template <int JR, bool BF, bool EXACT>
__device__ __forceinline__ void read_row(const float* buf, int ck, int chp, int p, int J, float (&v)[JR]) {
#pragma unroll
  for (int j = 0; j < JR; ++j) v[j] = 0.f;
  if constexpr (!BF) {
#pragma unroll
    for (int c = 0; c < (JR + 3) / 4; ++c) {
      if (EXACT || 4 * c < J) {
        const f32x4 t = *reinterpret_cast<const f32x4*>(buf + ((ck + c) * chp + p) * 4);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (4 * c + e < JR) v[4 * c + e] = t[e];
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < (JR + 7) / 8; ++c) {
      if (EXACT || 8 * c < J) {
        const u32x4 t = *reinterpret_cast<const u32x4*>(buf + ((ck + c) * chp + p) * 4);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (8 * c + e < JR)
            v[8 * c + e] = bf16_val((unsigned short)((e & 1) ? (t[e >> 1] >> 16) : (t[e >> 1] & 0xFFFFu)));
      }
    }
  }
}

// Overwrite sample p's row of a mode (values j < J) with v (rounded to BF16
// in BF16 mode).
template <int JR, bool BF, bool EXACT>
__device__ __forceinline__ void write_row(float* buf, int ck, int chp, int p, int J, const float (&v)[JR]) {
#pragma unroll
  for (int j = 0; j < JR; ++j) {
    if (EXACT || j < J) {
      if constexpr (!BF) {
        buf[((ck + (j >> 2)) * chp + p) * 4 + (j & 3)] = v[j];
      } else {
        unsigned short* b16 = reinterpret_cast<unsigned short*>(buf);
        b16[((ck + (j >> 3)) * chp + p) * 8 + (j & 7)] = bf16_bits(v[j]);
      }
    }
  }
}

// Segmented inclusive sum over the 64 lanes of a wave (fixed order): lane l
// adds the values of lanes [ws, l), ws = the first lane of its segment
// (ws <= l).  Within each row of 16 lanes by DPP row shifts (1, 2, 4, 8),
// then across rows by the row broadcasts of lanes 15 and 31.
template <int D>
__device__ __forceinline__ float dpp_row_shr(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + D, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_bcast15(float v) {  // rows 1 and 3 get lanes 15 and 47, rows 0 and 2 get 0
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));
}
__device__ __forceinline__ float dpp_bcast31(float v) {  // rows 2 and 3 get lane 31, rows 0 and 1 get 0
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false));
}

template <int JR, bool EXACT>
__device__ __forceinline__ void wave_segmented_scan(float (&u)[JR], int Jn, int lane, int ws) {
  const int rl = lane & 15;
  const bool t1 = rl >= 1 && lane - 1 >= ws, t2 = rl >= 2 && lane - 2 >= ws;
  const bool t4 = rl >= 4 && lane - 4 >= ws, t8 = rl >= 8 && lane - 8 >= ws;
  const int row = lane >> 4;
  const bool t15 = (row & 1) && (lane | 15) - 16 >= ws;  // lane 16*row - 1
  const bool t31 = row >= 2 && 31 >= ws;
#pragma unroll
  for (int j = 0; j < JR; ++j) {
    if (EXACT || j < Jn) {
      float v = u[j];
      float o = dpp_row_shr<1>(v);
      v += t1 ? o : 0.f;
      o = dpp_row_shr<2>(v);
      v += t2 ? o : 0.f;
      o = dpp_row_shr<4>(v);
      v += t4 ? o : 0.f;
      o = dpp_row_shr<8>(v);
      v += t8 ? o : 0.f;
      o = dpp_bcast15(v);
      v += t15 ? o : 0.f;
      o = dpp_bcast31(v);
      v += t31 ? o : 0.f;
      u[j] = v;
    }
  }
}

// The step of one straddling row from its summed run partials F (plus the
// after-slot's own partial first if add_b) and the old row (and velocity)
// that chunk cw, where the run began, left in the carry (layout at
// finish_split_rows).  vrow: where the new velocity goes (momentum, the
// storing workgroup), else null.
template <int JR, bool EXACT, bool MOM>
__device__ __forceinline__ void load_split_ops(const ChainArgs& a, const float* cbuf, int cw, int pJ, float (&Fb)[JR],
                                               float (&old)[JR], float (&vo)[JR]) {
  const int NS = 2 * a.W;
  const float* slotB = cbuf + cw * 2 + 1;
  const float* rowB = cbuf + (2 + pJ) * NS + cw;
#pragma unroll
  for (int j = 0; j < JR; ++j) {
    Fb[j] = (EXACT || j < pJ) ? slotB[(2 + j) * NS] : 0.f;
    old[j] = (EXACT || j < pJ) ? rowB[j * a.W] : 0.f;
    vo[j] = (MOM && (EXACT || j < pJ)) ? rowB[(pJ + j) * a.W] : 0.f;
  }
}

template <int JR, bool EXACT, bool MOM>
__device__ __forceinline__ void apply_split_step(const ChainArgs& a, int pJ, const float (&Fb)[JR], const float (&old)[JR],
                                                 const float (&vo)[JR], const float* F, bool add_b, float inv_c,
                                                 float* ent, float* vrow) {
#pragma unroll
  for (int j = 0; j < JR; ++j) {
    if (EXACT || j < pJ) {
      float st = (add_b ? Fb[j] + F[j] : F[j]) * inv_c + a.lA * old[j];
      if constexpr (MOM) {
        st = a.mu * vo[j] + st;
        if (vrow) vrow[j] = st;
      }
      ent[4 + j] = old[j] - a.gA * st;
    }
  }
}

template <int JR, bool EXACT, bool MOM>
__device__ __forceinline__ void split_row_step(const ChainArgs& a, const float* cbuf, int cw, int pJ, const float* F,
                                               bool add_b, float inv_c, float* ent, float* vrow) {
  // (every LDS read before the first write: the compiler cannot tell the
  // table from the slots and would otherwise order each read after it)
  float old[JR], Fb[JR], vo[JR];
  load_split_ops<JR, EXACT, MOM>(a, cbuf, cw, pJ, Fb, old, vo);
  apply_split_step<JR, EXACT, MOM>(a, pJ, Fb, old, vo, F, add_b, inv_c, ent, vrow);
}

// Finish the rows that straddled chunk boundaries in the previous factor
// sub-step (mode pm).  xr[bw] is the straddling row at boundary bw or -1,
// xn[bw] the entry number of a row's first boundary or -1 (both from the
// schedule); cbuf holds the LDS copy of the carry of chunks 0..W-1 for mode
// pm (pJ = J_pm): two slots per chunk, element-major, element e of slot sl
// at cbuf[e * 2W + sl] for e < 2 + pJ (slot 2w the run that began before
// chunk w, slot 2w+1 the run that goes on after it; elements [row, count,
// partial sum (pJ)]: adjacent boundaries read adjacent words), then for the
// after-slots only the old master row, value j of chunk w at
// cbuf[(2 + pJ) 2W + j W + w], and with momentum the old velocity, value j
// at cbuf[(2 + pJ) 2W + (pJ + j) W + w] (a run that straddles took its old
// row, and velocity, in the chunk where it began).  Fills the LDS table
// `split` (row, the run's first boundary, then the new master row at +4) in
// row order.  Workgroup st_w of st_n (st_n > 0) writes the rows of the
// entries e with e mod st_n = st_w (master, and BF16 copy in BF16 mode) and
// their velocities, so the stores are spread over the chain's workgroups.

template <int JR, bool EXACT, bool BF, bool GROUPED, bool MOM>
__device__ __forceinline__ void finish_split_rows(const ChainArgs& a, int pm, const int* xr, const int* xn, int nsplit,
                                  const float* cbuf, float* split, int sstride, int st_w, int st_n, int64_t kb) {
  const int tid = threadIdx.x, BT = blockDim.x;
  const int pJ = EXACT ? JR : a.s.J[pm];
  const int NS = 2 * a.W;
  if (a.W <= 64) {
    // all boundaries in one wave: lane v loads the before-slot of chunk v,
    // a segmented scan over the runs of equal rows adds them in a fixed
    // tree order, and the run's last lane adds the after-slot of the chunk
    // where the run began and writes the entry
    if (tid < 64) {
      const int v = tid;
      // every LDS read first, with clamped indices, so they are in flight
      // together: the rows at the boundaries, this lane's before-slot, and
      // the after-slot and entry number of the chunk where its run began
      // (the run's start comes from the ballot, before the scans)
      const int x0 = xr[min(v, a.W - 1)], xm = xr[min(max(v - 1, 0), a.W - 1)], xp = xr[min(v + 1, a.W - 1)];
      const float* slotA = cbuf + min(v, a.W - 1) * 2;
      const int ca = __float_as_int(slotA[NS]);
      float u[JR], cc[1];
#pragma unroll
      for (int j = 0; j < JR; ++j) u[j] = (EXACT || j < pJ) ? slotA[(2 + j) * NS] : 0.f;
      const int rowv = (v >= 1 && v < a.W) ? x0 : -1;
      const int rowp = (v >= 2 && v - 1 < a.W) ? xm : -1;
      const int rown = (v + 1 < a.W) ? xp : -1;
      const bool live = rowv >= 0;
      const bool first = live && rowp != rowv;
      const bool last = live && rown != rowv;
      const unsigned long long starts = __ballot(first);
      const unsigned long long upto = v == 63 ? ~0ull : ((2ull << v) - 1);
      const int ws = live ? 63 - __clzll(starts & upto) : v;  // first boundary of my run
      const int wsc = min(max(ws, 1), a.W - 1);
      const int e = xn[wsc];
      const int cb = __float_as_int(cbuf[(wsc - 1) * 2 + 1 + NS]);
      float Fb[JR], old[JR], vo[JR];
      load_split_ops<JR, EXACT, MOM>(a, cbuf, wsc - 1, pJ, Fb, old, vo);
      cc[0] = live ? (float)ca : 0.f;
#pragma unroll
      for (int j = 0; j < JR; ++j) u[j] = live ? u[j] : 0.f;
      wave_segmented_scan<JR, EXACT>(u, pJ, v, ws);
      wave_segmented_scan<1, true>(cc, 1, v, ws);
      if (last) {
        const int c = (int)cc[0] + cb;
        float* ent = split + e * sstride;
        float* vrow = (MOM && st_n > 0 && e % st_n == st_w) ? a.VA[pm] + (int64_t)rowv * a.s.Jp[pm] : nullptr;
        apply_split_step<JR, EXACT, MOM>(a, pJ, Fb, old, vo, u, true, 1.0f / (float)c, ent, vrow);
        ent[0] = __int_as_float(rowv);
      }
    }
  } else if (!GROUPED) {
    // one thread per boundary where a run starts, summing the run's slots in
    // chunk order
    for (int bw = tid + 1; bw < a.W; bw += BT) {
      const int e = xn[bw];
      if (e < 0) continue;
      const int row = xr[bw];
      const float* slotB = cbuf + (bw - 1) * 2 + 1;
      float F[JR];
      int c = __float_as_int(slotB[NS]);
#pragma unroll
      for (int j = 0; j < JR; ++j) F[j] = (EXACT || j < pJ) ? slotB[(2 + j) * NS] : 0.f;
      for (int v = bw; v < a.W && xr[v] == row; ++v) {
        const float* slotA = cbuf + v * 2;
        c += __float_as_int(slotA[NS]);
#pragma unroll
        for (int j = 0; j < JR; ++j)
          if (EXACT || j < pJ) F[j] += slotA[(2 + j) * NS];
      }
      float* ent = split + e * sstride;
      float* vrow = (MOM && st_n > 0 && e % st_n == st_w) ? a.VA[pm] + (int64_t)row * a.s.Jp[pm] : nullptr;
      split_row_step<JR, EXACT, MOM>(a, cbuf, bw - 1, pJ, F, false, 1.0f / (float)c, ent, vrow);
      ent[0] = __int_as_float(row);
    }
  } else {
    // entry -> its first boundary (kept in the entry's header word 1)
    for (int bw = tid + 1; bw < a.W; bw += BT) {
      const int e = xn[bw];
      if (e >= 0) split[e * sstride + 1] = __int_as_float(bw);
    }
    __syncthreads();
    // A group of GL lanes per entry (GL = 4, or fewer when there are more
    // entries than the workgroup has quads): lane i sums the before-slots of
    // boundaries bw + i, bw + i + GL, ... of the run (a long run of a popular
    // row crosses many chunks), then the group adds up by a fixed butterfly
    // (quad DPP) and its first lane adds the after-slot of the chunk where the
    // run began.
    const int GL = nsplit * 4 <= BT ? 4 : (nsplit * 2 <= BT ? 2 : 1);
    const int g = tid / GL, i = tid % GL, ng = BT / GL;
    for (int e0 = 0; e0 < nsplit; e0 += ng) {
      const int e = e0 + g;
      const bool ok = e < nsplit;
      const int bw = ok ? __float_as_int(split[e * sstride + 1]) : 1;
      const int row = ok ? xr[bw] : -2;
      float F[JR];
      int c = 0;
#pragma unroll
      for (int j = 0; j < JR; ++j) F[j] = 0.f;
      for (int v = bw + i; ok && v < a.W && xr[v] == row; v += GL) {
        const float* slotA = cbuf + v * 2;
        c += __float_as_int(slotA[NS]);
#pragma unroll
        for (int j = 0; j < JR; ++j)
          if (EXACT || j < pJ) F[j] += slotA[(2 + j) * NS];
      }
      if (GL >= 2) {  // lanes 2q, 2q+1 (and then the pairs of a quad): xor 1, then xor 2
        c += __builtin_amdgcn_mov_dpp(c, 0xB1, 0xF, 0xF, false);
#pragma unroll
        for (int j = 0; j < JR; ++j)
          if (EXACT || j < pJ) F[j] += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(F[j]), 0xB1, 0xF, 0xF, false));
        if (GL == 4) {
          c += __builtin_amdgcn_mov_dpp(c, 0x4E, 0xF, 0xF, false);
#pragma unroll
          for (int j = 0; j < JR; ++j)
            if (EXACT || j < pJ) F[j] += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(F[j]), 0x4E, 0xF, 0xF, false));
        }
      }
      if (ok && i == 0) {
        const float* slotB = cbuf + (bw - 1) * 2 + 1;
        const int cb = __float_as_int(slotB[NS]);
        float* ent = split + e * sstride;
        float* vrow = (MOM && st_n > 0 && e % st_n == st_w) ? a.VA[pm] + (int64_t)row * a.s.Jp[pm] : nullptr;
        split_row_step<JR, EXACT, MOM>(a, cbuf, bw - 1, pJ, F, true, 1.0f / (float)(c + cb), ent, vrow);
        ent[0] = __int_as_float(row);
      }
    }
  }
  __syncthreads();
  if (st_n > 0) {
    for (int e = tid; e < nsplit * pJ; e += BT) {
      const int en = e / pJ, j = e - en * pJ;
      if (en % st_n != st_w) continue;
      const int row = __float_as_int(split[en * sstride]);
      const float v = split[en * sstride + 4 + j];
      a.A[pm][(int64_t)row * a.s.Jp[pm] + j] = v;
      if (BF) a.Ab[pm][(int64_t)row * a.Jb[pm] + j] = bf16_bits(v);
      if (!__builtin_isfinite(v)) report_nonfinite(a, nf_key(kb, pm + 1, row));
    }
  }
}

// Tables of the contraction (MFMA B operands), built from the core Gs:
//   FP32, two-stage (TS): TB[(ct * ks2 + ks) * 64 + l] = G_(n)[j_n, k + J_lo h] with
//         k = 2 ks + l / 32, l % 32 = j_n + J_n hh, h = ct * hpt + hh
//   BF16, two-stage:      TB16[((ct * ks2 + ks) * 64 + l) * 4 + i] = bf16(same) with
//         k = 8 ks + 4 (l / 32) + i
//   FP32, direct:         TB[((h * nt + t) * kp + k) * 16 + c] = G_(n)[16t + c, k + J_lo h]
//   BF16, direct:         TB16[((h * nt + t) * 16 + c) * kp + k] = bf16(G_(n)[16t + c, k + J_lo h])
// (zero outside j_n < J_n, k < J_lo, hh < hpt, h < khi).  With a host-built gather map (tmap[e]
// = offset in the core or -1) the build is one load and one store per element.
template <bool BF>
__device__ __forceinline__ void build_table_map(const float* Gs, const int* tmap, int len, float* TB) {
  unsigned short* TB16 = reinterpret_cast<unsigned short*>(TB);
  const int BT = blockDim.x;
  for (int e0 = threadIdx.x; e0 < len; e0 += 4 * BT) {
    int o[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) o[u] = tmap[min(e0 + u * BT, len - 1)];
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float g = Gs[max(o[u], 0)];
      v[u] = o[u] >= 0 ? g : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * BT;
      if (e < len) {
        if (BF) TB16[e] = bf16_bits(v[u]);
        else TB[e] = v[u];
      }
    }
  }
}

// The same table without a map (when the maps do not fit in LDS): index
// arithmetic per element; hmap[h] is the core offset of multi-index h.  With
// compile-time equal ranks every mode's table has its zero entries (k >= J_lo,
// j_n >= J_n) in the same places, so they are written once at set-up
// (zero_only) and each rebuild writes only the J_lo J_n khi core values.
template <int JR, bool BF, bool EXACT, bool TS>
__device__ __forceinline__ void build_table_arith(const PhaseTab& pt, const float* Gs, const int* hmap, float* TB,
                                                  bool zero_only = false) {
  unsigned short* TB16 = reinterpret_cast<unsigned short*>(TB);
  const int BT = blockDim.x;
  if constexpr (EXACT) {
    constexpr int KP = BF ? ((JR + 15) & ~15) : ((JR + 3) & ~3);
    constexpr int NT = (JR + 15) / 16;
    if (zero_only) {
      const int total = pt.tb_len;
      for (int e = threadIdx.x; e < total; e += BT) {
        if (BF) TB16[e] = 0;
        else TB[e] = 0.f;
      }
      return;
    }
    constexpr int PER_H = JR * JR;  // (k, j_n) pairs of one h
    const int total = pt.khi * PER_H;
    for (int q0 = threadIdx.x; q0 < total; q0 += 4 * BT) {
      float v[4];
      int e[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = min(q0 + u * BT, total - 1);
        const int jn = q % JR, k = (q / JR) % JR, h = q / PER_H;
        v[u] = Gs[hmap[h] + k * pt.ls_lo + jn * pt.ls_n];
        if (BF && !TS) {
          e[u] = ((h * NT + (jn >> 4)) * 16 + (jn & 15)) * KP + k;
        } else if (BF) {
          constexpr int HPT = 32 / JR, KS8 = (JR + 7) / 8;
          const int ct = h / HPT, hh = h - ct * HPT;
          e[u] = ((ct * KS8 + (k >> 3)) * 64 + (((k >> 2) & 1) << 5) + hh * JR + jn) * 4 + (k & 3);
        } else if (!TS) {
          e[u] = ((h * NT + (jn >> 4)) * KP + k) * 16 + (jn & 15);
        } else {
          constexpr int HPT = 32 / JR, KS2 = (JR + 1) / 2;
          const int ct = h / HPT, hh = h - ct * HPT;
          e[u] = (ct * KS2 + (k >> 1)) * 64 + ((k & 1) << 5) + hh * JR + jn;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (q0 + u * BT < total) {
          if (BF) TB16[e[u]] = bf16_bits(v[u]);
          else TB[e[u]] = v[u];
        }
      }
    }
  } else {
    if (zero_only) return;
    const int total = pt.tb_len;
    for (int e0 = threadIdx.x; e0 < total; e0 += 4 * BT) {
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * BT;
        v[u] = 0.f;
        if (e < total) {
          if (!TS) {
            int k, c, ht;
            if (BF) {  // e = (ht * 16 + c) * kp + k
              k = e % pt.kp;
              const int r = e / pt.kp;
              c = r & 15;
              ht = r >> 4;
            } else {   // e = (ht * kp + k) * 16 + c
              c = e & 15;
              const int r = e >> 4;
              k = r % pt.kp;
              ht = r / pt.kp;
            }
            const int h = pt.nt == 1 ? ht : ht / pt.nt;
            const int t = ht - h * pt.nt;
            const int jn = 16 * t + c;
            if (k < pt.jlo && jn < pt.Jn) v[u] = Gs[hmap[h] + k * pt.ls_lo + jn * pt.ls_n];
          } else {   // e = ((ct * ks2 + ks) * 64 + l) * lw + ee, column l % 32 = j_n + J_n hh
            const int lw = BF ? 4 : 1;
            const int ct = e / (pt.ks2 * 64 * lw), r = e - ct * pt.ks2 * 64 * lw;
            const int l = (r / lw) & 63, ks = r / (64 * lw), ee = r % lw;
            const int k = BF ? 8 * ks + 4 * (l >> 5) + ee : 2 * ks + (l >> 5), c = l & 31;
            const int hh = c / pt.Jn, jn = c - hh * pt.Jn;
            const int h = ct * pt.hpt + hh;
            if (k < pt.jlo && hh < pt.hpt && h < pt.khi) v[u] = Gs[hmap[h] + k * pt.ls_lo + jn * pt.ls_n];
          }
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
}

// hp[h * hs + p] = prod over the remaining modes of the sample's rows at h
// (1 when there are none); zero for positions p >= cnt.  hmap[khi + h * nhi + i]
// is the position of remaining mode i's value at h in the row buffer less
// the sample term (p * 4 floats, or p * 8 BF16 values).  Reads are batched
// ahead of the writes, four h at a time.
template <bool BF>
__device__ __forceinline__ void build_hp(const PhaseTab& pt, const float* rowbuf, const int* hmap, int cnt, int chp,
                                         float* hp, int hs) {
  const int p = threadIdx.x;
  if (p >= chp) return;
  const int khi = pt.khi, nhi = pt.nhi;
  if (p >= cnt) {
    for (int h = 0; h < khi; ++h) hp[h * hs + p] = 0.f;
    return;
  }
  if (nhi == 0) {
    hp[p] = 1.f;
    return;
  }
  const int* ro = hmap + khi;
  const unsigned short* b16 = reinterpret_cast<const unsigned short*>(rowbuf);
  for (int h0 = 0; h0 < khi; h0 += 4) {
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int h = h0 + u;
      v[u] = 1.f;
      if (h < khi)
        for (int i = 0; i < nhi; ++i) {
          const int o = ro[h * nhi + i];
          v[u] *= BF ? bf16_val(b16[o + p * 8]) : rowbuf[o + p * 4];
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (h0 + u < khi) hp[(h0 + u) * hs + p] = v[u];
  }
}

// hp for two remaining modes and compile-time equal ranks: both rows of the
// sample in registers, hp[(d1 + J d2) * hs + p] = row1[d1] row2[d2] (the
// first remaining mode fastest, as in the maps).  The workgroup's threads
// form BT / chp groups that split the d2 range.
template <int JR, bool BF>
__device__ __forceinline__ void build_hp2(const PhaseTab& pt, const float* rowbuf, int cnt, int chp, float* hp,
                                          int hs) {
  const int G = blockDim.x / chp;
  const int p = threadIdx.x % chp, g = threadIdx.x / chp;
  if (g >= G) return;
  float r1[JR], r2[JR];
  read_row<JR, BF, true>(rowbuf, pt.c_hi, chp, p, JR, r1);
  read_row<JR, BF, true>(rowbuf, pt.c_hi2, chp, p, JR, r2);
  if (p >= cnt) {
#pragma unroll
    for (int j = 0; j < JR; ++j) r1[j] = 0.f;
  }
  for (int d2 = g; d2 < JR; d2 += G) {
    float v2 = r2[0];
#pragma unroll
    for (int j = 1; j < JR; ++j)
      if (j == d2) v2 = r2[j];
#pragma unroll
    for (int d1 = 0; d1 < JR; ++d1) hp[(d1 + JR * d2) * hs + p] = r1[d1] * v2;
  }
}

// Lane l gets lane (l + M) mod 16 of its row of 16 (DPP row rotate).
template <int M>
__device__ __forceinline__ float dpp_ror(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + M, 0xF, 0xF, false));
}
// Lane l gets lane l xor 16 (swizzle within groups of 32 lanes).
__device__ __forceinline__ float swizzle_xor16(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
}

// Where the products hp_p[h] are read from: the hp buffer (hp[h * hs + p]),
// or, with a single remaining mode (three-mode tensors), that mode's rows in
// the row buffer directly.
template <bool HPV, bool BF>
struct HpRef {
  const float* base;  // hp buffer, or the row buffer
  int st;             // hp buffer: its row stride; row buffer: chp
  int ck;             // (row buffer) chunk offset of the remaining mode
  __device__ __forceinline__ float one(int p, int h) const {
    if constexpr (!HPV) return base[h * st + p];
    else return row_at<BF>(base, ck, st, p, h);
  }
  __device__ __forceinline__ f32x4 quad(int p, int h) const {  // samples p .. p+3
    if constexpr (!HPV) {
      return *reinterpret_cast<const f32x4*>(base + h * st + p);
    } else {
      f32x4 v;
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = row_at<BF>(base, ck, st, p + i, h);
      return v;
    }
  }
};

// E_p for the chunk's samples (MFMA, see the file header).
//
// FP32, three-mode kernels (HPV): one MFMA chain per 16-sample tile over
// K = (j_lo, h), the A operand a(lo)_p[j_lo] hp_p[h] formed per lane, the B
// operand the table of mode n (16 columns, j_n); E_p to ebuf[p * es + j_n].
//
// Other kernels: two stages on 32x32 tiles (FP32 32x32x2, BF16 32x32x8).  Stage 1, per 32-sample block and
// 32-column tile, C[p][(j_n, h)] = sum_{j_lo} a(lo)_p[j_lo] G_(n)[j_n, j_lo + J_lo h]
// (K = J_lo in steps of 2 or 8, every column used: a tile holds hpt whole h);
// stage 2, on the accumulators, S[p][j_n] += hp_p[h] C[p][(j_n, h)].  The
// waves of a block share its column tiles; lane partial sums go to slot
// (wave part, h mod hpt) of ebuf[p * es + slot * J_n + j_n] and the reader adds
// the g.ens slots in order.
//
// BF16, three-mode kernels: a job is TPJ 16-sample tiles (one, or two sharing the B loads) times
// one 16-wide j_n tile, C[p][j_n] per h on 16x16x16 BF16 MFMAs and the sum
// over h on the accumulators; E_p goes to ebuf[p * es + j_n] (one slot).  The
// caller picks TPJ = 1 when there are at least as many waves as single-tile
// jobs (the FP32 three-mode path takes TPJ the same way).
template <int JR, bool BF, bool EXACT, bool HPV, int KHI, int TPJ>
__device__ __forceinline__ void mfma_E(const Shape& s, const PhaseTab& g, const float* TB, const float* rowbuf,
                                       const HpRef<HPV, BF>& hpr, int cnt, int chp, float* ebuf, int es) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int Jn = EXACT ? JR : g.Jn;
  const int clo = g.c_lo;
  const int khi = g.khi;
  if constexpr (!HPV) {
    constexpr int KSM = BF ? (JR + 7) / 8 : (JR + 1) / 2;  // K steps (upper bound when not EXACT)
    const int ks2 = EXACT ? KSM : g.ks2;
    const int hpt = EXACT ? 32 / JR : g.hpt;
    const int ctn = g.ctn;
    const int nblk = chp >> 5;                 // chp is a multiple of 32
    const int nwb = max(1, nwaves / nblk);     // waves per block
    const int c32 = lane & 31, khalf = lane >> 5;
    const int hh = c32 / Jn, jj = c32 - hh * Jn;
    const bool colok = hh < hpt;
    for (int bj = wv; bj < nblk * nwb; bj += nwaves) {
      const int blk = bj / nwb, wp = bj - blk * nwb;
      if (blk * 32 >= cnt) continue;  // no live sample in the block (uniform)
      // A operand: row 32 blk + c32 of the block, k = 2 ks + khalf of the lo-mode
      // row (zero padding past J_lo; rows p >= cnt hold finite values that
      // reach only samples that are not read)
      float av[KSM];
      s16x4 avb[KSM];
      const int pa = blk * 32 + c32;
#pragma unroll
      for (int ks = 0; ks < KSM; ++ks) {
        if constexpr (!BF) {
          const int k = 2 * ks + khalf;
          av[ks] = (EXACT || ks < ks2) ? rowbuf[((clo + (k >> 2)) * chp + pa) * 4 + (k & 3)] : 0.f;
        } else {  // k = 8 ks + 4 khalf + i: chunk ks, BF16 words 4 khalf + i
          const unsigned short* b16 = reinterpret_cast<const unsigned short*>(rowbuf);
          avb[ks] = (EXACT || ks < ks2) ? *reinterpret_cast<const s16x4*>(b16 + ((clo + ks) * chp + pa) * 8 + 4 * khalf)
                                        : s16x4{0, 0, 0, 0};
        }
      }
      const int prow = blk * 32 + 4 * khalf;  // this lane's accumulator rows: prow + 8 q + i
      float S[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) S[i] = 0.f;
      constexpr int TT = 4;  // column tiles in flight (independent MFMA chains)
      for (int ct0 = wp; ct0 < ctn; ct0 += TT * nwb) {
        f32x16 acc[TT];
#pragma unroll
        for (int t = 0; t < TT; ++t)
#pragma unroll
          for (int i = 0; i < 16; ++i) acc[t][i] = 0.f;
#pragma unroll
        for (int ks = 0; ks < KSM; ++ks) {
          if (EXACT || ks < ks2) {
            if constexpr (!BF) {
              float bv[TT];
#pragma unroll
              for (int t = 0; t < TT; ++t) bv[t] = TB[(min(ct0 + t * nwb, ctn - 1) * ks2 + ks) * 64 + lane];
#pragma unroll
              for (int t = 0; t < TT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[ks], bv[t], acc[t], 0, 0, 0);
            } else {
              const unsigned short* tb16 = reinterpret_cast<const unsigned short*>(TB);
              s16x4 bv[TT];
#pragma unroll
              for (int t = 0; t < TT; ++t)
                bv[t] = *reinterpret_cast<const s16x4*>(tb16 + ((min(ct0 + t * nwb, ctn - 1) * ks2 + ks) * 64 + lane) * 4);
              // (all four loads in flight before the first MFMA: without this use
              // the register allocator, at its bound, gives them one register pair
              // and serialises them)
              asm volatile("" ::"v"(bv[0]), "v"(bv[1]), "v"(bv[2]), "v"(bv[3]));
#pragma unroll
              for (int t = 0; t < TT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(avb[ks], bv[t], acc[t], 0, 0, 0);
            }
          }
        }
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          const int ct = ct0 + t * nwb;
          const int h = ct * hpt + hh;
          if (colok && ct < ctn && h < khi) {
            f32x4 hq[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) hq[q] = hpr.quad(prow + 8 * q, h);
            asm volatile("" ::"v"(hq[0]), "v"(hq[1]), "v"(hq[2]), "v"(hq[3]));  // (the four reads in one batch)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
              for (int i = 0; i < 4; ++i) S[4 * q + i] = fmaf(hq[q][i], acc[t][4 * q + i], S[4 * q + i]);
          }
        }
      }
      // hpt a power of two with hpt J_n = 32: add the hpt lanes of each j_n
      // (a fixed rotate-and-add order), one slot per wave part
      const bool fold = hpt > 1 && (hpt & (hpt - 1)) == 0 && hpt * Jn == 32;
      if (fold) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          float v = S[i];
          if (Jn <= 1) v += dpp_ror<1>(v);
          if (Jn <= 2) v += dpp_ror<2>(v);
          if (Jn <= 4) v += dpp_ror<4>(v);
          if (Jn <= 8) v += dpp_ror<8>(v);
          v += swizzle_xor16(v);
          S[i] = v;
        }
      }
      if (fold ? hh == 0 : colok) {
        const int slot = (fold ? wp : wp * hpt + hh) * Jn + jj;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i = 0; i < 4; ++i) ebuf[(prow + 8 * q + i) * es + slot] = S[4 * q + i];
      }
    }
  } else {
    constexpr bool TWO = TPJ == 2;
    const int r16 = lane & 15, kq = lane >> 4;
    constexpr int KPX = BF ? ((JR + 15) & ~15) : ((JR + 3) & ~3);
    const int MT = (cnt + 15) >> 4;
    const int kp = EXACT ? KPX : g.kp;
    const int nt = EXACT ? (JR + 15) / 16 : g.nt;
    const int jobs = ((MT + TPJ - 1) / TPJ) * nt;  // job = (tile group, j_n tile)
    for (int job = wv; job < jobs; job += nwaves) {
      const int mp = job / nt, t = job - mp * nt;
      const int mt0 = TPJ * mp, mt1 = mt0 + 1;
      const int prow0 = mt0 * 16 + r16, prow1 = mt1 * 16 + r16;
      const int prow0c = min(prow0, chp - 1), prow1c = min(prow1, chp - 1);
      f32x4 e0 = {0.f, 0.f, 0.f, 0.f}, e1 = {0.f, 0.f, 0.f, 0.f};
      if constexpr (!BF) {
        constexpr int KS = (JR + 3) / 4;
        float a0[KS], a1[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          // no masks: the table rows k >= J_lo are zero, samples p >= cnt are
          // not stored, and the row buffer holds finite values only.
          // value k = 4 ks + kq of the lo-mode row: chunk ks, word kq
          a0[ks] = rowbuf[((clo + ks) * chp + prow0c) * 4 + kq];
          a1[ks] = TWO ? rowbuf[((clo + ks) * chp + prow1c) * 4 + kq] : 0.f;
        }
        // One accumulation chain per tile and K chunk ks (and parity of h when
        // that gives fewer than four chains) over K = (j_lo, h): the A operand
        // is a(lo)_p[j_lo] * hp_p[h] (p = the lane's tile row), so the second
        // stage folds into the MFMA chain, and consecutive MFMAs of a step go
        // to different chains.
        const int nks = kp >> 2;
        const float* tb = TB + (t * kp + kq) * 16 + r16;
        const int hstride = nt * kp * 16;
        constexpr int PAR = TPJ * KS >= 4 ? 1 : 2;
        f32x4 acc0[KS][PAR], acc1[KS][PAR];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
          for (int q = 0; q < PAR; ++q) acc0[ks][q] = acc1[ks][q] = f32x4{0.f, 0.f, 0.f, 0.f};
        auto mfmas = [&](int q, float hv0, float hv1, const float (&bv)[KS]) {
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) {
            if (ks < nks) {
              acc0[ks][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[ks] * hv0, bv[ks], acc0[ks][q], 0, 0, 0);
              if constexpr (TWO) acc1[ks][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[ks] * hv1, bv[ks], acc1[ks][q], 0, 0, 0);
            }
          }
        };
        if constexpr (KHI > 0) {  // trip count known: straight-line code, loads scheduled early
#pragma unroll
          for (int h = 0; h < KHI; ++h) {
            float bv[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) bv[ks] = ks < nks ? tb[h * hstride + ks * 64] : 0.f;
            mfmas(h % PAR, hpr.one(prow0c, h), TWO ? hpr.one(prow1c, h) : 0.f, bv);
          }
        } else {
          // runtime trip count: h in groups of four, the operands of the next
          // group read before the MFMAs of the current one (clamped reads stay
          // in the buffers; an h past the end gets a zero A operand)
          constexpr int HG = 4;
          struct Ops {
            float hv0[HG], hv1[HG], bv[HG][KS];
          };
          auto load = [&](int h0, Ops& o) {
#pragma unroll
            for (int u = 0; u < HG; ++u) {
              const int hc = min(h0 + u, khi - 1);
              const bool live = h0 + u < khi;
              const float x0 = hpr.one(prow0c, hc);
              const float x1 = TWO ? hpr.one(prow1c, hc) : 0.f;
              o.hv0[u] = live ? x0 : 0.f;
              o.hv1[u] = live ? x1 : 0.f;
#pragma unroll
              for (int ks = 0; ks < KS; ++ks) o.bv[u][ks] = ks < nks ? tb[hc * hstride + ks * 64] : 0.f;
            }
          };
          Ops cur, nxt;
          load(0, cur);
          for (int h0 = 0; h0 < khi; h0 += HG) {
            load(h0 + HG, nxt);
#pragma unroll
            for (int u = 0; u < HG; ++u) mfmas(u % PAR, cur.hv0[u], cur.hv1[u], cur.bv[u]);
            cur = nxt;
          }
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
          for (int q = 0; q < PAR; ++q) {
            e0 += acc0[ks][q];
            if constexpr (TWO) e1 += acc1[ks][q];
          }
      } else {
          constexpr int KS = (JR + 15) / 16;
          s16x4 a0[KS], a1[KS];
          const unsigned short* b16 = reinterpret_cast<const unsigned short*>(rowbuf);
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) {
            // values k = 16 ks + 4 kq + e (e < 4): chunk 2 ks + kq / 2, BF16 words 4 (kq & 1) + e
            const int ch = clo + 2 * ks + (kq >> 1);
            a0[ks] = *reinterpret_cast<const s16x4*>(b16 + (ch * chp + prow0c) * 8 + 4 * (kq & 1));
            if constexpr (TWO) a1[ks] = *reinterpret_cast<const s16x4*>(b16 + (ch * chp + prow1c) * 8 + 4 * (kq & 1));
          }
          const int nks = kp >> 4;
          const unsigned short* tb = reinterpret_cast<const unsigned short*>(TB) + (t * 16 + r16) * kp + 4 * kq;
          const int hstride = nt * 16 * kp;
          const int hq0 = mt0 * 16 + 4 * kq;
          const int hq1 = min(mt1, MT - 1) * 16 + 4 * kq;  // (a missing tile mt1 is never stored)
          for (int h = 0; h < khi; ++h) {
            f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
              if (ks < nks) {
                const s16x4 bv = *reinterpret_cast<const s16x4*>(tb + h * hstride + 16 * ks);
                c0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0[ks], bv, c0, 0, 0, 0);
                if constexpr (TWO) c1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[ks], bv, c1, 0, 0, 0);
              }
            }
            const f32x4 h0 = hpr.quad(hq0, h);
#pragma unroll
            for (int i = 0; i < 4; ++i) e0[i] = fmaf(c0[i], h0[i], e0[i]);
            if constexpr (TWO) {
              const f32x4 h1 = hpr.quad(hq1, h);
#pragma unroll
              for (int i = 0; i < 4; ++i) e1[i] = fmaf(c1[i], h1[i], e1[i]);
            }
          }
      }
      const int jn = 16 * t + r16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p0 = mt0 * 16 + 4 * kq + i, p1 = mt1 * 16 + 4 * kq + i;
        if (p0 < cnt && jn < Jn) ebuf[p0 * es + jn] = e0[i];
        if (TWO && p1 < cnt && jn < Jn) ebuf[p1 * es + jn] = e1[i];
      }
    }
  }
}

// E_p[j] of one sample: the sum of its ens partial slots in slot order.
template <int JR, bool EXACT>
__device__ __forceinline__ void read_e(const float* eb, int ens, int Jn, float (&ev)[JR]) {
#pragma unroll
  for (int j = 0; j < JR; ++j) ev[j] = (EXACT || j < Jn) ? eb[j] : 0.f;
  for (int sl = 1; sl < ens; ++sl) {
#pragma unroll
    for (int j = 0; j < JR; ++j)
      if (EXACT || j < Jn) ev[j] += eb[sl * Jn + j];
  }
}

// partial[lin] = sum over the chunk of r_p h_p[lin], lin = j0 + J0 * col with
// col = j_lo + J_lo h: the GEMM dG[j0, col] = sum_p ra[p][j0] * B[p][col],
// B[p][col] = a(lo)_p[j_lo] hp_p[h] (ra[p * ras + j0] = r_p a(0)_p[j0], zero
// for p >= cnt), K = the chunk's samples.  The columns are packed, so J_lo khi
// of them fill ceil(J_lo khi / 16) tiles; a wave runs two output tiles at a
// time (two independent MFMA chains sharing the A loads when they share rows).
template <int JR, bool BF, bool EXACT, bool HPV>
__device__ __forceinline__ void mfma_core_grad(const Shape& s, const PhaseTab& g, const float* rowbuf, const float* ra,
                                               int ras, const HpRef<HPV, BF>& hpr, int cnt, int chp, float* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int J0 = EXACT ? JR : g.Jn;  // the core phase contracts with mode 0
  const int jlo = EXACT ? JR : g.jlo;
  const int khi = g.khi;
  const int ncol = jlo * khi;
  const int MT0 = EXACT && JR <= 16 ? 1 : (J0 + 15) >> 4;
  const int NTC = (ncol + 15) >> 4;
  const int clo = g.c_lo;
  const int jobs = MT0 * NTC;
  constexpr int KSTEP = BF ? 16 : 4;
  const int nsteps = (cnt + KSTEP - 1) / KSTEP;  // KSTEP * nsteps <= chp
  for (int jb = wv; jb < jobs; jb += 2 * nwaves) {
    const int jb2 = min(jb + nwaves, jobs - 1);  // second tile (a repeat of the first when absent: not stored)
    const bool has2 = jb + nwaves < jobs;
    const int t0a = MT0 == 1 ? 0 : jb / NTC, tca = jb - t0a * NTC;
    const int t0b = MT0 == 1 ? 0 : jb2 / NTC, tcb = jb2 - t0b * NTC;
    const int j0a = 16 * t0a + r16, j0b = 16 * t0b + r16;  // A rows of this lane
    const int cola = 16 * tca + r16, colb = 16 * tcb + r16;  // B columns of this lane
    const int ca = min(cola, ncol - 1), cb = min(colb, ncol - 1);
    const int ha = ca / jlo, jla = ca - ha * jlo, hb = cb / jlo, jlb = cb - hb * jlo;
    f32x4 acca = {0.f, 0.f, 0.f, 0.f}, accb = {0.f, 0.f, 0.f, 0.f};
    if constexpr (!BF) {
      // K in groups of four steps (16 samples), the operands of group gi+1
      // read before the MFMAs of group gi.  No masks: positions p >= cnt have
      // zero r a(0), the row buffer holds finite values only, and rows j0 >= J0
      // and columns col >= J_lo khi reach only outputs that are not stored.
      const int ngroups = (nsteps + 3) >> 2;
      auto load = [&](int gi, float (&aa)[4], float (&ab)[4], float (&ba)[4], float (&bb)[4]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int p = (4 * gi + u) * 4 + kq;
          aa[u] = ra[p * ras + j0a];
          ab[u] = ra[p * ras + j0b];
          ba[u] = rowbuf[((clo + (jla >> 2)) * chp + p) * 4 + (jla & 3)] * hpr.one(p, ha);
          bb[u] = rowbuf[((clo + (jlb >> 2)) * chp + p) * 4 + (jlb & 3)] * hpr.one(p, hb);
        }
      };
      float aa[4], ab[4], ba[4], bb[4];
      if (ngroups > 0) load(0, aa, ab, ba, bb);
      for (int gi = 0; gi < ngroups; ++gi) {
        float na[4], nb[4], nc[4], nd[4];
        load(gi + 1 < ngroups ? gi + 1 : gi, na, nb, nc, nd);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          acca = __builtin_amdgcn_mfma_f32_16x16x4f32(aa[u], ba[u], acca, 0, 0, 0);
          accb = __builtin_amdgcn_mfma_f32_16x16x4f32(ab[u], bb[u], accb, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          aa[u] = na[u];
          ab[u] = nb[u];
          ba[u] = nc[u];
          bb[u] = nd[u];
        }
      }
    } else {
      // no masks (see the FP32 path); 16 * nsteps <= chp.  The operands of
      // step st + 1 are read before the MFMAs of step st; with one row tile
      // both output tiles share the A operand.
      const bool oneA = MT0 == 1;
      struct Ops {
        s16x4 aa, ab, ba, bb;
      };
      auto load = [&](int st, Ops& o) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int p = st * 16 + 4 * kq + e;
          o.aa[e] = (short)bf16_bits(ra[p * ras + j0a]);
          o.ab[e] = oneA ? o.aa[e] : (short)bf16_bits(ra[p * ras + j0b]);
          o.ba[e] = (short)bf16_bits(row_at<BF>(rowbuf, clo, chp, p, jla) * hpr.one(p, ha));
          o.bb[e] = (short)bf16_bits(row_at<BF>(rowbuf, clo, chp, p, jlb) * hpr.one(p, hb));
        }
      };
      Ops cur, nxt;
      if (nsteps > 0) load(0, cur);
      for (int st = 0; st < nsteps; ++st) {
        load(st + 1 < nsteps ? st + 1 : st, nxt);
        acca = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(cur.aa, cur.ba, acca, 0, 0, 0);
        accb = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(cur.ab, cur.bb, accb, 0, 0, 0);
        cur = nxt;
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int jra = 16 * t0a + 4 * kq + i, jrb = 16 * t0b + 4 * kq + i;
      if (jra < J0 && cola < ncol) out[jra + J0 * cola] = acca[i];
      if (has2 && jrb < J0 && colb < ncol) out[jrb + J0 * colb] = accb[i];
    }
  }
}

// The core gradient of a four-mode tensor with equal ranks, as one balanced
// GEMM: rows (j0, j1) = j0 + J j1, columns h = (j2, j3) (the hp index),
// dG[row, h] = sum_p (r_p a(0)_p[j0] a(1)_p[j1]) hp_p[h], K = the chunk's
// samples; lin = row + J^2 h.  A wave takes one 16-row tile and up to four
// 16-column tiles, so each A operand feeds four MFMA chains.
template <int JR, bool BF>
__device__ __forceinline__ void mfma_core_grad4(const PhaseTab& g, const float* rowbuf, const float* ra, int ras,
                                                const float* hp, int hs, int cnt, int chp, float* out) {
  constexpr int R = JR * JR;            // rows and columns
  constexpr int T16 = (R + 15) / 16;    // tiles per side
  constexpr int CG = T16 < 4 ? T16 : 4; // column tiles per job
  constexpr int NCG = (T16 + CG - 1) / CG;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int clo = g.c_lo;
  for (int job = wv; job < T16 * NCG; job += nwaves) {
    const int rt = job / NCG, cg0 = (job - rt * NCG) * CG;
    const int row = min(rt * 16 + r16, R - 1);
    const int j0 = row % JR, j1 = row / JR;
    int colc[CG];
#pragma unroll
    for (int c = 0; c < CG; ++c) colc[c] = min((cg0 + c) * 16 + r16, R - 1);
    f32x4 acc[CG];
#pragma unroll
    for (int c = 0; c < CG; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (!BF) {
      // K in groups of four steps (16 samples), the next group's operands
      // read before the current group's MFMAs.  No masks: ra is zero for
      // p >= cnt and every value read is finite.
      const int ngroups = (cnt + 15) >> 4;
      struct Ops {
        float av[4], bv[4][CG];
      };
      auto load = [&](int gi, Ops& o) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int p = (4 * gi + u) * 4 + kq;
          o.av[u] = ra[p * ras + j0] * rowbuf[((clo + (j1 >> 2)) * chp + p) * 4 + (j1 & 3)];
#pragma unroll
          for (int c = 0; c < CG; ++c) o.bv[u][c] = hp[colc[c] * hs + p];
        }
      };
      Ops cur, nxt;
      if (ngroups > 0) load(0, cur);
      for (int gi = 0; gi < ngroups; ++gi) {
        load(gi + 1 < ngroups ? gi + 1 : gi, nxt);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
          for (int c = 0; c < CG; ++c)
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur.av[u], cur.bv[u][c], acc[c], 0, 0, 0);
        }
        cur = nxt;
      }
    } else {
      const int nsteps = (cnt + 15) >> 4;  // 16 * nsteps <= chp
      for (int st = 0; st < nsteps; ++st) {
        const int p0 = st * 16 + 4 * kq;
        s16x4 av;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          av[e] = (short)bf16_bits(ra[(p0 + e) * ras + j0] * row_at<BF>(rowbuf, clo, chp, p0 + e, j1));
        s16x4 bv[CG];
#pragma unroll
        for (int c = 0; c < CG; ++c) {
          const f32x4 h4 = *reinterpret_cast<const f32x4*>(hp + colc[c] * hs + p0);
#pragma unroll
          for (int e = 0; e < 4; ++e) bv[c][e] = (short)bf16_bits(h4[e]);
        }
#pragma unroll
        for (int c = 0; c < CG; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv[c], acc[c], 0, 0, 0);
      }
    }
#pragma unroll
    for (int c = 0; c < CG; ++c) {
      const int col = (cg0 + c) * 16 + r16;
      const int r0 = rt * 16 + 4 * kq;  // this lane's four rows r0 .. r0 + 3 are adjacent in out
      if constexpr (R % 4 == 0) {  // one 16-byte store (r0 and R multiples of four)
        if (cg0 + c < T16 && r0 < R && col < R) *reinterpret_cast<f32x4*>(out + r0 + R * col) = acc[c];
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (cg0 + c < T16 && r0 + i < R && col < R) out[r0 + i + R * col] = acc[c][i];
      }
    }
  }
}

// Copy the carry slots of parity `par` into LDS (all loads issued before the
// stores when they fit four vectors per thread).
__device__ __forceinline__ void copy_carry(const ChainArgs& a, int par, float* cbuf) {
  const int tot = (int)(((size_t)a.W * a.carry_stride) >> 2);
  const f32x4* src = reinterpret_cast<const f32x4*>(a.carry + (size_t)par * a.W * a.carry_stride);
  f32x4* dst = reinterpret_cast<f32x4*>(cbuf);
  const int BT = blockDim.x;
  for (int i0 = threadIdx.x; i0 < tot; i0 += 4 * BT) {
    f32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + u * BT < tot) v[u] = src[i0 + u * BT];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + u * BT < tot) dst[i0 + u * BT] = v[u];
  }
}

// ---------------------------------------------------------------------------
// Kruskal core sub-step (Section "Optimization Process for the Core Tensor",
// Eqs. CP-Decomposition, eventual0, Q_r, eventual_approximated,
// Gradient_core_tensor; Algorithm 1, core loop).  The core is the Kruskal
// product G = sum_r b(1)_r o ... o b(N)_r of B(n) in R^{J_n x R}; for each
// mode n in turn, every column b_c of B(n) in turn takes the averaged SGD
// step on (1/2m) ||x - sum_r W_r b_r||^2 + (lambda/2) ||b_c||^2 with
//   W_r[p, a] = a(n)_p[a] prod_{k != n} (a(k)_p . b(k)_r)
// (the rows of H_Psi O_r, which depend on the other modes' B only), i.e.
//   b_c <- b_c - gG ( V_c / m + lG b_c ),  V_c = -W_c^T x + sum_r W_c^T W_r b_r.
// Each workgroup forms the Gram matrix of [W_0 .. W_{R-1} | x] over its
// chunk's samples (packed upper triangle), the workgroups' matrices are
// summed in a fixed order (each reduces a slice, one grid barrier, then all
// read the sum), and every workgroup takes the R column steps identically on
// the summed matrix.  Two grid barriers per mode; then G is formed from B.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int tri_index(int e1, int e2, int ke) { return e1 * ke - ((e1 * (e1 - 1)) >> 1) + (e2 - e1); }

template <int JR, bool BF, bool EXACT>
__device__ bool kruskal_core_step(const ChainArgs& a, int w, int64_t b, int m, int cnt, const float* rowbuf, float x,
                                  unsigned& passed, int* flag_lds) {
  extern __shared__ float lds[];
  const ChainLayout& L = a.lay;
  const Shape& s = a.s;
  const int N = s.N, R = a.R, tid = threadIdx.x, BT = blockDim.x, chp = L.chp;
  const int lane = tid & 63, wv = tid >> 6, nwaves = BT >> 6, r16 = lane & 15, kq = lane >> 4;
  float* Bs = lds + L.kb;
  float* wt = lds + L.kwt;
  float* g = lds + L.kg;  // full symmetric matrix, ke x ke (row stride ke)
  const int klgp = pad4(L.klg);
  const float inv_m = 1.0f / (float)m;
  for (int n = 0; n < N; ++n) {
    const int Jn = EXACT ? JR : s.J[n];
    const int E = R * Jn;
    const int ke = E + 1;
    const int lg = (ke * (ke + 1)) >> 1;
    const int T16 = (ke + 15) >> 4;  // 16-column tiles
    const int kpar = n & 1;          // partial buffers alternate between modes
    // 1. rows of [W_0 .. W_{R-1} | x] for the chunk's samples (zero beyond the
    //    count and in the padding columns up to the tile edge)
    if (tid < chp) {
      float* wrow = wt + tid * L.kws;
      if (tid < cnt) {
        float an[JR];
        read_row<JR, BF, EXACT>(rowbuf, L.coff[n], chp, tid, Jn, an);
        for (int c0 = 0; c0 < R; c0 += 8) {  // eight columns at a time, the other modes' rows in registers
          float q[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) q[u] = 1.f;
          for (int k = 0; k < N; ++k) {
            if (k == n) continue;
            const int Jk = EXACT ? JR : s.J[k];
            float rk[JR];
            read_row<JR, BF, EXACT>(rowbuf, L.coff[k], chp, tid, Jk, rk);
            const float* bk = Bs + L.kboff[k] + c0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              if (c0 + u < R) {
                float d = 0.f;
#pragma unroll
                for (int j = 0; j < JR; ++j)
                  if (EXACT || j < Jk) d = fmaf(rk[j], bk[j * R + u], d);
                q[u] *= d;
              }
            }
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (c0 + u < R) {
#pragma unroll
              for (int aa = 0; aa < JR; ++aa)
                if (EXACT || aa < Jn) wrow[(c0 + u) * Jn + aa] = an[aa] * q[u];
            }
          }
        }
        wrow[E] = x;
      } else {
        for (int e = 0; e < ke; ++e) wrow[e] = 0.f;
      }
      for (int e = ke; e < 16 * T16; ++e) wrow[e] = 0.f;
    }
    __syncthreads();
    // 2. this chunk's Gram matrix [W|x]^T [W|x] (MFMA 16x16x4, K = samples):
    //    the upper-triangle tile pairs, one per wave at a time, the operands of
    //    the next four K steps read before the MFMAs of these; only entries
    //    e1 <= e2 < ke are stored (packed upper triangle)
    {
      float* part = a.partial + ((size_t)kpar * a.W + w) * klgp;
      const int npairs = (T16 * (T16 + 1)) >> 1;
      const int ngroups = chp >> 4;  // four K steps (16 samples) per group; chp is a multiple of 32
      for (int pi = wv; pi < npairs; pi += nwaves) {
        int ti = 0, rem = pi;
        while (rem >= T16 - ti) {
          rem -= T16 - ti;
          ++ti;
        }
        const int tj = ti + rem;
        const float* colA = wt + 16 * ti + r16;
        const float* colB = wt + 16 * tj + r16;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        float av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          av[u] = colA[(4 * u + kq) * L.kws];
          bv[u] = colB[(4 * u + kq) * L.kws];
        }
        for (int gi = 0; gi < ngroups; ++gi) {
          const int gn = gi + 1 < ngroups ? gi + 1 : gi;
          float an2[4], bn2[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            an2[u] = colA[(16 * gn + 4 * u + kq) * L.kws];
            bn2[u] = colB[(16 * gn + 4 * u + kq) * L.kws];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], bv[u], acc, 0, 0, 0);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            av[u] = an2[u];
            bv[u] = bn2[u];
          }
        }
        const int e2 = 16 * tj + r16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e1 = 16 * ti + 4 * kq + i;
          if (e1 <= e2 && e2 < ke) part[tri_index(e1, e2, ke)] = acc[i];
        }
      }
    }
    passed += 1;
    barrier_arrive<false>(a, w, passed);
    if (!barrier_wait<false>(a, passed, flag_lds)) return false;
    // 3. this workgroup's slice of the sum over workgroups (groups of threads
    //    add runs of workgroups in order, eight loads in flight, then the
    //    groups are added in order)
    {
      const float* pb = a.partial + (size_t)kpar * a.W * klgp;
      float* gs = a.partial + (size_t)2 * a.W * klgp + (size_t)kpar * klgp;
      const int per = (lg + a.W - 1) / a.W;
      const int e0 = w * per, e1 = min(lg, e0 + per);
      if (per <= BT) {
        const int ng = min(BT / per, a.W), vg = (a.W + ng - 1) / ng;
        const int i = tid % per, grp = tid / per;
        if (grp < ng) {
          float sum = 0.f;
          const int e = min(e0 + i, lg - 1);
          const int v1 = min(a.W, (grp + 1) * vg);
          for (int v = grp * vg; v < v1; v += 8) {
            float t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = pb[(size_t)min(v + u, a.W - 1) * klgp + e];
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (v + u < v1) sum += t[u];
          }
          g[grp * per + i] = sum;
        }
        __syncthreads();
        if (tid < per && e0 + tid < e1) {
          float sum = 0.f;
          for (int g2 = 0; g2 < ng; ++g2) sum += g[g2 * per + tid];
          gs[e0 + tid] = sum;
        }
      } else {
        for (int e = e0 + tid; e < e1; e += BT) {
          float sum = 0.f;
          for (int v = 0; v < a.W; v += 8) {
            float t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = pb[(size_t)min(v + u, a.W - 1) * klgp + e];
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (v + u < a.W) sum += t[u];
          }
          gs[e] = sum;
        }
      }
    }
    passed += 1;
    barrier_arrive<false>(a, w, passed);
    if (!barrier_wait<false>(a, passed, flag_lds)) return false;
    // 4. the summed matrix (every workgroup): the packed triangle into the
    //    [W | x] region, which the Gram is done with (coalesced, eight loads in
    //    flight), then unpacked within LDS
    {
      const float* gs = a.partial + (size_t)2 * a.W * klgp + (size_t)kpar * klgp;
      for (int e0 = tid; e0 < lg; e0 += 8 * BT) {
        float t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = gs[min(e0 + u * BT, lg - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (e0 + u * BT < lg) wt[e0 + u * BT] = t[u];
      }
      __syncthreads();
      for (int r1 = wv; r1 < ke; r1 += nwaves)
        for (int c1 = lane; c1 < ke; c1 += 64)
          g[r1 * ke + c1] = wt[r1 <= c1 ? tri_index(r1, c1, ke) : tri_index(c1, r1, ke)];
    }
    __syncthreads();
    // 5. the column steps, c = 0 .. R-1 in order, by wave 0 alone: row a of
    //    V_c by a group of tpr lanes (a power of two), summed by xor shuffles.
    //    Within one wave LDS operations complete in program order, so every
    //    lane's read of b_c precedes the write of its new value, and that
    //    write precedes the next column's reads; no workgroup barrier is needed.
    if (wv == 0) {
      float* Bn = Bs + L.kboff[n];
      int tpr = 64;
      while (tpr > 1 && tpr * Jn > 64) tpr >>= 1;
      const int ra = lane / tpr, l = lane % tpr;
      for (int c = 0; c < R; ++c) {
        float V = 0.f;
        if (ra < Jn) {
          const float* grow = g + (c * Jn + ra) * ke;
          for (int e2 = l; e2 < E; e2 += tpr) {
            const int r = e2 / Jn, bb = e2 - r * Jn;
            V = fmaf(grow[e2], Bn[bb * R + r], V);
          }
        }
        for (int off = 1; off < tpr; off <<= 1) V += __shfl_xor(V, off, 64);
        float old = 0.f;
        if (ra < Jn) {
          V -= g[(c * Jn + ra) * ke + E];  // - (W_c^T x)[a]
          old = Bn[ra * R + c];
        }
        if (ra < Jn && l == 0) {
          const float nb = old - a.gG * (V * inv_m + a.lG * old);
          Bn[ra * R + c] = nb;
          if (!__builtin_isfinite(nb)) report_nonfinite(a, nf_key(b, 0, L.kboff[n] + ra * R + c));
        }
      }
    }
    __syncthreads();
  }
  // 6. the core of the updated B, G[lin] = sum_r prod_k B(k)[j_k, r], by
  //    halves of the modes: Lf[jl][r] = prod_{k < h} B(k)[j_k, r] and
  //    Rf[jr][r] = prod_{k >= h} B(k)[j_k, r] (in the [W | x] region), then
  //    G[jl + PL jr] = sum_r Lf[jl][r] Rf[jr][r]
  {
    float* Gs = lds + L.gs;
    const int h = N >> 1, PL = s.lstride[h], PR = s.P / PL;
    float* Lf = wt;
    float* Rf = wt + PL * R;
    for (int e = tid; e < (PL + PR) * R; e += BT) {
      const bool left = e < PL * R;
      const int e2 = left ? e : e - PL * R;
      const int jx = e2 / R, r = e2 - jx * R;
      const int lin = left ? jx : jx * PL;
      float t = 1.f;
      for (int k = left ? 0 : h; k < (left ? h : N); ++k) t *= Bs[L.kboff[k] + ((lin / s.lstride[k]) % s.J[k]) * R + r];
      wt[e] = t;
    }
    __syncthreads();
    for (int lin = tid; lin < s.P; lin += BT) {
      const int jr = lin / PL, jl = lin - jr * PL;
      float acc = 0.f;
      for (int r = 0; r < R; ++r) acc = fmaf(Lf[jl * R + r], Rf[jr * R + r], acc);
      Gs[lin] = acc;
    }
  }
  __syncthreads();
  return true;
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
//   table; workgroup w stores the entries e with e mod W = w; until the next
//   barrier nobody else reads them from global memory, and the rows of that
//   mode are read after the barrier that follows).
// Carry layout: at finish_split_rows.
// ---------------------------------------------------------------------------
template <int JU, int NU, int BFI>
__device__ __forceinline__ void chain_body(const ChainArgs& a, const int w) {
  constexpr int JR = JU ? JU : kMaxRank;
  constexpr int NM = NU ? NU : kMaxOrder;  // modes the per-mode loops cover
  constexpr bool EXACT = JU != 0;
  constexpr bool BF = (BFI & 1) != 0;
  constexpr bool KR = (BFI & 2) != 0;  // Kruskal core (a.R > 0)
  constexpr bool MOM = (BFI & 4) != 0;  // heavy-ball momentum (a.mom; never with the Kruskal core)
  constexpr bool XL = (BFI & 8) != 0;   // one-XCC barrier (a.xid >= 0; dense core, no momentum)
  constexpr bool TS = NU != 3;  // two-stage contraction (layout of the tables)
  extern __shared__ float lds[];
  const Shape& s = a.s;
  const int N = NU ? NU : s.N;
  const int P = s.P;
  const int Pp = pad4(P);
  const int tid = threadIdx.x;
  const int BT = blockDim.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const ChainLayout& L = a.lay;
  const bool CORE2 = !KR && NU != 3 && L.core2;  // two-level core update (never planned for three modes)

  float* Gs = lds + L.gs;
  float* vgs = lds + L.vg;  // momentum: the core velocity this workgroup updates
  float* TB = lds + L.tb;
  float* const rows0 = lds + L.row0;  // the two row buffers (rows1 = rows0 + rowsz), one per sub-step in turn
  float* const rows1 = lds + L.row1;
  float* hp = lds + L.hp;
  float* ebuf = lds + L.ebuf;
  float* rabuf = lds + L.ra;
  float* split = lds + L.split;
  float* cbuf = lds + L.cbuf;
  int* hmap = reinterpret_cast<int*>(lds + L.hmap);
  int* tmap = reinterpret_cast<int*>(lds + L.tmap);
  float* wscr = lds + L.wscr;
  int* ints = reinterpret_cast<int*>(lds + L.ints);
  int* xa = ints;            // W  straddling rows of the previous sub-step's boundaries
  int* xn = xa + a.W;        // W  their entry numbers
  int* misc = xn + a.W;      // 8
  const int chp = L.chp, es = L.es, ras = L.ras, sstride = L.sstride, wstride = L.wstride;
  const unsigned allm = (1u << N) - 1u;
  const int XS = xrow_stride(a.W);
  const size_t carry_par_stride = (size_t)a.W * a.carry_stride;
  const int64_t T = a.T, M = a.M;

  // ---- set-up: core, index maps, resident tables
  for (int lin = tid; lin < P; lin += BT) Gs[lin] = a.G[lin];
  if constexpr (MOM) {
    if (CORE2) {  // this workgroup's slice of the velocity (the slice of G it updates)
      for (int i = tid; i < 4 * L.cper; i += BT) {
        const int lin = 4 * w * L.cper + i;
        vgs[i] = lin < P ? a.VG[lin] : 0.f;
      }
    } else {
      for (int lin = tid; lin < P; lin += BT) vgs[lin] = a.VG[lin];
    }
  }
  if constexpr (KR) {
    const int nb = L.kboff[N - 1] + s.J[N - 1] * a.R;
    for (int i = tid; i < nb; i += BT) lds[L.kb + i] = a.B[i];
  }
  // (both row buffers and a zero tail: the MFMA K steps read up to 31 words past a row)
  for (int i = tid; i < 2 * L.rowsz + kRowTail; i += BT) rows0[i] = 0.f;
  for (int i = tid; i < L.aux_len; i += BT) {
    const int v = a.aux[i];
    if (i < L.hm_len) hmap[i] = v;
    else tmap[i - L.hm_len] = v;
  }
  if (!L.tb_all) build_table_arith<JR, BF, EXACT, TS>(a.pt[1], Gs, hmap, TB, true);
  __syncthreads();
  // (one table region: each phase's table is built in the previous phase's
  // barrier window, the first here, and mode 0's after the core update)
  if (!L.tb_all) build_table_arith<JR, BF, EXACT, TS>(a.pt[0], Gs, hmap + a.pt[0].hm_off, TB);
  if (L.tb_all) {
    for (int n = 0; n < N; ++n) {
      const PhaseTab& q = a.pt[n + 1];
      build_table_map<BF>(Gs, tmap + q.tb_off, q.tb_len, BF ? TB + (q.tb_off >> 1) : TB + q.tb_off);
    }
  }

  unsigned passed = a.passed0;
  int ppar = 0;  // carry parity written by the previous phase
  int par = 0;   // carry parity of the current phase
  bool first = true;

  // records of this phase (cur) and the next (nx); the one after is read in
  // each phase's barrier window
  LaneRec<NM> cur, nx;
  if (a.b_begin < a.b_end) {
    load_lane_rec<NM>(a, w, N, a.b_begin, 0, cur);
    load_lane_rec<NM>(a, w, N, a.b_begin, 1, nx);
  } else {
    cur.valid = nx.valid = false;
  }
  int bsel = 0;  // which row buffer holds the current sub-step's rows
  float an_cur[JR], an_nxt[JR];  // BF16 mode: FP32 master row of the lane's own-mode row
#pragma unroll
  for (int j = 0; j < JR; ++j) an_cur[j] = an_nxt[j] = 0.f;

  for (int64_t b = a.b_begin; b < a.b_end; ++b) {
    const int64_t base = b * M;
    const int m = (int)((T - base < M) ? (T - base) : M);
    const int lo = w * a.chunk;
    const int cnt = max(0, min(a.chunk, m - lo));

    for (int ph = 0; ph <= N; ++ph) {
      const PhaseTab& pt = a.pt[ph];
      const int n = pt.n;
      const int Jn = EXACT ? JR : pt.Jn;
      const int pm = first ? -1 : pt.pm;
      const bool active = tid < cnt;
      const bool splits = pm >= 0 && a.W > 1;
      float* const rowbuf = bsel ? rows1 : rows0;
      float* const rownext = bsel ? rows0 : rows1;

      // ---- 1. after the barrier, one batch of loads: the rows of the modes
      //      the two previous phases updated, the carry slots and boundary
      //      rows of the previous phase, the first core partials
      const int P4 = Pp >> 2;
      const f32x4* psrc = reinterpret_cast<const f32x4*>(a.partial);
      f32x4 pp[8];  // core phase 1: the first 8 workgroups' partials of column tid
      {
        const unsigned post = first ? allm : ((unsigned)pt.post & allm);
        const int64_t bp = ph == 0 ? b - 1 : b;
        const int* xsrc = a.xrow + ((size_t)(splits ? bp : 0) * N + (splits ? pm : 0)) * XS;
        const int ctot = (int)(carry_par_stride >> 2);
        const f32x4* csrc = reinterpret_cast<const f32x4*>(a.carry + (size_t)ppar * carry_par_stride);
        f32x4 cv[4];
        int xv = -1, xnv = -1, xc = 0;
        if (splits) {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (tid + u * BT < ctot) cv[u] = csrc[tid + u * BT];
          if (tid < a.W) {
            xv = xsrc[tid];
            xnv = xsrc[a.W + tid];
          }
          if (tid == 0) xc = xsrc[2 * a.W];
        }
        if (!KR && ph == 1 && !CORE2 && tid < P4) {
#pragma unroll
          for (int v = 0; v < 8; ++v)
            if (v < a.W) pp[v] = psrc[(size_t)v * P4 + tid];
        }
        if (ph == 1 && CORE2) {  // this thread's share of the workgroup's slice
          const int i = tid % L.cper, grp = tid / L.cper;
          const int l4 = min(w * L.cper + i, P4 - 1);
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int v = min(grp * L.cvg + u, a.W - 1);
            if (u < L.cvg) pp[u] = psrc[(size_t)v * P4 + l4];
          }
        }
        issue_rows_lds<JR, BF, EXACT, NM>(a, cur.idx, post, rowbuf, chp, active);
        if (splits) {
          f32x4* cdst = reinterpret_cast<f32x4*>(cbuf);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (tid + u * BT < ctot) cdst[tid + u * BT] = cv[u];
          for (int i = tid + 4 * BT; i < ctot; i += BT) cdst[i] = csrc[i];
          for (int bw = tid; bw < a.W; bw += BT) {
            xa[bw] = bw == tid ? xv : xsrc[bw];
            xn[bw] = bw == tid ? xnv : xsrc[a.W + bw];
          }
          if (tid == 0) misc[0] = xc;
        }
      }
      __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);  // the rows written straight into LDS have landed
      __syncthreads();
      // the next phase (its record nx was read one phase ahead)
      int nph = ph + 1;
      int64_t nbb = b;
      if (nph > N) {
        nph = 0;
        ++nbb;
      }
      const bool has_next = nbb < a.b_end;

      // ---- 2. core: finish the core step of this minibatch
      if (KR && ph == 1) {
        // (the Kruskal core sub-step formed G in phase 0)
        if (L.tb_all)
          build_table_map<BF>(Gs, tmap + pt.tb_off, pt.tb_len, BF ? TB + (pt.tb_off >> 1) : TB + pt.tb_off);
      } else if (ph == 1 && CORE2) {
        // two levels: this workgroup's slice of G, one grid barrier, then all of G
        f32x4* red = reinterpret_cast<f32x4*>(lds + L.red);
        const int i = tid % L.cper, grp = tid / L.cper;
        if (grp < L.cgrp) {
          f32x4 sum = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (u < L.cvg && grp * L.cvg + u < a.W) sum += pp[u];
          red[grp * L.cper + i] = sum;
        }
        __syncthreads();
        const int l4 = w * L.cper + tid;
        if (tid < L.cper && l4 < P4) {
          f32x4 sum = {0.f, 0.f, 0.f, 0.f};
          // the groups in order, eight loads in flight
          for (int g0 = 0; g0 < L.cgrp; g0 += 8) {
            f32x4 t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = red[min(g0 + u, L.cgrp - 1) * L.cper + tid];
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (g0 + u < L.cgrp) sum += t[u];
          }
          const float inv_m = 1.0f / (float)m;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int lin = 4 * l4 + e;
            if (lin < P) {
              float st = -sum[e] * inv_m + a.lG * Gs[lin];
              if constexpr (MOM) {
                st = a.mu * vgs[4 * tid + e] + st;
                vgs[4 * tid + e] = st;
              }
              const float g = Gs[lin] - a.gG * st;
              a.G[lin] = g;
              if (!__builtin_isfinite(g)) report_nonfinite(a, nf_key(b, 0, lin));
            }
          }
        }
        passed += 1;
        barrier_arrive<XL>(a, w, passed);
        if (!barrier_wait<XL>(a, passed, misc + 7)) return;
        // (all of a thread's loads issued before its first LDS store: one round trip)
        for (int l0 = tid; l0 < P4; l0 += 4 * BT) {
          float gv[4][4];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) gv[u][e] = a.G[min(4 * (l0 + u * BT) + e, P - 1)];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (4 * (l0 + u * BT) + e < P) Gs[4 * (l0 + u * BT) + e] = gv[u][e];
        }
        __syncthreads();
        if (L.tb_all)  // mode 0's table now; the others after this phase's arrival
          build_table_map<BF>(Gs, tmap + pt.tb_off, pt.tb_len, BF ? TB + (pt.tb_off >> 1) : TB + pt.tb_off);
      } else if (ph == 1) {
        const float inv_m = 1.0f / (float)m;
        for (int l4 = tid; l4 < P4; l4 += BT) {
          f32x4 sum = {0.f, 0.f, 0.f, 0.f};
          int v0 = 0;
          if (l4 == tid) {  // the loads issued with the batch
#pragma unroll
            for (int v = 0; v < 8; ++v)
              if (v < a.W) sum += pp[v];
            v0 = 8;
          }
          for (int vb = v0; vb < a.W; vb += 16) {  // 16 loads in flight, summed in order
            f32x4 t[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) t[u] = psrc[(size_t)min(vb + u, a.W - 1) * P4 + l4];
#pragma unroll
            for (int u = 0; u < 16; ++u)
              if (vb + u < a.W) sum += t[u];
          }
          float gv[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) gv[i] = Gs[min(4 * l4 + i, P - 1)];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (4 * l4 + i < P) {
              float st = -sum[i] * inv_m + a.lG * gv[i];
              if constexpr (MOM) {
                st = a.mu * vgs[4 * l4 + i] + st;
                vgs[4 * l4 + i] = st;
              }
              const float g = gv[i] - a.gG * st;
              Gs[4 * l4 + i] = g;
              // (every workgroup checks its own copy before it writes any row of this phase)
              if (!__builtin_isfinite(g)) report_nonfinite(a, nf_key(b, 0, 4 * l4 + i));
            }
          }
        }
        __syncthreads();
        if (L.tb_all)  // mode 0's table now; the others after this phase's arrival
          build_table_map<BF>(Gs, tmap + pt.tb_off, pt.tb_len, BF ? TB + (pt.tb_off >> 1) : TB + pt.tb_off);
      }
      if (!L.tb_all && ph == 1) build_table_arith<JR, BF, EXACT, TS>(pt, Gs, hmap + pt.hm_off, TB);

      // ---- 3. rows of the previous factor sub-step that straddled chunks
      if (splits) {
        const int nsplit = misc[0];
        finish_split_rows<JR, EXACT, BF, NU != 3, MOM>(a, pm, xa, xn, nsplit, cbuf, split, sstride, w, a.W,
                                                       ph == 0 ? b - 1 : b);
        // the schedule says which entry (if any) holds this sample's mode-pm row
        const int pe = (cur.meta >> kMetaPatchShift) & 0xFF;
        if (active && pe > 0) {
          const int pJ = EXACT ? JR : s.J[pm];
          const float* ent = split + (pe - 1) * sstride + 4;
          float v[JR];
#pragma unroll
          for (int j = 0; j < JR; ++j) v[j] = (EXACT || j < pJ) ? ent[j] : 0.f;
          write_row<JR, BF, EXACT>(rowbuf, L.coff[pm], chp, tid, pJ, v);
        }
      }

      // ---- 4. the next phase's rows that no phase writes before it: straight
      //      into the other row buffer (they land before this phase's arrival)
      if (has_next) {
        const unsigned pre = allm & ~(unsigned)a.pt[nph].post;
        if (pre) issue_rows_lds<JR, BF, EXACT, NM>(a, nx.idx, pre, rownext, chp, nx.valid);
      }
      if (BF && has_next && nx.valid && nph > 0) {
        const float* src = a.A[a.pt[nph].n] + (int64_t)nx.rown * s.Jp[a.pt[nph].n];
        const int Jx = EXACT ? JR : a.pt[nph].Jn;
#pragma unroll
        for (int j = 0; j < JR; ++j)
          if (EXACT || j < Jx) an_nxt[j] = src[j];
      }

      // ---- 5. E_p for every sample of the chunk
      constexpr bool HPV = NU == 3;  // one remaining mode: hp is a view of its rows
      HpRef<HPV, BF> hpr;
      if (KR && ph == 0) {
        // ================= Kruskal core sub-step =================
        __syncthreads();  // (rows patched by other threads above)
        if (!kruskal_core_step<JR, BF, EXACT>(a, w, b, m, cnt, rowbuf, cur.x, passed, misc + 7)) return;
      } else {
      if constexpr (HPV) {
        hpr = HpRef<HPV, BF>{rowbuf, chp, pt.c_hi};
      } else {
        // (build_hp2 reads other threads' samples: the patched rows must have landed)
        if (splits && EXACT && pt.nhi == 2) __syncthreads();
        if (EXACT && pt.nhi == 2) build_hp2<JR, BF>(pt, rowbuf, cnt, chp, hp, L.hs);
        else build_hp<BF>(pt, rowbuf, hmap + pt.hm_off, cnt, chp, hp, L.hs);
        hpr = HpRef<HPV, BF>{hp, L.hs, 0};
      }
      __syncthreads();
      const float* TBn = L.tb_all ? (BF ? TB + (pt.tb_off >> 1) : TB + pt.tb_off) : TB;
      constexpr int KHI = (EXACT && NU == 3) ? JR : 0;  // h trip count of three-mode equal-rank kernels
      if constexpr (!HPV) {
        mfma_E<JR, BF, EXACT, HPV, KHI, 1>(s, pt, TBn, rowbuf, hpr, cnt, chp, ebuf, es);
      } else {
        if (((cnt + 15) >> 4) * pt.nt <= (BT >> 6))  // enough waves for one tile each
          mfma_E<JR, BF, EXACT, HPV, KHI, 1>(s, pt, TBn, rowbuf, hpr, cnt, chp, ebuf, es);
        else
          mfma_E<JR, BF, EXACT, HPV, KHI, 2>(s, pt, TBn, rowbuf, hpr, cnt, chp, ebuf, es);
      }
      __syncthreads();

      if (ph == 0) {
        // ================= core sub-step =================
        if (tid < chp) {
          float r = 0.f, a0r[JR];
          read_row<JR, BF, EXACT>(rowbuf, pt.c_n, chp, min(tid, chp - 1), Jn, a0r);
          if (active) {
            float ev[JR];
            read_e<JR, EXACT>(ebuf + tid * es, pt.ens, Jn, ev);
            float xh = 0.f;
#pragma unroll
            for (int j = 0; j < JR; ++j)
              if (EXACT || j < Jn) xh = fmaf(a0r[j], ev[j], xh);
            r = cur.x - xh;
          }
#pragma unroll
          for (int j = 0; j < JR; ++j)
            if (EXACT || j < Jn) rabuf[tid * ras + j] = active ? r * a0r[j] : 0.f;
        }
        __syncthreads();
        // (the core-gradient tiles reuse hp of mode 0: the remaining modes of mode 1's columns)
        if (!HPV && EXACT && pt.nhi == 2)
          mfma_core_grad4<JR, BF>(pt, rowbuf, rabuf, ras, hp, L.hs, cnt, chp, a.partial + (size_t)w * Pp);
        else
          mfma_core_grad<JR, BF, EXACT, HPV>(s, pt, rowbuf, rabuf, ras, hpr, cnt, chp, a.partial + (size_t)w * Pp);
      } else {
        // ================= mode-n sub-step =================
        float u[JR], an[JR], vold[JR];
#pragma unroll
        for (int j = 0; j < JR; ++j) u[j] = an[j] = vold[j] = 0.f;
        if (active) {
          // momentum: the old velocity of the row whose run ends at this lane
          // (only this sub-step and the finish of its straddling rows write
          // velocities of this mode; read here, where few registers are live)
          if (MOM && (cur.meta & kMetaTail)) {
            const float* src = a.VA[n] + (int64_t)cur.rown * s.Jp[n];
#pragma unroll
            for (int j = 0; j < JR; ++j)
              if (EXACT || j < Jn) vold[j] = src[j];
          }
          float xh = 0.f, av[JR], ev[JR];
          read_row<JR, BF, EXACT>(rowbuf, pt.c_n, chp, tid, Jn, av);
          read_e<JR, EXACT>(ebuf + tid * es, pt.ens, Jn, ev);
#pragma unroll
          for (int j = 0; j < JR; ++j) {
            if (EXACT || j < Jn) {
              const float e = ev[j];
              an[j] = BF ? an_cur[j] : av[j];
              xh = fmaf(av[j], e, xh);
              u[j] = e;
            }
          }
          const float r = cur.x - xh;
#pragma unroll
          for (int j = 0; j < JR; ++j)
            if (EXACT || j < Jn) u[j] = -r * u[j];
        }
        // wave-level segmented inclusive scan of u (Hillis-Steele, fixed order);
        // sf = first chunk position of my row's run (from the schedule)
        const int meta = cur.meta;
        const int sf = meta & 511;
        const int wstart = max(sf, wv * 64) - wv * 64;
        wave_segmented_scan<JR, EXACT>(u, Jn, lane, wstart);
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
        if (active && (meta & kMetaTail)) {
          const int row = cur.rown;
          const int c = tid - sf + 1;
          const bool before = (meta & kMetaBefore) != 0;  // run began in an earlier chunk
          const bool after = (meta & kMetaAfter) != 0;    // run goes on in the next chunk
          if (!before && !after) {
            float* arow = a.A[n] + (int64_t)row * s.Jp[n];
            unsigned short* brow = BF ? a.Ab[n] + (int64_t)row * a.Jb[n] : nullptr;
            float* vrow = a.VA[n] + (int64_t)row * s.Jp[n];  // (momentum only)
            const float inv_c = 1.0f / (float)c;
            bool fin = true;
#pragma unroll
            for (int j = 0; j < JR; ++j) {
              if (EXACT || j < Jn) {
                float st = u[j] * inv_c + a.lA * an[j];
                if constexpr (MOM) {
                  st = a.mu * vold[j] + st;
                  vrow[j] = st;
                }
                const float v = an[j] - a.gA * st;
                arow[j] = v;
                if (BF) brow[j] = bf16_bits(v);
                fin = fin && __builtin_isfinite(v);
              }
            }
            if (!fin) report_nonfinite(a, nf_key(b, ph, row));
          } else {
            // the carry of this chunk (layout at finish_split_rows): the run's
            // slot, and the old row (and velocity) if the run begins here
            const int NS = 2 * a.W;
            float* base = a.carry + (size_t)par * carry_par_stride;
            float* slot = base + (size_t)w * 2 + (before ? 0 : 1);
            float* rowB = base + (size_t)(2 + Jn) * NS + w;
            slot[0] = __int_as_float(row);
            slot[NS] = __int_as_float(c);
#pragma unroll
            for (int j = 0; j < JR; ++j) {
              if (EXACT || j < Jn) {
                slot[(size_t)(2 + j) * NS] = u[j];
                if (!before) {
                  rowB[(size_t)j * a.W] = an[j];
                  if (MOM) rowB[(size_t)(Jn + j) * a.W] = vold[j];
                }
              }
            }
          }
        }
      }
      }  // (Kruskal core sub-step, or the contraction and the sub-step)
      // ---- 6. barrier: the next sub-step needs this one's result.  Between
      //      arrival and wait (no reads of what other workgroups write): build
      //      the resident tables the core update changed, or, with one table
      //      region, the next phase's table.
      passed += 1;
      barrier_arrive<XL>(a, w, passed);
      if (ph == 1 && L.tb_all) {
        for (int n2 = 1; n2 < N; ++n2) {
          const PhaseTab& q = a.pt[n2 + 1];
          build_table_map<BF>(Gs, tmap + q.tb_off, q.tb_len, BF ? TB + (q.tb_off >> 1) : TB + q.tb_off);
        }
      }
      if (!L.tb_all && has_next && nph != 1)  // (this phase's contraction is done: the arrival synchronised)
        build_table_arith<JR, BF, EXACT, TS>(a.pt[nph], Gs, hmap + a.pt[nph].hm_off, TB);
      // the record of the phase after next (read-only schedule data)
      LaneRec<NM> nx2;
      {
        int ph2 = nph + 1;
        int64_t b2 = nbb;
        if (ph2 > N) {
          ph2 = 0;
          ++b2;
        }
        if (b2 < a.b_end) load_lane_rec<NM>(a, w, N, b2, ph2, nx2);
        else nx2.valid = false;
      }
      if (!barrier_wait<XL>(a, passed, misc + 7)) return;
      first = false;
      bsel ^= 1;
      cur = nx;
      nx = nx2;
#pragma unroll
      for (int j = 0; j < JR; ++j) an_cur[j] = an_nxt[j];
      ppar = par;
      par ^= 1;
    }
  }
  // ---- flush: rows of the last factor sub-step that straddled chunks
  if (!first && a.W > 1 && w == 0) {
    const int pm = N - 1;
    const int* xsrc = a.xrow + ((size_t)(a.b_end - 1) * N + pm) * XS;
    for (int bw = tid; bw < a.W; bw += BT) {
      xa[bw] = xsrc[bw];
      xn[bw] = xsrc[a.W + bw];
    }
    if (tid == 0) misc[0] = xsrc[2 * a.W];
    copy_carry(a, ppar, cbuf);
    __syncthreads();
    finish_split_rows<JR, EXACT, BF, NU != 3, MOM>(a, pm, xa, xn, misc[0], cbuf, split, sstride, 0, 1, a.b_end - 1);
  }
  if constexpr (MOM) {  // the core velocity: each workgroup its slice (two levels), else workgroup 0
    if (CORE2) {
      for (int i = tid; i < 4 * L.cper; i += BT) {
        const int lin = 4 * w * L.cper + i;
        if (lin < P) a.VG[lin] = vgs[i];
      }
    } else if (w == 0) {
      for (int lin = tid; lin < P; lin += BT) a.VG[lin] = vgs[lin];
    }
  }
  if (w == 0) {
    for (int lin = tid; lin < P; lin += BT) a.G[lin] = Gs[lin];
    if constexpr (KR) {
      const int nb = L.kboff[N - 1] + s.J[N - 1] * a.R;
      for (int i = tid; i < nb; i += BT) a.B[i] = lds[L.kb + i];
    }
  }
}

template <int JU, int NU, int BFI>
__global__ __launch_bounds__(kChainThreads) void k_chain(ChainArgs a) {
  const int w = chain_workgroup<(BFI & 8) != 0>(a);
  if (w < 0) return;
  chain_body<JU, NU, BFI>(a, w);
}

// Many independent chains in one cooperative launch (a batch of tensors):
// slot q = the workgroups [q W, (q + 1) W) runs its list of chains one after
// another, workgroup w of the slot as workgroup w of each chain.  The slot's
// barrier flags keep counting from one chain to the next (each chain's
// passed0 says where it starts), so nothing is reset between chains.  The
// lists are balanced on the host (longest first, to the least loaded slot).
template <int NU, int BFI>
__global__ __launch_bounds__(kChainThreads) void k_chain_queue(const ChainArgs* __restrict__ all,
                                                               const int* __restrict__ list, int nslots, int W) {
  const int q = blockIdx.x / W, w = blockIdx.x - q * W;
  const int* models = list + nslots + 1;
  for (int i = list[q]; i < list[q + 1]; ++i) {
    const ChainArgs& a = all[models[i]];
    // (the body a chain runs alone, so that results are bit-identical)
    STDK_FOR_VARIANT(a.jv, (chain_body<JU, NU, BFI>(a, w)));
    // a workgroup of this chain gave up waiting: the slot's flags no longer
    // count in step, so the slot stops (the host reports the error)
    if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  }
}

// Cooperative launches of the chain kernels (the LDS is the plan's, set as the
// kernel's dynamic shared memory).
template <int JU, int NU, int BFI>
hipError_t launch_chain_t(const ChainArgs& a, int threads, size_t bytes, hipStream_t st) {
  ChainArgs args = a;
  void* params[] = {&args};
  hipError_t e = hipFuncSetAttribute((const void*)k_chain<JU, NU, BFI>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e == hipSuccess)
    e = hipLaunchCooperativeKernel((const void*)k_chain<JU, NU, BFI>, dim3(a.W * a.xs), dim3(threads), params,
                                   (unsigned)bytes, st);
  return e;
}

template <int NU, int BFI>
hipError_t launch_queue_t(const ChainArgs* dev_args, const int* dev_list, int nslots, int W, int threads, size_t bytes,
                          hipStream_t st) {
  const ChainArgs* pa = dev_args;
  const int* pl = dev_list;
  void* params[] = {&pa, &pl, &nslots, &W};
  hipError_t e = hipFuncSetAttribute((const void*)k_chain_queue<NU, BFI>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e == hipSuccess)
    e = hipLaunchCooperativeKernel((const void*)k_chain_queue<NU, BFI>, dim3(nslots * W), dim3(threads), params,
                                   (unsigned)bytes, st);
  return e;
}

}  // namespace stdk
