// Internal declarations shared by the host runtime and the gfx950 kernels of
// libstdecomp.  Not part of the public C ABI (include/stdecomp.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stdk {

constexpr int kMaxOrder = 8;
constexpr int kMaxRank = 32;      // largest J_n the kernels accept
constexpr int kMaxBatch = 16384;  // largest minibatch (positions are 16-bit)
constexpr int kChainThreads = 256;
constexpr int kSortThreads = 256;
constexpr int kFlagStride = 16;   // words between two workgroups' barrier flags (64 bytes)

// Round x up to a multiple of 4 floats (16-byte factor rows).
__host__ __device__ inline int pad4(int x) { return (x + 3) & ~3; }

// Shape of a sparse Tucker model, passed by value to every kernel.
struct Shape {
  int N;                 // order
  int J[kMaxOrder];      // core ranks J_n
  int Jp[kMaxOrder];     // row stride of A(n) in floats (J_n rounded up to 4)
  int64_t I[kMaxOrder];  // mode sizes
  int P;                 // prod_n J_n
  int R;                 // words per COO record: N indices then the value bits
  int rs_off[kMaxOrder]; // offset of mode k's row inside an LDS row buffer
  int rs;                // LDS row-buffer stride per sample (odd, avoids bank conflicts)
  int lstride[kMaxOrder];// stride of j_k in the flat core: prod_{k' < k} J_k'
};

// LDS regions of a chain workgroup (float offsets) and strides.
struct ChainLayout {
  int gs, tb, row0, row1, hp, ebuf, ra, split, cbuf, hmap, tmap, wscr, ints, total;
  int chp;      // chunk rounded up to 32 (MFMA tile rows)
  int hs;       // row stride of the hp buffer (chp + 4: lanes that read different h at one
                // sample fall in different banks)
  int es;       // stride of the E buffer (odd)
  int ras;      // stride of the r * a(0) buffer
  int sstride;  // stride of the split-row table
  int wstride;  // stride of the per-wave scan tails
  int tb_all;   // 1: the tables of every mode stay resident (rebuilt once per minibatch)
  // Two-level core update (large P * W): workgroup w reduces float4 columns
  // [w * cper, (w + 1) * cper) of the partials in cgrp thread groups of cvg
  // partials each (LDS region red, cgrp * cper float4), stores that slice of G,
  // and after one more grid barrier every workgroup reads the whole new G.
  int core2, red, cper, cgrp, cvg;
  int aux_len;  // ints of the host-built index maps (row-offset maps, then table gather maps)
  int hm_len;   // ints of the row-offset maps (the first part of aux)
  // Row buffers (two, alternating between sub-steps) are chunk-major: mode
  // k's values [c*V, c*V + V) (a 16-byte chunk, V = 4 FP32 or 8 BF16 values)
  // of sample p sit at float word ((coff[k] + c) * chp + p) * 4.
  int coff[kMaxOrder];
  int ctot;     // chunks per sample over all modes
  int rowsz;    // floats of one row buffer
  // Kruskal core (R > 0): kb = the matrices B(k) (J_k x R row-major, B(k) at
  // kb + kboff[k]); kwt = the chunk's rows of [W_0 .. W_{R-1} | x] for the
  // current mode (chp rows of stride kws: entry c J_n + a, then x at R J_n);
  // kg = the packed upper triangle of their Gram matrix (ke = R Jmax + 1
  // columns at most).  kwt and kg overlay the hp / E / r a(0) regions, which
  // the Kruskal core sub-step does not use.
  int kb, kwt, kg, kws, ke;
  int kboff[kMaxOrder];
  int klg;      // floats of the packed triangle for ke columns: ke (ke + 1) / 2
  // Heavy-ball momentum: vg = the core velocity this workgroup updates (all P
  // entries with the one-level core update, every workgroup holding the same
  // copy; its slice of cper float4 with the two-level update).
  int vg;
};

// Per-phase constants of the chain, built on the host.  Phase 0 is the core
// sub-step, phase ph >= 1 the sub-step of mode ph - 1.
struct PhaseTab {
  int n;         // mode whose unfolding the phase contracts with (0 for the core phase)
  int upd;       // mode the phase updates (-1: core phase)
  int pm;        // mode the previous phase updated (-1: none): its straddling rows are finished now
  int post;      // bit mask of modes whose rows are read after the barrier (updated by the two previous phases)
  int khi, nhi;  // product and count of the modes other than n and lo
  int jlo, kp, nt;
  int ls_n, ls_lo, Jn;
  int c_lo, c_n, c_hi;  // chunk offsets (ChainLayout::coff) of modes lo, n and the first remaining mode
  int c_hi2;     // chunk offset of the second remaining mode (0 if none)
  int tb_off;    // element offset of mode n's table in the table region
  int tb_len;    // elements of mode n's table
  int hm_off;    // int offset of mode n's row-offset map
  int tm_off;    // int offset of mode n's table gather map (resident tables only)
  // FP32 contraction (32x32 tiles, K = j_lo in steps of 2): ks2 K steps,
  // hpt multi-indices h per 32-column tile (columns j_n + J_n * (h mod hpt)),
  // ctn column tiles, ens partial-E slots per sample in the E buffer
  int ks2, hpt, ctn, ens;
};

// Schedule words per (minibatch, mode) in the chunk-boundary array:
// [0, W) straddling row or -1, [W, 2W) entry number of a straddling row's
// first boundary or -1, [2W] number of straddling rows.
__host__ __device__ inline int xrow_stride(int W) { return 2 * W + 4; }

// Per-position metadata of every phase ([N+1][T] words; phase 0 is the core
// sub-step in minibatch order, phase n+1 the (row, position) order of mode n).
// Factor phases: bits 0-8 the chunk-local position where the row's run
// starts in the chunk, bit 9 last position of the run in the chunk, bit 10
// run began in an earlier chunk, bit 11 run goes on in the next chunk.
// All phases: bits 16-23 hold 1 + the entry of the previous phase's table of
// straddling rows that holds this position's row of the mode that phase
// updated (0: none).
constexpr int kMetaTail = 1 << 9, kMetaBefore = 1 << 10, kMetaAfter = 1 << 11;
constexpr int kMetaPatchShift = 16;

// Location of a non-finite parameter written by the chain, ordered as the
// chain writes them: minibatch b (saturated at 2^29 - 1), phase ph (0: the
// core, whose "row" is the flat core index; ph >= 1: a row of mode ph - 1),
// row.  The smallest key over a run is the first non-finite value.
__host__ __device__ inline unsigned long long nf_key(int64_t b, int ph, int64_t row) {
  const unsigned long long bb = b < ((1ll << 29) - 1) ? (unsigned long long)b : ((1ull << 29) - 1);
  return ((bb * 16ull + (unsigned long long)ph) << 31) | (unsigned long long)(row & 0x7FFFFFFF);
}

// Arguments of the persistent minibatch chain kernel.
struct ChainArgs {
  Shape s;
  const uint32_t* coo;      // records in epoch order (T x R words)
  const uint16_t* sigma;    // [N][T] per-minibatch sorted positions
  const uint32_t* rec_sorted; // [N][T] records in (row, position) order per minibatch
  const int* xrow;          // [nb][N][xrow_stride(W)] chunk-boundary rows and their numbering
  const uint32_t* meta;     // [N+1][T] per-position metadata of every phase
  const int* aux;           // host-built maps (lay.aux_len ints)
  float* A[kMaxOrder];      // FP32 master factors, I_n x Jp_n
  uint16_t* Ab[kMaxOrder];  // BF16 read copies (null in FP32 mode), I_n x Jb_n
  int Jb[kMaxOrder];        // row stride of the BF16 copies (J_n rounded up to 8)
  int bf16;                 // 1: BF16 operands, FP32 masters and accumulation
  float* G;                 // FP32 master core (P)
  int mom;                  // 1: heavy-ball momentum (velocities VA, VG, factor mu)
  float mu;
  float* VA[kMaxOrder];     // row velocities, laid out as A (momentum)
  float* VG;                // core velocity (P, momentum)
  int R;                    // Kruskal rank of the core (0: dense core)
  float* B;                 // Kruskal core: FP32 masters of B(k), J_k x R each, back to back (R > 0)
  float* partial;           // [W][pad4(P)] per-workgroup core-gradient partials; Kruskal core:
                            // [2][W][pad4(klg)] Gram partials then [2][pad4(klg)] their sums
  float* carry;             // [2][W * carry_stride] per parity: the straddling runs' partials, old rows
                            // (and old velocities) of every chunk (layout at finish_split_rows)
  unsigned* bar;            // grid-barrier arrival flags, one per workgroup, kFlagStride apart (zero at launch)
  int* err;                 // set to nonzero by a workgroup that gives up
  unsigned long long* nf;   // earliest non-finite write: nf_key(b, phase, row), all ones if none
  int64_t T, M;
  int64_t b_begin, b_end;   // minibatches [b_begin, b_end) of the epoch
  float gA, lA, gG, lG;     // learning steps and L2 weights
  int W;                    // workgroups in the chain
  int chunk;                // samples per workgroup per phase (<= blockDim)
  int carry_stride;         // floats of carry per chunk: >= 4 + 3 J_max (4 + 4 J_max with momentum), x4
  long long spin_limit;     // barrier give-up bound (iterations)
  unsigned passed0;         // barriers the flags in bar have counted before this chain starts
  int jv;                   // rank variant of the chain body (chain_variant of s)
  int split_cap;            // entries of the LDS split-row table
  int lds_cap;              // LDS bytes a workgroup may use on the device (the plan keeps every
                            // mode's table resident when all of it fits; 0: 160 KiB)
  ChainLayout lay;          // filled by plan_chain_lds
  PhaseTab pt[kMaxOrder + 1];
  // (placement last, so that the fields above keep their kernel-argument offsets)
  int xs;                   // blocks per workgroup in the grid (W * xs blocks): 1 when spread, the
                            // device's XCC count when on one XCC
  int xid;                  // >= 0: the chain runs on the W blocks the dispatcher deals to XCC xid
                            // (see chain_workgroup), and its grid barrier orders memory in that
                            // XCC's L2; -1: blocks 0..W-1 spread over the XCCs, agent-scope barriers
};

// Which J specialisation of the chain serves a shape: the common rank when
// every mode has the same J_n in {2, 3, 4, 5, 6, 8, 10, 12, 16, 20}, else 0
// (generic, J_n <= 32).
int chain_variant(const Shape& s);

// Kernel launchers (stdecomp_kernels.hip).  All return hipError_t values.
hipError_t launch_perm_gather(const Shape& s, const uint32_t* coo, uint32_t* coo_perm, int64_t T,
                              uint64_t seed, int64_t epoch, hipStream_t st);
hipError_t launch_perm_only(int64_t T, uint64_t seed, int64_t epoch, int64_t* out, hipStream_t st);
hipError_t launch_sort(const Shape& s, const uint32_t* coo_perm, uint16_t* sigma, int* xrow, int* nseg,
                       uint32_t* rec_sorted, uint32_t* meta, int W, int chunk, int64_t T, int64_t M,
                       int64_t b_begin, int64_t b_end, hipStream_t st);
hipError_t launch_debug_segments(const Shape& s, const uint32_t* coo_perm, const uint16_t* sigma,
                                 int64_t T, int64_t M, int64_t b, int mode, int32_t* seg_off,
                                 int32_t* seg_row, int32_t* nseg, hipStream_t st);
// Fills a.lay and a.pt and the index maps (aux, a.lay.aux_len ints); returns
// the LDS bytes of one workgroup, or 0 if the request is inconsistent.
size_t plan_chain_lds(ChainArgs& a, int threads, bool bf16, int* aux = nullptr);
hipError_t launch_chain(const ChainArgs& a, int threads, hipStream_t st);
hipError_t launch_barrier_probe(const ChainArgs& a, int threads, int reps, hipStream_t st);
// The barrier reps times with a data exchange around each (slots: W
// kFlagStride words; stale: one counter, zero at launch).
hipError_t launch_barrier_check(const ChainArgs& a, int threads, int reps, unsigned* slots, unsigned long long* stale,
                                hipStream_t st);
// XCC of every block of a grid of `blocks` blocks (out[b], blocks ints).
hipError_t launch_xcc_probe(int* out, int blocks, hipStream_t st);
// Many independent chains in one cooperative launch: slot q (workgroups
// [q W, (q + 1) W)) runs the chains list[nslots + 1 + i], i in [list[q],
// list[q + 1]), one after another, each from its own arguments dev_args[m]
// (own buffers and minibatch range; bar = the slot's flags, passed0 = the
// barriers the slot counted before it).  Every chain has W workgroups, the
// same order class (three modes or other), the dense core and the same
// dtype; ranks may differ (each chain runs the body it runs alone).  bytes = the
// largest LDS plan among them.  mom: every chain has heavy-ball momentum (the
// kernels of stdecomp_chain_mom.hip), else none has.
hipError_t launch_chain_queue(int n3, int bf, int mom, const ChainArgs* dev_args, const int* dev_list, int nslots,
                              int W, int threads, size_t bytes, hipStream_t st);
// The chain kernels with heavy-ball momentum (stdecomp_chain_mom.hip): one
// chain (a.mom, dense core, plan already checked) and a batch of chains.
hipError_t launch_chain_mom(const ChainArgs& a, int threads, size_t bytes, hipStream_t st);
// The dense-core chain kernels without momentum with the one-XCC barrier
// (stdecomp_chain_xcc.hip; a.xid >= 0, plan already checked).
hipError_t launch_chain_xcc(const ChainArgs& a, int threads, size_t bytes, hipStream_t st);
hipError_t launch_chain_queue_mom(int n3, int bf, const ChainArgs* dev_args, const int* dev_list, int nslots, int W,
                                  int threads, size_t bytes, hipStream_t st);
hipError_t launch_pack_records(const Shape& s, const int32_t* idx, const float* vals, int64_t n,
                               uint32_t* rec, int* bad, hipStream_t st);
struct FactorPtrs {
  const float* A[kMaxOrder];
};
hipError_t launch_predict(const Shape& s, const uint32_t* rec, int64_t n, FactorPtrs A, const float* G, float* out,
                          int nblocks, hipStream_t st);
hipError_t launch_loss(const Shape& s, const uint32_t* rec, int64_t n, FactorPtrs A, const float* G,
                       double* block_out, int nblocks, double* out3, hipStream_t st);
hipError_t launch_sumsq(const float* p, int64_t n, double* block_out, int nblocks, hipStream_t st);
hipError_t launch_count_nonfinite(const float* p, int64_t n, int* flag, hipStream_t st);
hipError_t launch_fill_i32(int* p, int v, int64_t n, hipStream_t st);
hipError_t launch_to_bf16(const float* src, uint16_t* dst, int64_t n, hipStream_t st);
// rows x cols FP32 (row stride sstride) -> BF16 (row stride dstride), round to nearest even
hipError_t launch_rows_to_bf16(const float* src, int sstride, uint16_t* dst, int dstride, int64_t rows, int cols,
                               hipStream_t st);

}  // namespace stdk
