// Host runtime of libstdecomp: argument validation, device memory, the epoch
// driver (sampler -> row-set sort -> minibatch chain) and the C ABI declared
// in include/stdecomp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/stdecomp.h"
#include "stdecomp_internal.h"

using stdk::kMaxOrder;
using stdk::kMaxRank;

struct stdecomp_handle {
  stdk::Shape s{};
  int64_t T = 0, M = 0, nb = 0;
  float gA = 0, lA = 0, gG = 0, lG = 0;
  uint64_t seed_sample = 0;
  int dtype = 0;
  int64_t epoch = 0;
  int64_t cursor = 0;  // next minibatch of epoch `epoch` for stdecomp_step_batched (0: at an epoch start)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t qstream = nullptr;  // predictions (may run while another thread trains the handle)
  int device = 0;
  int num_cus = 0;
  int lds_cap = 0;  // LDS bytes per workgroup on the device (the chain plan's bound)
  int xs = 1, xid = -1;  // chain placement (ChainArgs::xs / xid): one XCC when xid >= 0
  // chain configuration
  int W = 1, chunk = 1, threads = 64, split_cap = 0, carry_stride = 0;
  size_t chain_lds = 0;
  stdk::ChainLayout lay{};
  stdk::PhaseTab pt[kMaxOrder + 1] = {};
  std::vector<int> aux_host;  // index maps of the chain (uploaded to aux)
  // device buffers
  uint32_t* coo = nullptr;
  uint32_t* coo_perm = nullptr;
  uint16_t* sigma = nullptr;
  uint32_t* rec_sorted = nullptr;
  int* xrow = nullptr;
  int* nseg = nullptr;
  uint32_t* meta = nullptr;
  int* aux = nullptr;
  float* A[kMaxOrder] = {};
  uint16_t* Ab[kMaxOrder] = {};  // BF16 read copies (BF16 mode)
  int Jb[kMaxOrder] = {};
  float* G = nullptr;
  float mu = 0;                  // heavy-ball momentum (0: none, no velocity buffers)
  float* VA[kMaxOrder] = {};     // row velocities, laid out as A
  float* VG = nullptr;           // core velocity (P)
  int R = 0;             // Kruskal rank of the core (0: dense core)
  float* B = nullptr;    // Kruskal core: B(n), J_n x R each, back to back
  int64_t nB = 0;        // floats of B
  float* partial = nullptr;
  float* carry = nullptr;
  unsigned* bar = nullptr;
  int* err = nullptr;
  unsigned long long* nf = nullptr;  // first non-finite write of the chain (stdk::nf_key), all ones if none
  double* dscratch = nullptr;  // loss/sum-of-squares block partials
  int dscratch_blocks = 0;
  int* flag = nullptr;
  int* qflag = nullptr;  // bad-index flag of the prediction calls
  size_t device_bytes = 0;
  int64_t sched_epoch = -1;  // epoch whose schedule coo_perm/sigma hold
  std::string last_error;
  std::mutex err_mu;  // last_error may be set by a prediction beside a training call
  hipEvent_t ev[4] = {};
  stdecomp_alloc_fn dev_alloc = nullptr;  // caller's device allocator (NULL: hipMalloc)
  stdecomp_free_fn dev_free = nullptr;
  void* alloc_ctx = nullptr;
  bool train_rmse = false;  // epoch stats carry the training RMSE
};

// Scratch memory of stdecomp_predict_noalloc: a file-scope device array (one
// copy on every device the library runs on, held until the process ends).
// Host code never uses its name as an address: stdecomp_init resolves the
// device address once per device (hipGetSymbolAddress with that device
// current) and the entry point passes that address to the kernels and copies.
static constexpr size_t kNoAllocScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace stdk {
// One chain with momentum on one XCC (stdecomp_chain_mom_xcc.hip).
hipError_t launch_chain_mom_xcc(const ChainArgs& a, int threads, hipStream_t st);
// Batched chains with every slot on one XCC (stdecomp_chain_queue_xcc.hip).
hipError_t launch_chain_queue_xcc(int n3, int bf, const ChainArgs* dev_args, const int* dev_list, int nslots, int W,
                                  int nx, int threads, size_t bytes, hipStream_t st);
}  // namespace stdk

namespace {

int fail(stdecomp_handle* h, int code, const std::string& msg) {
  if (h) {
    std::lock_guard<std::mutex> lock(h->err_mu);
    h->last_error = msg;
  }
  return code;
}

int hip_fail(stdecomp_handle* h, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(h, STD_E_DEVICE, m);
}

#define HIPCHK(h, call)                                  \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail((h), e_, #call); \
  } while (0)

// Device workspace of stdecomp_epoch_batched (argument table and workgroup
// map), one per device, kept for the life of the process.
struct BatchWorkspace {
  struct Dev {
    void* ptr = nullptr;
    size_t bytes = 0;
  };
  std::mutex mu;
  Dev dev[64];
};
BatchWorkspace g_batch_ws;

// Why the calling thread's last stdecomp_init failed (stdecomp_last_error(NULL)).
thread_local std::string g_init_error;

// Per-device address of the scratch array (filled by resolve_scratch).
struct ScratchTable {
  std::mutex mu;
  void* ptr[64] = {};
};
ScratchTable g_scratch;

// Resolve the scratch array's address on the current device (once per device).
const char* const kMisplaced =
    "the dispatch did not deal the chain's blocks to the XCCs in turn, as the one-XCC placement needs "
    "(create the handle with placement STD_PLACE_SPREAD)";

// Placement of the chain (STD_PLACE_*).  One XCC needs W <= CUs per XCC and a
// dispatch that deals the blocks to the X XCCs in turn (block b and block
// b + X on the same XCC), which is checked here on a grid of W X blocks; the
// chain then runs on the W blocks of a grid of W X that land on the XCC block 0
// of this probe ran on (chain_workgroup).  A device with one XCC keeps blocks
// 0..W-1 with the L2-ordered barrier.
int choose_placement(stdecomp_handle* h, int req) {
  h->xs = 1;
  h->xid = -1;
  if (req == STD_PLACE_SPREAD) return STD_OK;
  if (h->R > 0) {  // (one-XCC kernels exist for the dense core, with and without momentum)
    if (req == STD_PLACE_ONE_XCC)
      return fail(h, STD_E_INVAL, "placement STD_PLACE_ONE_XCC: not available with the Kruskal core");
    return STD_OK;
  }
  int nx = 1;
  if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, h->device) != hipSuccess || nx < 1) nx = 1;
  const bool fits = h->num_cus % nx == 0 && h->W <= h->num_cus / nx;
  int xid = -1;
  if (fits) {
    const int blocks = h->W * nx;
    std::vector<int> ids((size_t)blocks, -1);
    int* dids = reinterpret_cast<int*>(h->dscratch);  // (3 * 4096 doubles; blocks <= CUs)
    if (stdk::launch_xcc_probe(dids, blocks, h->stream) != hipSuccess ||
        hipMemcpyAsync(ids.data(), dids, (size_t)blocks * 4, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
      return fail(h, STD_E_DEVICE, "XCC placement probe failed");
    bool rr = true;
    for (int b = 0; b < blocks; ++b) rr = rr && ids[(size_t)b] == ids[(size_t)(b % nx)];
    for (int x = 0; x < nx; ++x)
      for (int y = 0; y < x; ++y) rr = rr && ids[(size_t)x] != ids[(size_t)y];
    if (rr) xid = ids[0];
  }
  if (xid < 0) {
    if (req == STD_PLACE_ONE_XCC)
      return fail(h, STD_E_INVAL,
                  fits ? "placement STD_PLACE_ONE_XCC: the dispatch does not place blocks round-robin over the XCCs"
                       : "placement STD_PLACE_ONE_XCC: the chain has more workgroups than one XCC has compute units");
    return STD_OK;
  }
  h->xs = nx;
  h->xid = xid;
  return STD_OK;
}

int resolve_scratch(stdecomp_handle* h) {
  std::lock_guard<std::mutex> lock(g_scratch.mu);
  if (h->device < 0 || h->device >= 64) return fail(h, STD_E_DEVICE, "device ordinal out of range");
  if (g_scratch.ptr[h->device]) return STD_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(h, STD_E_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
  }
  g_scratch.ptr[h->device] = p;
  return STD_OK;
}

int64_t noalloc_max_queries(const stdecomp_handle* h, int32_t on_device) {
  // largest q with pad256(q R 4) + [pad256(q N 4) + q 4] <= the scratch size
  const int64_t per = (int64_t)h->s.R * 4 + (on_device ? 0 : (int64_t)h->s.N * 4 + 4);
  int64_t q = (int64_t)kNoAllocScratchBytes / per;
  while (q > 0) {
    const size_t need = (((size_t)q * h->s.R * 4 + 255) & ~(size_t)255) +
                        (on_device ? 0 : (((size_t)q * h->s.N * 4 + 255) & ~(size_t)255) + (size_t)q * 4);
    if (need <= kNoAllocScratchBytes) break;
    --q;
  }
  return q;
}

constexpr int kBatchesPerLaunch = 2048;  // bounds the duration of one chain launch
constexpr long long kSpinLimit = 1ll << 24;


// Device memory of a handle: from the caller's allocator when the options
// give one (stdecomp_options.dev_alloc / dev_free), else hipMalloc / hipFree.
// account: count the buffer in device_bytes (buffers held by the handle; the
// temporary buffers of a call are not counted).  st: the stream the buffer is
// used on (the handle's stream by default).
template <typename T>
int dalloc(stdecomp_handle* h, T** p, size_t count, bool account = true, hipStream_t st = nullptr) {
  *p = nullptr;
  if (count == 0) count = 1;
  const size_t bytes = count * sizeof(T);
  if (h->dev_alloc) {
    void* q = h->dev_alloc(h->alloc_ctx, bytes, (void*)(st ? st : h->stream));
    if (!q) return fail(h, STD_E_NOMEM, "the caller's allocator returned NULL for " + std::to_string(bytes) + " bytes");
    *p = static_cast<T*>(q);
  } else {
    hipError_t e = hipMalloc((void**)p, bytes);
    if (e != hipSuccess) {
      *p = nullptr;
      (void)hipGetLastError();
      return fail(h, STD_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
  }
  if (account) h->device_bytes += bytes;
  return STD_OK;
}

template <typename T>
void dfree(stdecomp_handle* h, T*& p, hipStream_t st = nullptr) {
  if (p) {
    if (h->dev_free) h->dev_free(h->alloc_ctx, (void*)p, (void*)(st ? st : h->stream));
    else (void)hipFree((void*)p);
  }
  p = nullptr;
}

// Host initialiser: SplitMix64 stream, Box-Muller normals.
struct HostRng {
  uint64_t state;
  explicit HostRng(uint64_t seed) : state(seed) {}
  uint64_t next() {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u1 = uniform(), u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

int64_t total_minibatches(int64_t T, int64_t M) { return (T + M - 1) / M; }

// Four waves per chain workgroup (one per SIMD) whatever the chunk: the MFMA
// tiles and table builds use all of them, the per-sample steps the first
// `chunk` lanes.  (Eight waves hide more latency in the contraction but cost
// more at every workgroup barrier; measured slower overall.)
int chain_threads_for(int /*chunk*/) { return stdk::kChainThreads; }

// Pick the chain geometry and check that it fits one workgroup's LDS.
int configure_chain(stdecomp_handle* h, int chunk_req) {
  const stdk::Shape& s = h->s;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, h->device) != hipSuccess)
    return fail(h, STD_E_DEVICE, "hipGetDeviceProperties failed");
  const size_t lds_cap = prop.maxSharedMemoryPerMultiProcessor ? prop.maxSharedMemoryPerMultiProcessor
                                                                : prop.sharedMemPerBlock;
  int chunk = chunk_req;
  if (chunk <= 0) {
    // about 32 workgroups for large minibatches, at least 64 entries each;
    // for large cores more, smaller chunks (at most 2^18 core-sized
    // contractions per workgroup and sub-step for three modes, 2^19 for more:
    // the two-stage contraction of those kernels gains from longer chunks)
    chunk = (int)((h->M + 31) / 32);
    if (chunk < 64) chunk = 64;
    chunk = ((chunk + 63) / 64) * 64;
    const int64_t lim = s.N == 3 ? (1 << 18) : (1 << 19);
    while (chunk > 64 && (int64_t)chunk * s.P > lim && (h->M + chunk / 2 - 1) / (chunk / 2) <= h->num_cus)
      chunk /= 2;
  }
  if (chunk > stdk::kChainThreads) chunk = stdk::kChainThreads;
  if (chunk > h->M) chunk = (int)h->M;
  for (;;) {
    int W = (int)((h->M + chunk - 1) / chunk);
    if (W > h->num_cus) return fail(h, STD_E_INVAL, "minibatch needs more chain workgroups than compute units");
    h->chunk = chunk;
    h->W = W;
    h->threads = chain_threads_for(chunk);
    h->split_cap = W > 1 ? W - 1 : 0;
    int jmax = 0;
    for (int n = 0; n < s.N; ++n) jmax = s.J[n] > jmax ? s.J[n] : jmax;
    // carry of a chunk: two slots (row, count, partial sum), the old row (and old velocity)
    h->carry_stride = stdk::pad4(4 + (h->mu > 0 ? 4 : 3) * jmax);
    stdk::ChainArgs a{};
    a.s = s;
    a.R = h->R;
    a.mom = h->mu > 0 ? 1 : 0;
    a.W = W;
    a.chunk = chunk;
    a.split_cap = h->split_cap;
    a.carry_stride = h->carry_stride;
    a.lds_cap = (int)lds_cap;
    h->lds_cap = (int)lds_cap;
    h->chain_lds = stdk::plan_chain_lds(a, h->threads, h->dtype == STD_DTYPE_BF16);
    if (h->chain_lds == 0) return fail(h, STD_E_INVAL, "inconsistent chain plan");
    // With the default chunk, halve it (more, smaller workgroups) until the
    // row buffers of one workgroup fit its LDS.
    if (h->chain_lds > lds_cap && chunk_req <= 0 && chunk > 64 &&
        (h->M + chunk / 2 - 1) / (chunk / 2) <= h->num_cus) {
      chunk /= 2;
      continue;
    }
    if (h->chain_lds > lds_cap)
      return fail(h, STD_E_INVAL, "core or factor rows too large for one workgroup's LDS (" +
                                      std::to_string(h->chain_lds) + " > " + std::to_string(lds_cap) + " bytes)");
    h->aux_host.assign((size_t)(a.lay.aux_len > 0 ? a.lay.aux_len : 1), 0);
    if (stdk::plan_chain_lds(a, h->threads, h->dtype == STD_DTYPE_BF16, h->aux_host.data()) != h->chain_lds)
      return fail(h, STD_E_INVAL, "inconsistent chain plan");
    h->lay = a.lay;
    for (int i = 0; i <= kMaxOrder; ++i) h->pt[i] = a.pt[i];
    break;
  }
  return STD_OK;
}

stdk::ChainArgs chain_args(stdecomp_handle* h) {
  stdk::ChainArgs a{};
  a.s = h->s;
  a.coo = h->coo_perm;
  a.sigma = h->sigma;
  a.rec_sorted = h->rec_sorted;
  a.xrow = h->xrow;
  a.meta = h->meta;
  a.aux = h->aux;
  for (int n = 0; n < h->s.N; ++n) {
    a.A[n] = h->A[n];
    a.Ab[n] = h->Ab[n];
    a.Jb[n] = h->Jb[n];
  }
  a.bf16 = h->dtype == STD_DTYPE_BF16 ? 1 : 0;
  a.lay = h->lay;
  for (int i = 0; i <= kMaxOrder; ++i) a.pt[i] = h->pt[i];
  a.G = h->G;
  a.mom = h->mu > 0 ? 1 : 0;
  a.mu = h->mu;
  for (int n = 0; n < h->s.N; ++n) a.VA[n] = h->VA[n];
  a.VG = h->VG;
  a.R = h->R;
  a.B = h->B;
  a.partial = h->partial;
  a.carry = h->carry;
  a.bar = h->bar;
  a.err = h->err;
  a.nf = h->nf;
  a.T = h->T;
  a.M = h->M;
  a.gA = h->gA;
  a.lA = h->lA;
  a.gG = h->gG;
  a.lG = h->lG;
  a.W = h->W;
  a.xs = h->xs;
  a.xid = h->xid;
  a.chunk = h->chunk;
  a.carry_stride = h->carry_stride;
  a.lds_cap = h->lds_cap;
  a.spin_limit = kSpinLimit;
  a.split_cap = h->split_cap;
  return a;
}

int run_schedule(stdecomp_handle* h, int64_t epoch) {
  HIPCHK(h, stdk::launch_perm_gather(h->s, h->coo, h->coo_perm, h->T, h->seed_sample, epoch, h->stream));
  HIPCHK(h, stdk::launch_sort(h->s, h->coo_perm, h->sigma, h->xrow, h->nseg, h->rec_sorted, h->meta, h->W, h->chunk, h->T,
                              h->M, 0, h->nb, h->stream));
  h->sched_epoch = epoch;
  return STD_OK;
}

// Pack caller COO (host or device SoA) into device records on stream st
// (bad-index flag `flag`).  *rec_out is freshly allocated (caller frees it on
// st).  Index range violations -> STD_E_INVAL.
int pack_caller_entries(stdecomp_handle* h, int64_t n, const int32_t* idx, const float* vals, int on_device,
                        uint32_t** rec_out, hipStream_t st, int* flag) {
  *rec_out = nullptr;
  const int N = h->s.N;
  const int32_t* didx = idx;
  const float* dvals = vals;
  int32_t* tidx = nullptr;
  float* tvals = nullptr;
  if (!on_device) {
    for (int k = 0; k < N; ++k)
      for (int64_t t = 0; t < n; ++t) {
        const int32_t v = idx[(int64_t)k * n + t];
        if (v < 0 || v >= h->s.I[k]) return fail(h, STD_E_INVAL, "index out of range");
      }
    int rc = dalloc(h, &tidx, (size_t)N * n, false, st);
    if (rc) return rc;
    HIPCHK(h, hipMemcpyAsync(tidx, idx, (size_t)N * n * 4, hipMemcpyHostToDevice, st));
    if (vals) {
      rc = dalloc(h, &tvals, (size_t)n, false, st);
      if (rc) {
        dfree(h, tidx, st);
        return rc;
      }
      HIPCHK(h, hipMemcpyAsync(tvals, vals, (size_t)n * 4, hipMemcpyHostToDevice, st));
    }
    didx = tidx;
    dvals = tvals;
  }
  uint32_t* rec = nullptr;
  int rc = dalloc(h, &rec, (size_t)n * h->s.R, false, st);
  if (rc) {
    dfree(h, tidx, st);
    dfree(h, tvals, st);
    return rc;
  }
  hipError_t e = stdk::launch_fill_i32(flag, 0, 1, st);
  if (e == hipSuccess) e = stdk::launch_pack_records(h->s, didx, dvals, n, rec, flag, st);
  int bad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dfree(h, tidx, st);
  dfree(h, tvals, st);
  if (e != hipSuccess) {
    dfree(h, rec, st);
    return hip_fail(h, e, "packing entries");
  }
  if (bad) {
    dfree(h, rec, st);
    return fail(h, STD_E_INVAL, "index out of range");
  }
  *rec_out = rec;
  return STD_OK;
}

stdk::FactorPtrs factor_ptrs(const stdecomp_handle* h) {
  stdk::FactorPtrs f{};
  for (int n = 0; n < h->s.N; ++n) f.A[n] = h->A[n];
  return f;
}

int eval_blocks(const stdecomp_handle* h, int64_t n) {
  int64_t b = (n + 255) / 256;
  const int64_t cap = (int64_t)h->num_cus * 4;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (int)b;
}

int device_sumsq(stdecomp_handle* h, const float* p, int64_t n, double* out) {
  const int nb = 256;
  HIPCHK(h, stdk::launch_sumsq(p, n, h->dscratch, nb, h->stream));
  std::vector<double> v(nb);
  HIPCHK(h, hipMemcpyAsync(v.data(), h->dscratch, nb * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  double acc = 0.0;
  for (int i = 0; i < nb; ++i) acc += v[i];
  *out = acc;
  return STD_OK;
}

// BF16 read copies from the FP32 masters (BF16 mode only).
int refresh_bf16(stdecomp_handle* h) {
  if (h->dtype != STD_DTYPE_BF16) return STD_OK;
  for (int n = 0; n < h->s.N; ++n)
    HIPCHK(h, stdk::launch_rows_to_bf16(h->A[n], h->s.Jp[n], h->Ab[n], h->Jb[n], h->s.I[n], h->s.J[n], h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return STD_OK;
}

// Floats of the chain's partial buffer: per-workgroup core-gradient partials
// (dense core) or, for the Kruskal core, two sets of per-workgroup Gram
// partials and two summed Gram matrices (packed triangles).
size_t partial_floats(const stdecomp_handle* h) {
  size_t n = (size_t)h->W * stdk::pad4(h->s.P);
  if (h->R > 0) {
    const size_t klgp = (size_t)stdk::pad4(h->lay.klg);
    const size_t k = 2 * (size_t)h->W * klgp + 2 * klgp;
    n = k > n ? k : n;
  }
  return n;
}

// G = sum_r prod_k B(k)[j_k, r] on the host (Eq. CP-Decomposition; G flat with
// j_1 fastest, B(k) J_k x R row-major, back to back).
void kruskal_product_host(const stdk::Shape& s, int R, const float* B, std::vector<float>& G) {
  G.assign((size_t)s.P, 0.f);
  std::vector<int64_t> off(s.N, 0);
  for (int k = 1; k < s.N; ++k) off[k] = off[k - 1] + (int64_t)s.J[k - 1] * R;
  for (int lin = 0; lin < s.P; ++lin) {
    double acc = 0.0;
    for (int r = 0; r < R; ++r) {
      double t = 1.0;
      for (int k = 0; k < s.N; ++k) t *= B[off[k] + (int64_t)((lin / s.lstride[k]) % s.J[k]) * R + r];
      acc += t;
    }
    G[lin] = (float)acc;
  }
}

void release(stdecomp_handle* h) {
  if (!h) return;
  dfree(h, h->coo);
  dfree(h, h->coo_perm);
  dfree(h, h->sigma);
  dfree(h, h->rec_sorted);
  dfree(h, h->xrow);
  dfree(h, h->nseg);
  dfree(h, h->meta);
  dfree(h, h->aux);
  for (int n = 0; n < kMaxOrder; ++n) {
    dfree(h, h->A[n]);
    dfree(h, h->Ab[n]);
    dfree(h, h->VA[n]);
  }
  dfree(h, h->G);
  dfree(h, h->VG);
  dfree(h, h->B);
  dfree(h, h->partial);
  dfree(h, h->carry);
  dfree(h, h->bar);
  dfree(h, h->err);
  dfree(h, h->nf);
  dfree(h, h->dscratch);
  dfree(h, h->flag);
  dfree(h, h->qflag);
  for (auto& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  if (h->qstream) (void)hipStreamDestroy(h->qstream);
}

bool finite_nonneg(float x) { return std::isfinite(x) && x >= 0.f; }

}  // namespace

extern "C" {

int stdecomp_default_options(stdecomp_options* o) {
  if (!o) return STD_E_INVAL;
  std::memset(o, 0, sizeof(*o));
  o->batch = 256;
  o->lr_factor = o->lr_core = 0.01f;
  o->lambda_factor = o->lambda_core = 0.01f;
  o->init_kind = STD_INIT_SCALED;
  o->dtype = STD_DTYPE_F32;
  return STD_OK;
}

const char* stdecomp_strerror(int code) {
  switch (code) {
    case STD_OK: return "ok";
    case STD_E_INVAL: return "invalid argument";
    case STD_E_NOMEM: return "out of memory";
    case STD_E_DEVICE: return "device error";
    case STD_E_STATE: return "invalid handle state";
    case STD_E_DIVERGED: return "diverged (non-finite values)";
    default: return "unknown error";
  }
}

const char* stdecomp_last_error(const stdecomp_handle* h) {
  if (h) return h->last_error.c_str();
  return g_init_error.empty() ? "no handle" : g_init_error.c_str();
}

int stdecomp_init(const stdecomp_problem* p, const stdecomp_options* o, stdecomp_handle** out) {
  if (!out) return STD_E_INVAL;
  *out = nullptr;
  if (!p || !o) return STD_E_INVAL;
  const int N = p->order;
  if (N < 2 || N > kMaxOrder || !p->dims || !p->ranks || p->nnz < 1 || !p->idx || !p->vals) return STD_E_INVAL;
  if (o->batch < 1 || o->batch > stdk::kMaxBatch) return STD_E_INVAL;
  if (!finite_nonneg(o->lr_factor) || !finite_nonneg(o->lr_core) || !finite_nonneg(o->lambda_factor) ||
      !finite_nonneg(o->lambda_core))
    return STD_E_INVAL;
  if (o->init_kind < STD_INIT_SCALED || o->init_kind > STD_INIT_CALLER) return STD_E_INVAL;
  if (o->dtype != STD_DTYPE_F32 && o->dtype != STD_DTYPE_BF16) return STD_E_INVAL;
  if (o->r_core < 0 || o->r_core > 64) return STD_E_INVAL;
  for (int i = 0; i < 9; ++i)
    if (o->reserved[i] != 0) return STD_E_INVAL;
  if (o->placement < STD_PLACE_AUTO || o->placement > STD_PLACE_ONE_XCC) return STD_E_INVAL;
  if (!(o->momentum >= 0.f && o->momentum < 1.f)) return STD_E_INVAL;
  if (o->momentum > 0.f && o->r_core > 0) return STD_E_INVAL;
  if ((o->dev_alloc == nullptr) != (o->dev_free == nullptr)) return STD_E_INVAL;
  if (o->report_train_rmse != 0 && o->report_train_rmse != 1) return STD_E_INVAL;
  int64_t P = 1;
  for (int n = 0; n < N; ++n) {
    if (p->dims[n] < 1 || p->dims[n] >= (1ll << 31) || p->ranks[n] < 1 || p->ranks[n] > kMaxRank)
      return STD_E_INVAL;
    P *= p->ranks[n];
    if (P > (1 << 20)) return STD_E_INVAL;
  }
  if (p->nnz >= (1ll << 40)) return STD_E_INVAL;

  stdecomp_handle* h = new (std::nothrow) stdecomp_handle();
  if (!h) return STD_E_NOMEM;
  h->dev_alloc = o->dev_alloc;
  h->dev_free = o->dev_free;
  h->alloc_ctx = o->alloc_ctx;
  h->train_rmse = o->report_train_rmse != 0;
  auto bail = [&](int rc) {
    std::fprintf(stderr, "stdecomp_init: %s\n", h->last_error.c_str());
    g_init_error = h->last_error;
    release(h);
    delete h;
    return rc;
  };
  if (hipGetDevice(&h->device) != hipSuccess) {
    h->last_error = "no HIP device";
    return bail(STD_E_DEVICE);
  }
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) != hipSuccess) {
      h->last_error = "hipGetDeviceProperties failed";
      return bail(STD_E_DEVICE);
    }
    h->num_cus = prop.multiProcessorCount;
  }
  stdk::Shape& s = h->s;
  s.N = N;
  s.P = (int)P;
  s.R = N + 1;
  int off = 0;
  for (int n = 0; n < N; ++n) {
    s.J[n] = p->ranks[n];
    s.Jp[n] = stdk::pad4(p->ranks[n]);
    s.I[n] = p->dims[n];
    s.rs_off[n] = off;
    off += s.J[n];
  }
  s.rs = off | 1;
  {
    int acc = 1;
    for (int n = 0; n < N; ++n) {
      s.lstride[n] = acc;
      acc *= s.J[n];
    }
  }
  h->T = p->nnz;
  h->M = o->batch;
  h->nb = total_minibatches(h->T, h->M);
  h->gA = o->lr_factor;
  h->lA = o->lambda_factor;
  h->gG = o->lr_core;
  h->lG = o->lambda_core;
  h->seed_sample = o->seed_sample;
  h->dtype = o->dtype;
  h->R = o->r_core;
  h->mu = o->momentum;
  h->nB = 0;
  for (int n = 0; n < N; ++n) h->nB += (int64_t)s.J[n] * h->R;
  if (o->stream) {
    h->stream = (hipStream_t)o->stream;
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      h->last_error = "hipStreamCreate failed";
      return bail(STD_E_DEVICE);
    }
    h->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&h->qstream, hipStreamNonBlocking) != hipSuccess) {
    h->qstream = nullptr;
    h->last_error = "hipStreamCreate failed";
    return bail(STD_E_DEVICE);
  }
  for (auto& e : h->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      h->last_error = "hipEventCreate failed";
      return bail(STD_E_DEVICE);
    }
  int rc = configure_chain(h, o->chain_chunk);
  if (rc) return bail(rc);
  if ((rc = resolve_scratch(h))) return bail(rc);

  // device memory
  const size_t T = (size_t)h->T;
  if ((rc = dalloc(h, &h->coo, T * s.R)) || (rc = dalloc(h, &h->coo_perm, T * s.R)) ||
      (rc = dalloc(h, &h->sigma, T * N)) || (rc = dalloc(h, &h->rec_sorted, T * N * s.R)) ||
      (rc = dalloc(h, &h->xrow, (size_t)h->nb * N * stdk::xrow_stride(h->W))) ||
      (rc = dalloc(h, &h->meta, T * (N + 1))) || (rc = dalloc(h, &h->aux, h->aux_host.size())) ||
      (rc = dalloc(h, &h->nseg, (size_t)h->nb * N)) || (rc = dalloc(h, &h->G, (size_t)P)) ||
      (rc = dalloc(h, &h->partial, partial_floats(h))) || (h->R > 0 && (rc = dalloc(h, &h->B, (size_t)h->nB))) ||
      (rc = dalloc(h, &h->carry, (size_t)2 * h->W * h->carry_stride)) ||
      (rc = dalloc(h, &h->bar, (size_t)h->W * stdk::kFlagStride)) ||
      (rc = dalloc(h, &h->err, 1)) || (rc = dalloc(h, &h->nf, 1)) || (rc = dalloc(h, &h->dscratch, 3 * 4096)) ||
      (rc = dalloc(h, &h->flag, 1)) || (rc = dalloc(h, &h->qflag, 1)) ||
      (h->mu > 0 && (rc = dalloc(h, &h->VG, (size_t)P))))
    return bail(rc);
  if ((rc = choose_placement(h, o->placement))) return bail(rc);
  if (h->mu > 0 && hipMemsetAsync(h->VG, 0, (size_t)P * 4, h->stream) != hipSuccess) {
    h->last_error = "hipMemset failed";
    return bail(STD_E_DEVICE);
  }
  for (int n = 0; n < N; ++n) {
    h->Jb[n] = (s.J[n] + 7) & ~7;
    if (h->dtype == STD_DTYPE_BF16 && (rc = dalloc(h, &h->Ab[n], (size_t)s.I[n] * h->Jb[n]))) return bail(rc);
    if ((rc = dalloc(h, &h->A[n], (size_t)s.I[n] * s.Jp[n]))) return bail(rc);
    if (hipMemsetAsync(h->A[n], 0, (size_t)s.I[n] * s.Jp[n] * 4, h->stream) != hipSuccess) {
      h->last_error = "hipMemset failed";
      return bail(STD_E_DEVICE);
    }
    if (h->mu > 0) {
      if ((rc = dalloc(h, &h->VA[n], (size_t)s.I[n] * s.Jp[n]))) return bail(rc);
      if (hipMemsetAsync(h->VA[n], 0, (size_t)s.I[n] * s.Jp[n] * 4, h->stream) != hipSuccess) {
        h->last_error = "hipMemset failed";
        return bail(STD_E_DEVICE);
      }
    }
  }
  if (hipMemsetAsync(h->xrow, 0xFF, (size_t)h->nb * N * stdk::xrow_stride(h->W) * 4, h->stream) != hipSuccess ||
      hipMemcpyAsync(h->aux, h->aux_host.data(), h->aux_host.size() * 4, hipMemcpyHostToDevice, h->stream) !=
          hipSuccess) {
    h->last_error = "hipMemset failed";
    return bail(STD_E_DEVICE);
  }

  // COO entries -> device records (the range check runs on the device)
  {
    int32_t* didx = nullptr;
    float* dvals = nullptr;
    const int32_t* src_idx = p->idx;
    const float* src_vals = p->vals;
    if (!o->inputs_on_device) {
      if ((rc = dalloc(h, &didx, T * N)) || (rc = dalloc(h, &dvals, T))) {
        dfree(h, didx);
        return bail(rc);
      }
      h->device_bytes -= T * N * 4 + T * 4;
      if (hipMemcpyAsync(didx, p->idx, T * N * 4, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
          hipMemcpyAsync(dvals, p->vals, T * 4, hipMemcpyHostToDevice, h->stream) != hipSuccess) {
        dfree(h, didx);
        dfree(h, dvals);
        h->last_error = "copying the COO entries failed";
        return bail(STD_E_DEVICE);
      }
      src_idx = didx;
      src_vals = dvals;
    }
    int bad = 0;
    hipError_t e = hipMemsetAsync(h->flag, 0, sizeof(int), h->stream);
    if (e == hipSuccess) e = stdk::launch_pack_records(s, src_idx, src_vals, h->T, h->coo, h->flag, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    dfree(h, didx);
    dfree(h, dvals);
    if (e != hipSuccess) {
      h->last_error = std::string("packing the COO entries: ") + hipGetErrorString(e);
      return bail(STD_E_DEVICE);
    }
    if (bad) {
      h->last_error = "COO index out of range";
      return bail(STD_E_INVAL);
    }
  }

  // initial parameters
  {
    HostRng rng(o->seed_init);
    std::vector<float> buf;
    for (int n = 0; n < N; ++n) {
      buf.assign((size_t)s.I[n] * s.Jp[n], 0.f);
      if (o->init_kind != STD_INIT_CALLER) {
        const double sd = o->init_kind == STD_INIT_PAPER ? 0.1 : 1.0 / std::sqrt((double)s.J[n]);
        const double mu = o->init_kind == STD_INIT_PAPER ? 0.5 : 0.0;
        for (int64_t i = 0; i < s.I[n]; ++i)
          for (int j = 0; j < s.J[n]; ++j) buf[(size_t)i * s.Jp[n] + j] = (float)(mu + sd * rng.normal());
      }
      if (hipMemcpy(h->A[n], buf.data(), buf.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
        h->last_error = "copying initial factors failed";
        return bail(STD_E_DEVICE);
      }
    }
    buf.assign((size_t)P, 0.f);
    if (h->R > 0) {
      // Kruskal core: B(k) entries N(0, sd^2) with R sd^(2N) = 1/J_1, so that G
      // = Kruskal(B) has the entry variance of the dense initialisation (or
      // the paper's N(0.5, 0.1^2)); G is their product
      std::vector<float> bb((size_t)h->nB, 0.f);
      if (o->init_kind != STD_INIT_CALLER) {
        const double sd = o->init_kind == STD_INIT_PAPER ? 0.1 : std::pow(1.0 / ((double)h->R * s.J[0]), 0.5 / N);
        const double mu = o->init_kind == STD_INIT_PAPER ? 0.5 : 0.0;
        for (auto& v : bb) v = (float)(mu + sd * rng.normal());
      }
      kruskal_product_host(s, h->R, bb.data(), buf);
      if (hipMemcpy(h->B, bb.data(), bb.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
        h->last_error = "copying the initial Kruskal factors failed";
        return bail(STD_E_DEVICE);
      }
    } else if (o->init_kind != STD_INIT_CALLER) {
      const double sd = o->init_kind == STD_INIT_PAPER ? 0.1 : 1.0 / std::sqrt((double)s.J[0]);
      const double mu = o->init_kind == STD_INIT_PAPER ? 0.5 : 0.0;
      for (int64_t i = 0; i < P; ++i) buf[i] = (float)(mu + sd * rng.normal());
    }
    if (hipMemcpy(h->G, buf.data(), buf.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      h->last_error = "copying the initial core failed";
      return bail(STD_E_DEVICE);
    }
  }
  if (hipMemsetAsync(h->partial, 0, partial_floats(h) * 4, h->stream) != hipSuccess ||
      refresh_bf16(h) != STD_OK) {
    h->last_error = "initialising device buffers failed";
    return bail(STD_E_DEVICE);
  }
  *out = h;
  return STD_OK;
}

}  // extern "C"

namespace {

// Algorithmic flops per nonzero-update.  Dense core: (2N + 4) prod(J) (the
// core step's contraction and gradient, and each mode's contraction).  Kruskal
// core: each mode's contraction, 2N prod(J), plus per mode n the row of
// [W | x] (R sum_{k != n} J_k dot-product terms and R J_n products) and its
// packed Gram matrix ((R J_n + 1)(R J_n + 2) / 2 multiply-adds).
double flops_per_update(const stdecomp_handle* h) {
  const stdk::Shape& s = h->s;
  if (h->R <= 0) return (2.0 * s.N + 4.0) * s.P;
  double f = 2.0 * s.N * s.P, sumJ = 0.0;
  for (int n = 0; n < s.N; ++n) sumJ += s.J[n];
  for (int n = 0; n < s.N; ++n) {
    const double e = (double)h->R * s.J[n] + 1.0;
    f += 2.0 * h->R * (sumJ - s.J[n]) + (double)h->R * s.J[n] + e * (e + 1.0);
  }
  return f;
}

// STD_E_DIVERGED naming the first non-finite parameter the chain wrote
// (stdk::nf_key of the record; all ones means none was recorded).
int diverged_at(stdecomp_handle* h, int64_t epoch, unsigned long long key) {
  const int64_t row = (int64_t)(key & 0x7FFFFFFFull);
  const unsigned long long bp = key >> 31;
  const int64_t b = (int64_t)(bp / 16);
  const int ph = (int)(bp % 16);
  std::string where = ph == 0 ? "core sub-step, core entry " + std::to_string(row)
                              : "mode-" + std::to_string(ph - 1) + " sub-step, row " + std::to_string(row);
  return fail(h, STD_E_DIVERGED, "non-finite parameters: first at epoch " + std::to_string(epoch) + ", minibatch " +
                                     std::to_string(b) + (b == (1ll << 29) - 1 ? " or later" : "") + ", " + where);
}

// Work of minibatches [b0, b1) into *acc: minibatches, nonzero-updates,
// algorithmic bytes (COO records; each touched row read and written once per
// minibatch and mode, 8 bytes per value in FP32, 12 in BF16 with its FP32
// master; the core, or the Kruskal factors, read and written once per
// minibatch) and algorithmic flops.  nseg_host: the distinct rows of every
// (minibatch, mode) of the epoch, as counted by the row-set sort.
void add_work(const stdecomp_handle* h, int64_t b0, int64_t b1, const std::vector<int>& nseg_host,
              stdecomp_epoch_stats* acc) {
  const int N = h->s.N;
  const double beta = h->dtype == STD_DTYPE_BF16 ? 12.0 : 8.0;
  double rows_bytes = 0.0;
  int64_t upd = 0;
  for (int64_t b = b0; b < b1; ++b) {
    const int64_t m = (h->T - b * h->M < h->M) ? h->T - b * h->M : h->M;
    upd += m;
    for (int n = 0; n < N; ++n) rows_bytes += (double)nseg_host[(size_t)b * N + n] * h->s.J[n] * beta;
  }
  acc->minibatches += b1 - b0;
  acc->updates += upd;
  const double core_words = h->R > 0 ? (double)h->nB : (double)h->s.P;
  acc->bytes_alg += (double)upd * (4.0 * N + 4.0) + rows_bytes + (double)(b1 - b0) * 2.0 * core_words * 4.0;
  acc->flops_alg += (double)upd * flops_per_update(h);
}

// Minibatches [b0, b1) of epoch `epoch`, accumulated into *acc.
int run_range(stdecomp_handle* h, int64_t epoch, int64_t b0, int64_t b1, stdecomp_epoch_stats* acc,
              std::vector<int>& nseg_host) {
  const int N = h->s.N;
  HIPCHK(h, hipEventRecord(h->ev[0], h->stream));
  if (h->sched_epoch != epoch) {
    int rc = run_schedule(h, epoch);
    if (rc) return rc;
  }
  HIPCHK(h, hipEventRecord(h->ev[1], h->stream));
  HIPCHK(h, hipMemsetAsync(h->err, 0, sizeof(int), h->stream));
  HIPCHK(h, hipMemsetAsync(h->nf, 0xFF, sizeof(unsigned long long), h->stream));
  stdk::ChainArgs a = chain_args(h);
  for (int64_t c0 = b0; c0 < b1; c0 += kBatchesPerLaunch) {
    a.b_begin = c0;
    a.b_end = (c0 + kBatchesPerLaunch < b1) ? c0 + kBatchesPerLaunch : b1;
    HIPCHK(h, hipMemsetAsync(h->bar, 0, (size_t)h->W * stdk::kFlagStride * sizeof(unsigned), h->stream));
    HIPCHK(h, (a.mom && a.xid >= 0) ? stdk::launch_chain_mom_xcc(a, h->threads, h->stream)
                                     : stdk::launch_chain(a, h->threads, h->stream));
    acc->chain_launches++;
  }
  HIPCHK(h, hipEventRecord(h->ev[2], h->stream));
  int err = 0;
  unsigned long long nf = ~0ull;
  HIPCHK(h, hipMemcpyAsync(&err, h->err, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(&nf, h->nf, sizeof(nf), hipMemcpyDeviceToHost, h->stream));
  nseg_host.resize((size_t)h->nb * N);
  HIPCHK(h, hipMemcpyAsync(nseg_host.data(), h->nseg, nseg_host.size() * 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (err == 2) return fail(h, STD_E_DEVICE, kMisplaced);
  if (err) return fail(h, STD_E_DEVICE, "chain workgroup gave up waiting at a grid barrier");
  if (nf != ~0ull) return diverged_at(h, epoch, nf);
  float t01 = 0, t12 = 0;
  HIPCHK(h, hipEventElapsedTime(&t01, h->ev[0], h->ev[1]));
  HIPCHK(h, hipEventElapsedTime(&t12, h->ev[1], h->ev[2]));
  acc->schedule_seconds += t01 * 1e-3;
  acc->chain_seconds += t12 * 1e-3;
  acc->device_seconds += (t01 + t12) * 1e-3;
  add_work(h, b0, b1, nseg_host, acc);
  return STD_OK;
}

int check_finite(stdecomp_handle* h) {
  HIPCHK(h, hipMemsetAsync(h->flag, 0, sizeof(int), h->stream));
  HIPCHK(h, stdk::launch_count_nonfinite(h->G, h->s.P, h->flag, h->stream));
  for (int n = 0; n < h->s.N; ++n)
    HIPCHK(h, stdk::launch_count_nonfinite(h->A[n], h->s.I[n] * h->s.Jp[n], h->flag, h->stream));
  int bad = 0;
  HIPCHK(h, hipMemcpyAsync(&bad, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (bad) return fail(h, STD_E_DIVERGED, "non-finite parameters");
  return STD_OK;
}

}  // namespace

extern "C" {

int stdecomp_epoch(stdecomp_handle* h, int32_t n_epochs, stdecomp_epoch_stats* st) {
  if (!h) return STD_E_STATE;
  if (n_epochs < 0) return fail(h, STD_E_INVAL, "n_epochs < 0");
  if (h->cursor != 0) return fail(h, STD_E_STATE, "the model is inside an epoch (stdecomp_step_batched)");
  stdecomp_epoch_stats acc{};
  acc.train_rmse = std::nan("");
  std::vector<int> nseg_host;
  for (int e = 0; e < n_epochs; ++e) {
    int rc = run_range(h, h->epoch, 0, h->nb, &acc, nseg_host);
    if (rc) return rc;
    acc.epochs_run++;
    h->epoch++;
  }
  int rc = check_finite(h);
  if (rc == STD_OK && h->train_rmse) {
    stdecomp_loss_out lo{};
    rc = stdecomp_loss(h, 0, nullptr, nullptr, 0, &lo);
    acc.train_rmse = lo.rmse;
  }
  if (st) *st = acc;
  return rc;
}

}  // extern "C"

namespace {

// Whether the handles can share one batched launch: distinct handles on one
// device with the same dtype, workgroup count, threads and order class
// (three modes or other), all with the dense core; ranks may differ.
bool batch_compatible(stdecomp_handle* const* hs, int n, size_t* lds) {
  const stdecomp_handle* h0 = hs[0];
  bool ok = h0->R == 0 && h0->W <= h0->num_cus;
  *lds = 0;
  for (int i = 0; i < n && ok; ++i) {
    const stdecomp_handle* h = hs[i];
    ok = h->device == h0->device && h->dtype == h0->dtype && h->threads == h0->threads && h->R == 0 &&
         h->W == h0->W && (h->s.N == 3) == (h0->s.N == 3) && (h->mu > 0) == (h0->mu > 0);
    for (int k = 0; k < i && ok; ++k) ok = hs[k] != h;
    *lds = h->chain_lds > *lds ? h->chain_lds : *lds;
  }
  return ok;
}

// Minibatches [b0[i], b1[i]) of each handle's current epoch, every chain in
// one cooperative launch per window of kBatchesPerLaunch minibatches: slots of
// W workgroups, as many as the device holds at once and the batch needs; the
// chains go to slots longest first, each to the slot with the least work so
// far (work ~ minibatches x sub-steps x (1 + prod(J) / 512), a cost model of
// the chain's latency-bound minibatch), and a slot runs its chains one after
// another.  acc[i] receives the work and the launches' time (the whole
// batched launch for every model).  Errors are reported on hs[0].
int run_batched_ranges(stdecomp_handle* const* hs, int n, size_t lds, const std::vector<int64_t>& b0,
                       const std::vector<int64_t>& b1, std::vector<stdecomp_epoch_stats>& acc) {
  stdecomp_handle* h0 = hs[0];
  const int W = h0->W;
  if (hipSetDevice(h0->device) != hipSuccess) return fail(h0, STD_E_DEVICE, "hipSetDevice failed");
  int nslots = std::min(n, h0->num_cus / W);
  // every slot on one XCC when every handle is placed on one (dense core, no
  // momentum in a batch, W <= CUs per XCC): nslots a multiple of the XCC count nx, the
  // slots of one XCC filling at most its CUs
  const int nx = h0->xs;
  bool local = true;
  for (int i = 0; i < n && local; ++i) local = hs[i]->xid >= 0 && hs[i]->xs == nx && hs[i]->mu == 0;
  if (local) {
    const int cap = h0->num_cus / W;
    int up = (nslots + nx - 1) / nx * nx;
    if (up > cap) up = cap / nx * nx;
    if (up < nx)
      local = false;
    else
      nslots = up;
  }
  std::vector<int> order((size_t)n);
  std::vector<double> cost((size_t)n);
  int64_t max_len = 0;
  for (int i = 0; i < n; ++i) {
    order[i] = i;
    cost[i] = (double)(b1[i] - b0[i]) * (hs[i]->s.N + 1) * (1.0 + hs[i]->s.P / 512.0);
    max_len = std::max(max_len, b1[i] - b0[i]);
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  std::vector<std::vector<int>> slot_models((size_t)nslots);
  std::vector<double> load((size_t)nslots, 0.0);
  for (int i : order) {
    int q = 0;
    for (int k = 1; k < nslots; ++k)
      if (load[k] < load[q]) q = k;
    slot_models[q].push_back(i);
    load[q] += cost[i];
  }
  std::vector<int> list((size_t)nslots + 1 + n);
  {
    int o = 0;
    for (int q = 0; q < nslots; ++q) {
      list[q] = o;
      for (int i : slot_models[q]) list[(size_t)nslots + 1 + o++] = i;
    }
    list[nslots] = o;
  }
  // the launch's argument table, slot lists and barrier flags live in a
  // per-device workspace that grows on demand and is kept, so a call
  // allocates only when it needs more than any call before it on that device
  std::lock_guard<std::mutex> lock(g_batch_ws.mu);
  BatchWorkspace::Dev& ws = g_batch_ws.dev[h0->device];
  auto pad256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t args_bytes = pad256(sizeof(stdk::ChainArgs) * n);
  const size_t list_bytes = pad256(sizeof(int) * list.size());
  const size_t flag_bytes = (size_t)nslots * W * stdk::kFlagStride * sizeof(unsigned);
  const size_t need = args_bytes + list_bytes + flag_bytes;
  if (ws.bytes < need) {
    if (ws.ptr) (void)hipFree(ws.ptr);
    ws.ptr = nullptr;
    ws.bytes = 0;
    if (hipMalloc(&ws.ptr, need) != hipSuccess) {
      (void)hipGetLastError();
      ws.ptr = nullptr;
      return fail(h0, STD_E_NOMEM, "batched launch: device workspace allocation failed");
    }
    ws.bytes = need;
  }
  stdk::ChainArgs* dargs = static_cast<stdk::ChainArgs*>(ws.ptr);
  int* dlist = reinterpret_cast<int*>(static_cast<char*>(ws.ptr) + args_bytes);
  unsigned* dflags = reinterpret_cast<unsigned*>(static_cast<char*>(ws.ptr) + args_bytes + list_bytes);
  std::vector<stdk::ChainArgs> args((size_t)n);
  std::vector<int> nseg_host;
  int rc = STD_OK;
  auto hipck = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && rc == STD_OK) rc = fail(h0, STD_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return e == hipSuccess;
  };
  for (int i = 0; i < n && rc == STD_OK; ++i) {
    stdecomp_handle* h = hs[i];
    if (h->sched_epoch != h->epoch) rc = run_schedule(h, h->epoch);
    if (rc == STD_OK) hipck(hipStreamSynchronize(h->stream), "schedule");
  }
  if (rc != STD_OK) return rc;
  hipck(hipMemcpyAsync(dlist, list.data(), sizeof(int) * list.size(), hipMemcpyHostToDevice, h0->stream),
        "batched launch lists");
  for (int i = 0; i < n; ++i) {
    hipck(hipMemsetAsync(hs[i]->err, 0, sizeof(int), h0->stream), "memset");
    hipck(hipMemsetAsync(hs[i]->nf, 0xFF, sizeof(unsigned long long), h0->stream), "memset");
  }
  hipck(hipEventRecord(h0->ev[1], h0->stream), "event");
  int64_t launches = 0;
  for (int64_t off = 0; off < max_len && rc == STD_OK; off += kBatchesPerLaunch) {
    for (int q = 0; q < nslots; ++q) {
      unsigned passed = 0;  // barriers the slot's flags count before each of its chains
      for (int i : slot_models[q]) {
        stdecomp_handle* h = hs[i];
        stdk::ChainArgs& a = args[i];
        a = chain_args(h);
        a.xs = 1;  // (the slot mapping is the queue kernel's)
        a.xid = local ? 0 : -1;
        a.b_begin = std::min(b0[i] + off, b1[i]);
        a.b_end = std::min(b0[i] + off + kBatchesPerLaunch, b1[i]);
        a.bar = dflags + (size_t)q * W * stdk::kFlagStride;
        a.passed0 = passed;
        a.jv = stdk::chain_variant(h->s);
        passed += (unsigned)((a.b_end - a.b_begin) * (h->s.N + 1 + (h->lay.core2 ? 1 : 0)));
      }
    }
    hipck(hipMemsetAsync(dflags, 0, flag_bytes, h0->stream), "memset");
    hipck(hipMemcpyAsync(dargs, args.data(), sizeof(stdk::ChainArgs) * n, hipMemcpyHostToDevice, h0->stream),
          "batched launch arguments");
    hipck(local ? stdk::launch_chain_queue_xcc(h0->s.N == 3, h0->dtype == STD_DTYPE_BF16, dargs, dlist, nslots, W, nx,
                                               h0->threads, lds, h0->stream)
                : stdk::launch_chain_queue(h0->s.N == 3, h0->dtype == STD_DTYPE_BF16, h0->mu > 0, dargs, dlist, nslots, W,
                                           h0->threads, lds, h0->stream),
          "batched chain launch");
    hipck(hipStreamSynchronize(h0->stream), "batched chain launch");  // (args reused next)
    ++launches;
  }
  hipck(hipEventRecord(h0->ev[2], h0->stream), "event");
  hipck(hipStreamSynchronize(h0->stream), "event");
  float ms = 0.f;
  hipck(hipEventElapsedTime(&ms, h0->ev[1], h0->ev[2]), "event");
  for (int i = 0; i < n && rc == STD_OK; ++i) {
    stdecomp_handle* h = hs[i];
    int err = 0;
    unsigned long long nf = ~0ull;
    nseg_host.resize((size_t)h->nb * h->s.N);
    const size_t N = (size_t)h->s.N;
    hipck(hipMemcpyAsync(&err, h->err, sizeof(int), hipMemcpyDeviceToHost, h0->stream), "error flag");
    hipck(hipMemcpyAsync(&nf, h->nf, sizeof(nf), hipMemcpyDeviceToHost, h0->stream), "non-finite record");
    if (b1[i] > b0[i])  // (the segment counts of the minibatches run)
      hipck(hipMemcpyAsync(nseg_host.data() + b0[i] * N, h->nseg + b0[i] * N, (size_t)(b1[i] - b0[i]) * N * 4,
                           hipMemcpyDeviceToHost, h0->stream),
            "segment counts");
    hipck(hipStreamSynchronize(h0->stream), "error flag");
    if (err == 2 && rc == STD_OK) rc = fail(h0, STD_E_DEVICE, kMisplaced);
    if (err && rc == STD_OK) rc = fail(h0, STD_E_DEVICE, "chain workgroup gave up waiting at a grid barrier");
    if (nf != ~0ull && rc == STD_OK) {
      diverged_at(h, h->epoch, nf);
      rc = fail(h0, STD_E_DIVERGED, "model " + std::to_string(i) + ": " + h->last_error);
    }
    acc[i].chain_seconds += ms * 1e-3;  // (the whole batched launch)
    acc[i].device_seconds += ms * 1e-3;
    acc[i].chain_launches += launches;
    add_work(h, b0[i], b1[i], nseg_host, &acc[i]);
  }
  return rc;
}

}  // namespace

extern "C" {

int stdecomp_epoch_batched(stdecomp_handle* const* hs, int32_t n, int32_t n_epochs, stdecomp_epoch_stats* st) {
  if (!hs || n < 1) return STD_E_INVAL;
  for (int i = 0; i < n; ++i)
    if (!hs[i]) return STD_E_STATE;
  stdecomp_handle* h0 = hs[0];
  if (n_epochs < 0) return fail(h0, STD_E_INVAL, "n_epochs < 0");
  for (int i = 0; i < n; ++i)
    if (hs[i]->cursor != 0)
      return fail(h0, STD_E_STATE, "model " + std::to_string(i) + " is inside an epoch (stdecomp_step_batched)");
  size_t lds = 0;
  if (!batch_compatible(hs, n, &lds)) {  // the same updates, one handle after another
    for (int i = 0; i < n; ++i) {
      int rc = stdecomp_epoch(hs[i], n_epochs, st ? &st[i] : nullptr);
      if (rc) return rc;
    }
    return STD_OK;
  }
  std::vector<stdecomp_epoch_stats> acc((size_t)n);
  for (auto& x : acc) x.train_rmse = std::nan("");
  std::vector<int64_t> b0((size_t)n, 0), b1((size_t)n);
  for (int i = 0; i < n; ++i) b1[i] = hs[i]->nb;
  for (int e = 0; e < n_epochs; ++e) {
    int rc = run_batched_ranges(hs, n, lds, b0, b1, acc);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) {
      acc[i].epochs_run++;
      hs[i]->epoch++;
    }
  }
  for (int i = 0; i < n; ++i) {
    if (st) st[i] = acc[i];
    int r2 = check_finite(hs[i]);
    if (r2) return r2;
  }
  return STD_OK;
}

int stdecomp_step_batched(stdecomp_handle* const* hs, int32_t n, int64_t max_minibatches, stdecomp_epoch_stats* st) {
  if (!hs || n < 1) return STD_E_INVAL;
  for (int i = 0; i < n; ++i)
    if (!hs[i]) return STD_E_STATE;
  stdecomp_handle* h0 = hs[0];
  if (max_minibatches < 1) return fail(h0, STD_E_INVAL, "max_minibatches < 1");
  std::vector<stdecomp_epoch_stats> acc((size_t)n);
  for (auto& x : acc) x.train_rmse = std::nan("");
  std::vector<int64_t> b0((size_t)n), b1((size_t)n);
  for (int i = 0; i < n; ++i) {
    b0[i] = hs[i]->cursor;
    b1[i] = std::min(hs[i]->nb, b0[i] + max_minibatches);
  }
  size_t lds = 0;
  if (batch_compatible(hs, n, &lds)) {
    int rc = run_batched_ranges(hs, n, lds, b0, b1, acc);
    if (rc) return rc;
  } else {  // the same updates, one handle after another
    std::vector<int> nseg_host;
    for (int i = 0; i < n; ++i) {
      int rc = run_range(hs[i], hs[i]->epoch, b0[i], b1[i], &acc[i], nseg_host);
      if (rc) return rc;
    }
  }
  for (int i = 0; i < n; ++i) {
    stdecomp_handle* h = hs[i];
    h->cursor = b1[i];
    if (h->cursor == h->nb) {
      h->cursor = 0;
      h->epoch++;
      acc[i].epochs_run++;
    }
  }
  for (int i = 0; i < n; ++i) {
    if (st) st[i] = acc[i];
    int r2 = check_finite(hs[i]);
    if (r2) return r2;
  }
  return STD_OK;
}

int stdecomp_run_minibatches(stdecomp_handle* h, int64_t epoch, int64_t b_begin, int64_t b_end,
                             stdecomp_epoch_stats* st) {
  if (!h) return STD_E_STATE;
  if (epoch < 0 || b_begin < 0 || b_end < b_begin || b_end > h->nb) return fail(h, STD_E_INVAL, "bad minibatch range");
  stdecomp_epoch_stats acc{};
  std::vector<int> nseg_host;
  if (b_end > b_begin) {
    int rc = run_range(h, epoch, b_begin, b_end, &acc, nseg_host);
    if (rc) return rc;
  }
  if (st) *st = acc;
  return check_finite(h);
}

int stdecomp_predict(stdecomp_handle* h, int64_t q, const int32_t* idx, float* out, int32_t on_device) {
  if (!h) return STD_E_STATE;
  if (q < 0 || (q > 0 && (!idx || !out))) return fail(h, STD_E_INVAL, "bad predict arguments");
  if (q == 0) return STD_OK;
  uint32_t* rec = nullptr;
  // (on the handle's query stream, with its own flag: this may run while
  // another thread trains the handle on its main stream)
  const hipStream_t qs = h->qstream;
  int rc = pack_caller_entries(h, q, idx, nullptr, on_device, &rec, qs, h->qflag);
  if (rc) return rc;
  float* dout = out;
  if (!on_device) {
    if ((rc = dalloc(h, &dout, (size_t)q, false, qs))) {
      dfree(h, rec, qs);
      return rc;
    }
  }
  hipError_t e = stdk::launch_predict(h->s, rec, q, factor_ptrs(h), h->G, dout, eval_blocks(h, q), qs);
  if (e == hipSuccess && !on_device) e = hipMemcpyAsync(out, dout, (size_t)q * 4, hipMemcpyDeviceToHost, qs);
  if (e == hipSuccess) e = hipStreamSynchronize(qs);
  dfree(h, rec, qs);
  if (!on_device) dfree(h, dout, qs);
  if (e != hipSuccess) return hip_fail(h, e, "predict");
  return STD_OK;
}

int stdecomp_predict_noalloc(stdecomp_handle* h, int64_t q, const int32_t* idx, float* out, int32_t on_device) {
  if (!h) return STD_E_STATE;
  if (q < 0 || (q > 0 && (!idx || !out))) return fail(h, STD_E_INVAL, "bad predict arguments");
  if (q == 0) return STD_OK;
  const int N = h->s.N;
  const size_t rec_bytes = ((size_t)q * h->s.R * 4 + 255) & ~(size_t)255;
  const size_t idx_bytes = on_device ? 0 : (((size_t)q * N * 4 + 255) & ~(size_t)255);
  const size_t out_bytes = on_device ? 0 : (size_t)q * 4;
  if (rec_bytes + idx_bytes + out_bytes > kNoAllocScratchBytes)
    return fail(h, STD_E_INVAL, "stdecomp_predict_noalloc: " + std::to_string(q) + " queries need " +
                                    std::to_string(rec_bytes + idx_bytes + out_bytes) + " bytes of scratch, more than " +
                                    std::to_string(kNoAllocScratchBytes) + " (at most " +
                                    std::to_string(noalloc_max_queries(h, on_device)) + " queries)");
  void* base = g_scratch.ptr[h->device];
  if (!base) return fail(h, STD_E_STATE, "scratch address not resolved for this device");
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, STD_E_DEVICE, "hipSetDevice failed");
  uint32_t* rec = static_cast<uint32_t*>(base);
  const int32_t* didx = idx;
  float* dout = out;
  if (!on_device) {
    // host indices are range-checked here, as stdecomp_predict does, then staged in scratch
    for (int k = 0; k < N; ++k)
      for (int64_t t = 0; t < q; ++t) {
        const int32_t v = idx[(int64_t)k * q + t];
        if (v < 0 || v >= h->s.I[k]) return fail(h, STD_E_INVAL, "index out of range");
      }
    int32_t* sidx = reinterpret_cast<int32_t*>(static_cast<unsigned char*>(base) + rec_bytes);
    HIPCHK(h, hipMemcpyAsync(sidx, idx, (size_t)q * N * 4, hipMemcpyHostToDevice, h->qstream));
    didx = sidx;
    dout = reinterpret_cast<float*>(static_cast<unsigned char*>(base) + rec_bytes + idx_bytes);
  }
  int bad = 0;
  hipError_t e = stdk::launch_fill_i32(h->qflag, 0, 1, h->qstream);
  if (e == hipSuccess) e = stdk::launch_pack_records(h->s, didx, nullptr, q, rec, h->qflag, h->qstream);
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, h->qflag, sizeof(int), hipMemcpyDeviceToHost, h->qstream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->qstream);
  if (e != hipSuccess) return hip_fail(h, e, "predict_noalloc: packing entries");
  if (bad) return fail(h, STD_E_INVAL, "index out of range");
  e = stdk::launch_predict(h->s, rec, q, factor_ptrs(h), h->G, dout, eval_blocks(h, q), h->qstream);
  if (e == hipSuccess && !on_device) e = hipMemcpyAsync(out, dout, (size_t)q * 4, hipMemcpyDeviceToHost, h->qstream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->qstream);
  if (e != hipSuccess) return hip_fail(h, e, "predict_noalloc");
  return STD_OK;
}

int stdecomp_loss(stdecomp_handle* h, int64_t n, const int32_t* idx, const float* vals, int32_t on_device,
                  stdecomp_loss_out* out) {
  if (!h) return STD_E_STATE;
  if (!out) return fail(h, STD_E_INVAL, "out is NULL");
  uint32_t* rec = nullptr;
  const uint32_t* use = nullptr;
  if (!idx && !vals) {
    n = h->T;
    use = h->coo;
  } else {
    if (n < 1 || !idx || !vals) return fail(h, STD_E_INVAL, "bad loss arguments");
    int rc = pack_caller_entries(h, n, idx, vals, on_device, &rec, h->stream, h->flag);
    if (rc) return rc;
    use = rec;
  }
  const int nb = eval_blocks(h, n);
  double sums[3] = {0, 0, 0};
  hipError_t e = stdk::launch_loss(h->s, use, n, factor_ptrs(h), h->G, h->dscratch, nb, h->dscratch + 3 * nb,
                                   h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(sums, h->dscratch + 3 * nb, sizeof(sums), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  dfree(h, rec);
  if (e != hipSuccess) return hip_fail(h, e, "loss");
  double regA = 0.0, regG = 0.0, t = 0.0;
  for (int k = 0; k < h->s.N; ++k) {
    int rc = device_sumsq(h, h->A[k], h->s.I[k] * h->s.Jp[k], &t);
    if (rc) return rc;
    regA += t;
  }
  int rc = device_sumsq(h, h->G, h->s.P, &regG);
  if (rc) return rc;
  out->count = n;
  out->sse = sums[0];
  out->rmse = std::sqrt(sums[0] / (double)n);
  out->mae = sums[1] / (double)n;
  out->nonfinite = (int64_t)sums[2];
  out->objective = 0.5 * sums[0] / (double)n + 0.5 * h->lA * regA + 0.5 * h->lG * regG;
  if (out->nonfinite > 0 || !std::isfinite(out->sse)) return fail(h, STD_E_DIVERGED, "non-finite loss");
  return STD_OK;
}

namespace {

// Copy factor-shaped device arrays (padded rows, dA[n] I_n x Jp_n) and a
// core-shaped one out to host arrays of I_n x J_n rows and P floats: one
// contiguous copy per factor (a pitched copy from pageable memory goes row by
// row), unpacked on the host.
int copy_params_out(stdecomp_handle* h, float* const* dA, const float* dG, float* const* A, float* G) {
  if (!A || !G) return fail(h, STD_E_INVAL, "NULL parameter pointer");
  std::vector<float> buf;
  for (int n = 0; n < h->s.N; ++n) {
    if (!A[n]) return fail(h, STD_E_INVAL, "NULL factor pointer");
    const int J = h->s.J[n], Jp = h->s.Jp[n];
    const size_t rows = (size_t)h->s.I[n];
    if (J == Jp) {
      HIPCHK(h, hipMemcpyAsync(A[n], dA[n], rows * J * 4, hipMemcpyDeviceToHost, h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
    } else {
      buf.resize(rows * Jp);
      HIPCHK(h, hipMemcpyAsync(buf.data(), dA[n], buf.size() * 4, hipMemcpyDeviceToHost, h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      for (size_t i = 0; i < rows; ++i) std::memcpy(A[n] + i * J, buf.data() + i * Jp, (size_t)J * 4);
    }
  }
  HIPCHK(h, hipMemcpyAsync(G, dG, (size_t)h->s.P * 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return STD_OK;
}

// The reverse: packed on the host into the padded row layout (padding stays
// zero) and sent in one contiguous copy per factor.
int copy_params_in(stdecomp_handle* h, float* const* dA, float* dG, const float* const* A, const float* G) {
  if (!A || !G) return fail(h, STD_E_INVAL, "NULL parameter pointer");
  for (int n = 0; n < h->s.N; ++n)
    if (!A[n]) return fail(h, STD_E_INVAL, "NULL factor pointer");
  std::vector<float> buf;
  for (int n = 0; n < h->s.N; ++n) {
    const int J = h->s.J[n], Jp = h->s.Jp[n];
    const size_t rows = (size_t)h->s.I[n];
    if (J == Jp) {
      HIPCHK(h, hipMemcpyAsync(dA[n], A[n], rows * J * 4, hipMemcpyHostToDevice, h->stream));
    } else {
      buf.assign(rows * Jp, 0.f);
      for (size_t i = 0; i < rows; ++i) std::memcpy(buf.data() + i * Jp, A[n] + i * J, (size_t)J * 4);
      HIPCHK(h, hipMemcpyAsync(dA[n], buf.data(), buf.size() * 4, hipMemcpyHostToDevice, h->stream));
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));  // buf is reused for the next factor
  }
  HIPCHK(h, hipMemcpyAsync(dG, G, (size_t)h->s.P * 4, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return STD_OK;
}

}  // namespace

int stdecomp_get_params(stdecomp_handle* h, float* const* A, float* G) {
  if (!h) return STD_E_STATE;
  return copy_params_out(h, h->A, h->G, A, G);
}

int stdecomp_set_params(stdecomp_handle* h, const float* const* A, const float* G) {
  if (!h) return STD_E_STATE;
  const int rc = copy_params_in(h, h->A, h->G, A, G);
  return rc ? rc : refresh_bf16(h);
}

int stdecomp_get_velocity(stdecomp_handle* h, float* const* VA, float* VG) {
  if (!h) return STD_E_STATE;
  if (!h->VG) return fail(h, STD_E_STATE, "the handle has no momentum (options.momentum = 0)");
  return copy_params_out(h, h->VA, h->VG, VA, VG);
}

int stdecomp_set_velocity(stdecomp_handle* h, const float* const* VA, const float* VG) {
  if (!h) return STD_E_STATE;
  if (!h->VG) return fail(h, STD_E_STATE, "the handle has no momentum (options.momentum = 0)");
  return copy_params_in(h, h->VA, h->VG, VA, VG);
}

int stdecomp_get_kruskal(stdecomp_handle* h, float* const* B) {
  if (!h) return STD_E_STATE;
  if (h->R <= 0) return fail(h, STD_E_STATE, "the handle has a dense core (options.r_core = 0)");
  if (!B) return fail(h, STD_E_INVAL, "NULL parameter pointer");
  std::vector<float> buf((size_t)h->nB);
  HIPCHK(h, hipMemcpyAsync(buf.data(), h->B, buf.size() * 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  size_t o = 0;
  for (int n = 0; n < h->s.N; ++n) {
    if (!B[n]) return fail(h, STD_E_INVAL, "NULL factor pointer");
    const size_t len = (size_t)h->s.J[n] * h->R;
    std::memcpy(B[n], buf.data() + o, len * 4);
    o += len;
  }
  return STD_OK;
}

int stdecomp_set_kruskal(stdecomp_handle* h, const float* const* B) {
  if (!h) return STD_E_STATE;
  if (h->R <= 0) return fail(h, STD_E_STATE, "the handle has a dense core (options.r_core = 0)");
  if (!B) return fail(h, STD_E_INVAL, "NULL parameter pointer");
  std::vector<float> buf((size_t)h->nB), G;
  size_t o = 0;
  for (int n = 0; n < h->s.N; ++n) {
    if (!B[n]) return fail(h, STD_E_INVAL, "NULL factor pointer");
    const size_t len = (size_t)h->s.J[n] * h->R;
    std::memcpy(buf.data() + o, B[n], len * 4);
    o += len;
  }
  kruskal_product_host(h->s, h->R, buf.data(), G);
  HIPCHK(h, hipMemcpyAsync(h->B, buf.data(), buf.size() * 4, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(h->G, G.data(), G.size() * 4, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return STD_OK;
}

int stdecomp_set_epoch(stdecomp_handle* h, int64_t e) {
  if (!h) return STD_E_STATE;
  if (e < 0) return fail(h, STD_E_INVAL, "negative epoch");
  h->epoch = e;
  h->cursor = 0;
  return STD_OK;
}

int stdecomp_debug_barrier(stdecomp_handle* h, int32_t reps, double* us_per_barrier) {
  if (!h) return STD_E_STATE;
  if (reps < 1 || reps > 1000000 || !us_per_barrier) return fail(h, STD_E_INVAL, "bad barrier probe arguments");
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, STD_E_DEVICE, "hipSetDevice failed");
  stdk::ChainArgs a = chain_args(h);
  HIPCHK(h, hipMemsetAsync(h->err, 0, sizeof(int), h->stream));
  HIPCHK(h, hipMemsetAsync(h->bar, 0, (size_t)h->W * stdk::kFlagStride * sizeof(unsigned), h->stream));
  HIPCHK(h, hipEventRecord(h->ev[0], h->stream));
  HIPCHK(h, stdk::launch_barrier_probe(a, h->threads, reps, h->stream));
  HIPCHK(h, hipEventRecord(h->ev[1], h->stream));
  int err = 0;
  HIPCHK(h, hipMemcpyAsync(&err, h->err, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (err == 2) return fail(h, STD_E_DEVICE, kMisplaced);
  if (err) return fail(h, STD_E_DEVICE, "barrier probe: a workgroup gave up waiting");
  float ms = 0.f;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
  *us_per_barrier = 1000.0 * ms / reps;
  return STD_OK;
}

int stdecomp_debug_barrier_check(stdecomp_handle* h, int32_t reps, int64_t* stale) {
  if (!h) return STD_E_STATE;
  if (reps < 1 || reps > 1000000 || !stale) return fail(h, STD_E_INVAL, "bad barrier check arguments");
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, STD_E_DEVICE, "hipSetDevice failed");
  stdk::ChainArgs a = chain_args(h);
  // (the handle's loss scratch: W <= CUs lines of kFlagStride words, then the counter)
  unsigned* slots = reinterpret_cast<unsigned*>(h->dscratch);
  const size_t slot_words = (size_t)h->W * stdk::kFlagStride;
  if ((slot_words + 2) * 4 > 3 * 4096 * sizeof(double)) return fail(h, STD_E_INVAL, "too many workgroups");
  unsigned long long* dstale = reinterpret_cast<unsigned long long*>(h->dscratch + (slot_words + 1) / 2);
  HIPCHK(h, hipMemsetAsync(h->err, 0, sizeof(int), h->stream));
  HIPCHK(h, hipMemsetAsync(h->bar, 0, (size_t)h->W * stdk::kFlagStride * sizeof(unsigned), h->stream));
  HIPCHK(h, hipMemsetAsync(slots, 0, slot_words * 4, h->stream));
  HIPCHK(h, hipMemsetAsync(dstale, 0, sizeof(unsigned long long), h->stream));
  HIPCHK(h, stdk::launch_barrier_check(a, h->threads, reps, slots, dstale, h->stream));
  int err = 0;
  unsigned long long n = 0;
  HIPCHK(h, hipMemcpyAsync(&err, h->err, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(&n, dstale, sizeof(n), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (err == 2) return fail(h, STD_E_DEVICE, kMisplaced);
  if (err) return fail(h, STD_E_DEVICE, "barrier check: a workgroup gave up waiting");
  *stale = (int64_t)n;
  return STD_OK;
}

int stdecomp_debug_schedule(stdecomp_handle* h, int64_t epoch, int64_t batch, int32_t mode, int64_t* entries,
                            int32_t* sigma, int32_t* seg_off, int32_t* seg_row, int32_t* nseg, int32_t* m_out) {
  if (!h) return STD_E_STATE;
  if (epoch < 0 || batch < 0 || batch >= h->nb || mode < 0 || mode >= h->s.N || !entries || !sigma || !seg_off ||
      !seg_row || !nseg || !m_out)
    return fail(h, STD_E_INVAL, "bad debug_schedule arguments");
  int rc = run_schedule(h, epoch);
  if (rc) return rc;
  const int64_t base = batch * h->M;
  const int m = (int)((h->T - base < h->M) ? h->T - base : h->M);
  int64_t* dperm = nullptr;
  int32_t *doff = nullptr, *drow = nullptr, *dn = nullptr;
  if ((rc = dalloc(h, &dperm, (size_t)h->T, false)) || (rc = dalloc(h, &doff, (size_t)m + 1, false)) ||
      (rc = dalloc(h, &drow, (size_t)m, false)) || (rc = dalloc(h, &dn, 1, false))) {
    dfree(h, dperm);
    dfree(h, doff);
    dfree(h, drow);
    return rc;
  }

  std::vector<uint16_t> sig(m);
  hipError_t e = stdk::launch_perm_only(h->T, h->seed_sample, epoch, dperm, h->stream);
  if (e == hipSuccess)
    e = stdk::launch_debug_segments(h->s, h->coo_perm, h->sigma, h->T, h->M, batch, mode, doff, drow, dn, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(entries, dperm + base, (size_t)m * 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sig.data(), h->sigma + (size_t)mode * h->T + base, (size_t)m * 2, hipMemcpyDeviceToHost,
                       h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(nseg, dn, 4, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(seg_off, doff, (size_t)(m + 1) * 4, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(seg_row, drow, (size_t)m * 4, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  dfree(h, dperm);
  dfree(h, doff);
  dfree(h, drow);
  dfree(h, dn);
  if (e != hipSuccess) return hip_fail(h, e, "debug_schedule");
  for (int q = 0; q < m; ++q) sigma[q] = sig[q];
  *m_out = m;
  return STD_OK;
}

int stdecomp_sample_order(int64_t T, uint64_t seed, int64_t epoch, int64_t* out, int32_t out_on_device,
                          void* stream) {
  if (T < 1 || epoch < 0 || !out) return STD_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  if (out_on_device) {
    hipError_t e = stdk::launch_perm_only(T, seed, epoch, out, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e == hipSuccess ? STD_OK : STD_E_DEVICE;
  }
  int64_t* d = nullptr;
  if (hipMalloc((void**)&d, (size_t)T * 8) != hipSuccess) {
    (void)hipGetLastError();
    return STD_E_NOMEM;
  }
  hipError_t e = stdk::launch_perm_only(T, seed, epoch, d, st);
  if (e == hipSuccess) e = hipMemcpyAsync(out, d, (size_t)T * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d);
  return e == hipSuccess ? STD_OK : STD_E_DEVICE;
}

int stdecomp_info(const stdecomp_handle* h, stdecomp_info_out* out) {
  if (!h) return STD_E_STATE;
  if (!out) return STD_E_INVAL;
  out->workgroups = h->W;
  out->chunk = h->chunk;
  out->threads = h->threads;
  out->variant = stdk::chain_variant(h->s);
  out->lds_bytes = (int64_t)h->chain_lds;
  out->device_bytes = (int64_t)h->device_bytes;
  out->minibatches = h->nb;
  out->epoch = h->epoch;
  out->cursor = h->cursor;
  out->placement = h->xid >= 0 ? STD_PLACE_ONE_XCC : STD_PLACE_SPREAD;
  return STD_OK;
}

int stdecomp_free(stdecomp_handle* h) {
  if (!h) return STD_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->qstream) (void)hipStreamSynchronize(h->qstream);
  release(h);
  delete h;
  return STD_OK;
}

}  // extern "C"
