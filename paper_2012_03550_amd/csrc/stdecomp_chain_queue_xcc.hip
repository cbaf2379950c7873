// gfx950 kernels of the batched chain launch with every slot on one XCC: the
// chain body of stdecomp_chain_body.h with the one-XCC grid barrier, run by
// slots of W workgroups as k_chain_queue runs them.  The dispatcher deals the
// blocks of a grid to the nx XCCs in turn, so the blocks of one residue
// b mod nx share an XCC; slot q takes W of them: residue r holds slots
// r (nslots / nx) .. (r + 1) (nslots / nx) - 1 (nslots a multiple of nx), and
// workgroup w of slot q is block nx (W (q mod (nslots / nx)) + w) + r.
// A translation unit of its own so that the spread kernels keep their code.
#include "stdecomp_chain_body.h"

namespace stdk {

template <int NU, int BFI>
__global__ __launch_bounds__(kChainThreads) void k_chain_queue_xcc(const ChainArgs* __restrict__ all,
                                                                   const int* __restrict__ list, int nslots, int W,
                                                                   int nx) {
  const int b = blockIdx.x;
  const int r = b % nx, k = b / nx;
  const int q = r * (nslots / nx) + k / W, w = k % W;
  if (list[q] == list[q + 1]) return;  // an empty slot
  const int* models = list + nslots + 1;
  {
    // the slot's workgroups must share one XCC: the first wave to arrive
    // claims its XCC in the last word of the slot's flags (zero at launch);
    // a block on another XCC sets the first chain's error flag to 2 and
    // leaves, and the slot's chains stop at their next barrier
    const ChainArgs& a0 = all[models[list[q]]];
    int ok = 1;
    if (__lane_id() == 0) {
      const unsigned x = (unsigned)xcc_id() + 1u;
      unsigned e = 0;
      ok = __hip_atomic_compare_exchange_strong(a0.bar + kClaim(W), &e, x, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT) || e == x;
      if (!ok) __hip_atomic_store(a0.err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!__builtin_amdgcn_readfirstlane(ok)) return;
  }
  for (int i = list[q]; i < list[q + 1]; ++i) {
    const ChainArgs& a = all[models[i]];
    // (the body a chain runs alone on one XCC, so that results are bit-identical)
    STDK_FOR_VARIANT(a.jv, (chain_body<JU, NU, BFI>(a, w)));
    if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  }
}

template <int NU, int BFI>
hipError_t launch_queue_xcc_t(const ChainArgs* dev_args, const int* dev_list, int nslots, int W, int nx, int threads,
                              size_t bytes, hipStream_t st) {
  const ChainArgs* pa = dev_args;
  const int* pl = dev_list;
  void* params[] = {&pa, &pl, &nslots, &W, &nx};
  hipError_t e = hipFuncSetAttribute((const void*)k_chain_queue_xcc<NU, BFI>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess)
    e = hipLaunchCooperativeKernel((const void*)k_chain_queue_xcc<NU, BFI>, dim3(nslots * W), dim3(threads), params,
                                   (unsigned)bytes, st);
  return e;
}

// Every chain of the batch: dense core, no momentum, its ChainArgs with
// xid >= 0 and its slot's flags zero; nslots a multiple of nx, nslots W
// blocks co-resident.
hipError_t launch_chain_queue_xcc(int n3, int bf, const ChainArgs* dev_args, const int* dev_list, int nslots, int W,
                                  int nx, int threads, size_t bytes, hipStream_t st) {
  if (nx < 1 || nslots % nx != 0 || W < 1) return hipErrorInvalidValue;
  if (bf) return n3 ? launch_queue_xcc_t<3, 9>(dev_args, dev_list, nslots, W, nx, threads, bytes, st)
                    : launch_queue_xcc_t<0, 9>(dev_args, dev_list, nslots, W, nx, threads, bytes, st);
  return n3 ? launch_queue_xcc_t<3, 8>(dev_args, dev_list, nslots, W, nx, threads, bytes, st)
            : launch_queue_xcc_t<0, 8>(dev_args, dev_list, nslots, W, nx, threads, bytes, st);
}

}  // namespace stdk
