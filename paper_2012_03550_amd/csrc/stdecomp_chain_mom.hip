// gfx950 kernels of the minibatch chain with heavy-ball momentum: the chain
// body of stdecomp_chain_body.h instantiated with velocities (v <- mu v + g,
// theta <- theta - gamma v on every sub-step), for every rank variant, alone
// and in batched launches.  A translation unit of its own so that the plain
// kernels keep their code and both sets compile side by side.
#include "stdecomp_chain_body.h"

namespace stdk {

template <int JU>
hipError_t launch_mom_n(const ChainArgs& a, int threads, size_t bytes, hipStream_t st) {
  const bool n3 = a.s.N == 3;
  if (a.bf16) return n3 ? launch_chain_t<JU, 3, 5>(a, threads, bytes, st) : launch_chain_t<JU, 0, 5>(a, threads, bytes, st);
  return n3 ? launch_chain_t<JU, 3, 4>(a, threads, bytes, st) : launch_chain_t<JU, 0, 4>(a, threads, bytes, st);
}

hipError_t launch_chain_mom(const ChainArgs& a, int threads, size_t bytes, hipStream_t st) {
  if (!a.mom || a.R > 0) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  STDK_FOR_VARIANT(chain_variant(a.s), { e = launch_mom_n<JU>(a, threads, bytes, st); });
  return e;
}

hipError_t launch_chain_queue_mom(int n3, int bf, const ChainArgs* dev_args, const int* dev_list, int nslots, int W,
                                  int threads, size_t bytes, hipStream_t st) {
  if (bf) return n3 ? launch_queue_t<3, 5>(dev_args, dev_list, nslots, W, threads, bytes, st)
                    : launch_queue_t<0, 5>(dev_args, dev_list, nslots, W, threads, bytes, st);
  return n3 ? launch_queue_t<3, 4>(dev_args, dev_list, nslots, W, threads, bytes, st)
            : launch_queue_t<0, 4>(dev_args, dev_list, nslots, W, threads, bytes, st);
}

}  // namespace stdk
