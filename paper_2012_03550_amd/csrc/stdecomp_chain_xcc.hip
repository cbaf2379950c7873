// gfx950 kernels of the minibatch chain for a chain placed on one XCC: the
// chain body of stdecomp_chain_body.h with the one-XCC grid barrier (flags
// packed and written without an L2 write-back), for every rank variant of the
// dense core without momentum.  A translation unit of its own so that the
// spread kernels keep their code and both sets compile side by side.
#include "stdecomp_chain_body.h"

namespace stdk {

template <int JU>
hipError_t launch_xcc_n(const ChainArgs& a, int threads, size_t bytes, hipStream_t st) {
  const bool n3 = a.s.N == 3;
  if (a.bf16) return n3 ? launch_chain_t<JU, 3, 9>(a, threads, bytes, st) : launch_chain_t<JU, 0, 9>(a, threads, bytes, st);
  return n3 ? launch_chain_t<JU, 3, 8>(a, threads, bytes, st) : launch_chain_t<JU, 0, 8>(a, threads, bytes, st);
}

hipError_t launch_chain_xcc(const ChainArgs& a, int threads, size_t bytes, hipStream_t st) {
  if (a.xid < 0 || a.mom || a.R > 0) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  STDK_FOR_VARIANT(chain_variant(a.s), { e = launch_xcc_n<JU>(a, threads, bytes, st); });
  return e;
}

}  // namespace stdk
