// gfx950 kernels of the minibatch chain with heavy-ball momentum for a chain
// placed on one XCC: the chain body of stdecomp_chain_body.h with velocities
// and the one-XCC grid barrier, for every rank variant.  A translation unit
// of its own so that the other kernels keep their code and all compile side
// by side.
#include "stdecomp_chain_body.h"

namespace stdk {

template <int JU>
hipError_t launch_mom_xcc_n(const ChainArgs& a, int threads, size_t bytes, hipStream_t st) {
  const bool n3 = a.s.N == 3;
  if (a.bf16)
    return n3 ? launch_chain_t<JU, 3, 13>(a, threads, bytes, st) : launch_chain_t<JU, 0, 13>(a, threads, bytes, st);
  return n3 ? launch_chain_t<JU, 3, 12>(a, threads, bytes, st) : launch_chain_t<JU, 0, 12>(a, threads, bytes, st);
}

// One chain with momentum on one XCC (a.xid >= 0, a.mom, dense core): the
// plan must be the one these arguments produce and every velocity buffer set.
hipError_t launch_chain_mom_xcc(const ChainArgs& a, int threads, hipStream_t st) {
  if (a.xid < 0 || !a.mom || a.R > 0 || !a.VG || !a.aux) return hipErrorInvalidValue;
  for (int n = 0; n < a.s.N; ++n)
    if (!a.VA[n]) return hipErrorInvalidValue;
  const size_t bytes = (size_t)a.lay.total * 4;
  ChainArgs chk = a;
  if (plan_chain_lds(chk, threads, a.bf16 != 0) != bytes || chk.lay.cbuf != a.lay.cbuf ||
      chk.lay.row1 != a.lay.row1 || chk.lay.ints != a.lay.ints || chk.lay.tmap != a.lay.tmap ||
      chk.lay.aux_len != a.lay.aux_len || chk.lay.hm_len != a.lay.hm_len || chk.lay.vg != a.lay.vg)
    return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  STDK_FOR_VARIANT(chain_variant(a.s), { e = launch_mom_xcc_n<JU>(a, threads, bytes, st); });
  return e;
}

}  // namespace stdk
