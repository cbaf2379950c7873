// gfx950 kernels of libstdecomp, the minibatch chain (device code in
// stdecomp_chain_body.h): the plain and Kruskal-core chain kernels, the
// barrier probe, and the host side of the chain: the LDS plan, the
// per-phase constants, the index maps and the launchers.
#include "stdecomp_chain_body.h"

namespace stdk {

// The chain's grid barrier alone, `reps` times in a row (no other work): the
// sync cost t_sync that bounds a chain at m / ((N + 1) t_sync) updates/s.
// (Placed as the chain is, so it times the chain's own barrier ordering.)
template <bool XL>
__global__ __launch_bounds__(kChainThreads) void k_barrier_probe(ChainArgs a, int reps) {
  __shared__ int flag[1];
  const int w = chain_workgroup<XL>(a);
  if (w < 0) return;
  unsigned passed = 0;
  for (int r = 0; r < reps; ++r) {
    passed += 1;
    barrier_arrive<XL>(a, w, passed);
    if (!barrier_wait<XL>(a, passed, flag)) return;
  }
}

hipError_t launch_barrier_probe(const ChainArgs& a, int threads, int reps, hipStream_t st) {
  ChainArgs args = a;
  void* params[] = {&args, &reps};
  const void* k = a.xid >= 0 ? (const void*)k_barrier_probe<true> : (const void*)k_barrier_probe<false>;
  return hipLaunchCooperativeKernel(k, dim3(a.W * a.xs), dim3(threads), params, 0, st);
}

// The barrier's memory ordering, checked: before each of `reps` barriers
// workgroup w writes the round number into its own line of `slots` (plain
// store), and after it reads every workgroup's line (plain loads); a second
// barrier keeps round r + 1's writes after every read of round r.  Each read
// that does not return the current round adds one to *stale.
template <bool XL>
__global__ __launch_bounds__(kChainThreads) void k_barrier_check(ChainArgs a, int reps, unsigned* slots,
                                                                 unsigned long long* stale) {
  __shared__ int flag[1];
  const int w = chain_workgroup<XL>(a);
  if (w < 0) return;
  unsigned passed = 0;
  unsigned long long bad = 0;
  for (int r = 1; r <= reps; ++r) {
    if (threadIdx.x == 0) slots[w * kFlagStride] = (unsigned)r;
    passed += 1;
    barrier_arrive<XL>(a, w, passed);
    if (!barrier_wait<XL>(a, passed, flag)) return;
    for (int v = threadIdx.x; v < a.W; v += blockDim.x) bad += slots[v * kFlagStride] != (unsigned)r ? 1 : 0;
    passed += 1;
    barrier_arrive<XL>(a, w, passed);
    if (!barrier_wait<XL>(a, passed, flag)) return;
  }
  if (bad) atomicAdd(stale, bad);
}

hipError_t launch_barrier_check(const ChainArgs& a, int threads, int reps, unsigned* slots, unsigned long long* stale,
                                hipStream_t st) {
  ChainArgs args = a;
  void* params[] = {&args, &reps, &slots, &stale};
  const void* k = a.xid >= 0 ? (const void*)k_barrier_check<true> : (const void*)k_barrier_check<false>;
  return hipLaunchCooperativeKernel(k, dim3(a.W * a.xs), dim3(threads), params, 0, st);
}

// Where the dispatcher puts the blocks of a grid: out[b] = the XCC of block b.
__global__ __launch_bounds__(64) void k_xcc_probe(int* out) {
  const int x = xcc_id();
  if (threadIdx.x == 0) out[blockIdx.x] = x;
}

hipError_t launch_xcc_probe(int* out, int blocks, hipStream_t st) {
  k_xcc_probe<<<blocks, 64, 0, st>>>(out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Host side: the LDS plan, the per-phase constants and the index maps.
// ---------------------------------------------------------------------------
size_t plan_chain_lds(ChainArgs& a, int threads, bool bf, int* aux) {
  // the row buffer is followed by kRowTail zero words (see k_chain)
  const Shape& s = a.s;
  // every region below is sized from these: refuse an incomplete request
  if (a.W < 1 || a.chunk < 1 || a.chunk > threads || (a.W > 1 && a.split_cap < a.W - 1)) return 0;
  if (s.N < 2 || s.N > kMaxOrder) return 0;
  const int N = s.N;
  const int JU = chain_variant(s);
  const int JR = JU ? JU : kMaxRank;
  auto al = [](size_t f) { return (f + 3) & ~(size_t)3; };
  struct ModeT {
    int lo, nhi, khi, jlo, kp, nt, hi[kMaxOrder];
    int hm_off, tb_off, tb_len;
    int ks2, hpt, ctn;
  } mt[kMaxOrder];
  int jmax = 0, hm_len = 0, tb_sum = 0, tb_max = 0, khimax = 1;
  const bool ts = N != 3;  // the contraction of the kernels for N != 3 is two-stage (32x32 tiles)
  for (int n = 0; n < N; ++n) {
    ModeT& q = mt[n];
    jmax = s.J[n] > jmax ? s.J[n] : jmax;
    q.lo = n == 0 ? 1 : 0;
    q.nhi = 0;
    q.khi = 1;
    for (int k = 0; k < N; ++k)
      if (k != n && k != q.lo) {
        q.hi[q.nhi++] = k;
        q.khi *= s.J[k];
      }
    q.jlo = s.J[q.lo];
    q.kp = bf ? ((q.jlo + 15) & ~15) : pad4(q.jlo);
    q.nt = (s.J[n] + 15) / 16;
    q.ks2 = bf ? (q.jlo + 7) / 8 : (q.jlo + 1) / 2;  // K steps of 8 (BF16) or 2 (FP32)
    q.hpt = 32 / s.J[n];
    q.ctn = (q.khi + q.hpt - 1) / q.hpt;
    // three-mode, BF16: [h][j_n tile][16 j_n][kp k]; FP32: [h][j_n tile][kp k][16 j_n];
    // two-stage: [column tile][K step][64 lanes] (BF16: 4 values per lane)
    q.tb_len = ts ? q.ctn * q.ks2 * 64 * (bf ? 4 : 1) : q.khi * q.nt * q.kp * 16;
    q.hm_off = hm_len;
    hm_len += q.khi * (1 + q.nhi);
    q.tb_off = tb_sum;
    tb_sum += q.tb_len;
    tb_max = q.tb_len > tb_max ? q.tb_len : tb_max;
    khimax = q.khi > khimax ? q.khi : khimax;
  }
  auto tbf = [&](int len) { return bf ? (size_t)(len + 1) / 2 : (size_t)len; };
  ChainLayout& L = a.lay;
  L.chp = (a.chunk + 31) & ~31;
  L.hs = L.chp + 4;
  {  // chunk-major row buffers: ceil(J_k / V) 16-byte chunks per mode and sample
    const int V = bf ? 8 : 4;
    int c = 0;
    for (int k = 0; k < kMaxOrder; ++k) {
      L.coff[k] = c;
      if (k < N) c += (s.J[k] + V - 1) / V;
    }
    L.ctot = c;
    L.rowsz = L.ctot * L.chp * 4;
  }
  // waves per 32-sample block in the FP32 contraction, each with its own
  // partial-E slots
  const int nwb = std::max(1, (threads / 64) / ((L.chp + 31) / 32));
  if (!ts) {
    L.es = 16 * ((jmax + 15) / 16) + 1;
  } else {
    int e = 1;
    for (int n = 0; n < N; ++n) e = std::max(e, nwb * mt[n].hpt * s.J[n]);
    L.es = e + 1 + (e & 1);  // odd, > e
  }
  // (sized by the largest rank, not the kernel's register bound: the generic
  // kernels read at most J_max values of a split-row entry, and the core GEMM
  // reads rows j0 >= J_0 of r a(0) only into output rows it does not store)
  // the carry of one chunk: two slots of 2 + J_n words, the old row and,
  // with momentum, the old velocity (a multiple of 4: it is copied as float4)
  if (a.W > 1 && (a.carry_stride < 4 + (a.mom ? 4 : 3) * jmax || (a.carry_stride & 3))) return 0;
  if (a.mom && a.R > 0) return 0;
  L.ras = pad4(jmax) + 1;
  L.sstride = 4 + pad4(jmax);
  L.wstride = pad4(JR) + 4;
  {  // two-level core update when every workgroup summing all partials would cost more than a barrier
    const int P4 = pad4(s.P) / 4;
    const int per = (P4 + a.W - 1) / a.W;
    const int grp = per <= threads ? threads / per : 0;
    const int vg = grp > 0 ? (a.W + grp - 1) / grp : 0;
    // (three-mode kernels always take the one-level update)
    L.core2 = (N != 3 && a.W >= 8 && grp >= 1 && vg <= 8 && (long long)P4 * a.W >= 8192) ? 1 : 0;
    L.cper = per;
    L.cgrp = grp;
    L.cvg = vg;
  }
  if (a.R > 0) L.core2 = 0;  // the Kruskal core has its own reduction
  // Kruskal core: B resident, and the [W | x] rows and their Gram matrix in
  // the space of the hp / E / r a(0) regions (grown if they are smaller)
  size_t kr_extra = 0;
  L.kb = L.kwt = L.kg = L.kws = L.ke = L.klg = 0;
  for (int k = 0; k < kMaxOrder; ++k) L.kboff[k] = 0;
  if (a.R > 0) {
    int o = 0;
    for (int k = 0; k < N; ++k) {
      L.kboff[k] = o;
      o += s.J[k] * a.R;
    }
    L.ke = a.R * jmax + 1;
    L.kws = ((L.ke + 15) & ~15) + 1;  // whole 16-column tiles, odd stride
    L.klg = (L.ke * (L.ke + 1)) / 2;
    const int PL = s.lstride[N / 2];
    const size_t halves = (size_t)(PL + s.P / PL) * a.R;  // the two half-products of forming G
    const size_t need = al(std::max(std::max((size_t)L.chp * L.kws, (size_t)L.klg), halves)) +
                        al(std::max((size_t)L.ke * L.ke, (size_t)threads));
    const size_t have = al((size_t)khimax * L.hs) + al((size_t)L.chp * L.es) + al((size_t)L.chp * L.ras);
    kr_extra = need > have ? need - have : 0;
  }
  const size_t kb_len = a.R > 0 ? al((size_t)(L.kboff[N - 1] + s.J[N - 1] * a.R)) : 0;
  const size_t red_len = L.core2 ? (size_t)L.cgrp * L.cper * 4 : 0;
  const size_t vg_len = a.mom ? (L.core2 ? (size_t)4 * L.cper : (size_t)s.P) : 0;
  size_t common = al(red_len) + al(vg_len) + kb_len + kr_extra + al(s.P) + al(2 * (size_t)L.rowsz + kRowTail) +
                  al((size_t)khimax * L.hs) + al((size_t)L.chp * L.es) +
                  al((size_t)L.chp * L.ras) + al((size_t)a.split_cap * L.sstride) +
                  al(a.W > 1 ? (size_t)a.W * a.carry_stride : 0) + al((size_t)hm_len) +
                  al((size_t)(threads / 64) * L.wstride) + 2 * (size_t)a.W + 8;
  const size_t all_resident = common + al(tbf(tb_sum)) + al((size_t)tb_sum);
  L.tb_all = all_resident * 4 <= (size_t)(a.lds_cap > 0 ? a.lds_cap : 163840) ? 1 : 0;
  size_t off = 0;
  L.gs = (int)off;    off += al(s.P);
  L.vg = (int)off;    off += al(vg_len);
  L.tb = (int)off;    off += al(L.tb_all ? tbf(tb_sum) : tbf(tb_max));
  L.row0 = (int)off;  // (the two buffers are adjacent: one zero fill covers both and the tail)
  L.row1 = L.row0 + L.rowsz;
  off += al(2 * (size_t)L.rowsz + kRowTail);
  L.hp = (int)off;    off += al((size_t)khimax * L.hs);
  L.ebuf = (int)off;  off += al((size_t)L.chp * L.es);
  L.ra = (int)off;    off += al((size_t)L.chp * L.ras) + kr_extra;
  L.kwt = L.hp;
  L.kg = L.hp + (int)al(std::max(std::max((size_t)L.chp * L.kws, (size_t)L.klg),
                                   a.R > 0 ? (size_t)(s.lstride[N / 2] + s.P / s.lstride[N / 2]) * a.R : (size_t)0));
  L.kb = (int)off;    off += kb_len;
  L.split = (int)off; off += al((size_t)a.split_cap * L.sstride);
  L.cbuf = (int)off;  off += al(a.W > 1 ? (size_t)a.W * a.carry_stride : 0);
  L.hmap = (int)off;  off += al((size_t)hm_len);
  L.tmap = (int)off;  off += L.tb_all ? al((size_t)tb_sum) : 0;
  L.wscr = (int)off;  off += al((size_t)(threads / 64) * L.wstride);
  L.red = (int)off;   off += al(red_len);
  L.ints = (int)off;  off += 2 * (size_t)a.W + 8;
  L.total = (int)off;
  L.aux_len = hm_len + (L.tb_all ? tb_sum : 0);
  L.hm_len = hm_len;

  // per-phase constants
  auto upd_of = [&](int ph) { return ph == 0 ? -1 : ph - 1; };
  for (int ph = 0; ph <= N; ++ph) {
    PhaseTab& t = a.pt[ph];
    const int n = ph == 0 ? 0 : ph - 1;
    const ModeT& q = mt[n];
    t.n = n;
    t.upd = upd_of(ph);
    t.pm = upd_of((ph + N) % (N + 1));
    const int pm2 = upd_of((ph + N - 1) % (N + 1));
    t.post = (t.pm >= 0 ? 1 << t.pm : 0) | (pm2 >= 0 ? 1 << pm2 : 0);
    t.khi = q.khi;
    t.nhi = q.nhi;
    t.jlo = q.jlo;
    t.kp = q.kp;
    t.nt = q.nt;
    t.ls_n = s.lstride[n];
    t.ls_lo = s.lstride[q.lo];
    t.c_lo = L.coff[q.lo];
    t.c_n = L.coff[n];
    t.Jn = s.J[n];
    t.c_hi = q.nhi > 0 ? L.coff[q.hi[0]] : 0;
    t.c_hi2 = q.nhi > 1 ? L.coff[q.hi[1]] : 0;
    t.tb_off = L.tb_all ? q.tb_off : 0;
    t.tb_len = q.tb_len;
    t.hm_off = q.hm_off;
    t.tm_off = t.tb_off;
    t.ks2 = q.ks2;
    t.hpt = q.hpt;
    t.ctn = q.ctn;
    // (hpt a power of two filling the 32 columns: the contraction folds the hpt slots into one)
    const bool fold = q.hpt > 1 && (q.hpt & (q.hpt - 1)) == 0 && q.hpt * s.J[n] == 32;
    t.ens = ts ? (fold ? nwb : nwb * q.hpt) : 1;
  }
  for (int ph = N + 1; ph <= kMaxOrder; ++ph) a.pt[ph] = PhaseTab{};

  // index maps: per mode, [khi core offsets][khi * nhi row-buffer offsets],
  // then (resident tables) the table gather maps in table layout
  if (aux) {
    for (int n = 0; n < N; ++n) {
      const ModeT& q = mt[n];
      int* hm = aux + q.hm_off;
      std::vector<int> hoff(q.khi);
      for (int h = 0; h < q.khi; ++h) {
        int hh = h, o = 0;
        for (int i = 0; i < q.nhi; ++i) {
          const int Jk = s.J[q.hi[i]];
          const int d = hh % Jk;
          hh /= Jk;
          o += d * s.lstride[q.hi[i]];
          // value d of mode hi[i] in the chunk-major row buffer, less the sample term
          hm[q.khi + h * q.nhi + i] = bf ? (L.coff[q.hi[i]] + d / 8) * L.chp * 8 + d % 8
                                         : (L.coff[q.hi[i]] + d / 4) * L.chp * 4 + d % 4;
        }
        hm[h] = o;
        hoff[h] = o;
      }
      if (L.tb_all) {
        int* tm = aux + hm_len + q.tb_off;
        for (int e = 0; e < q.tb_len; ++e) {
          if (!ts) {
            int k, c, ht;
            if (bf) {
              k = e % q.kp;
              const int r = e / q.kp;
              c = r & 15;
              ht = r >> 4;
            } else {
              c = e & 15;
              const int r = e >> 4;
              k = r % q.kp;
              ht = r / q.kp;
            }
            const int h = ht / q.nt, t = ht - h * q.nt;
            const int jn = 16 * t + c;
            tm[e] = (k < q.jlo && jn < s.J[n]) ? hoff[h] + k * s.lstride[q.lo] + jn * s.lstride[n] : -1;
          } else {
            const int lw = bf ? 4 : 1;  // values per lane
            const int ct = e / (q.ks2 * 64 * lw), r = e - ct * q.ks2 * 64 * lw;
            const int ks = r / (64 * lw), l = (r / lw) & 63, ee = r % lw;
            const int k = bf ? 8 * ks + 4 * (l >> 5) + ee : 2 * ks + (l >> 5), c = l & 31;
            const int hh = c / s.J[n], jn = c - hh * s.J[n];
            const int h = ct * q.hpt + hh;
            tm[e] = (k < q.jlo && hh < q.hpt && h < q.khi) ? hoff[h] + k * s.lstride[q.lo] + jn * s.lstride[n] : -1;
          }
        }
      }
    }
  }
  return off * 4;
}


// three-mode tensors get a kernel with the mode loops unrolled
template <int JU>
hipError_t launch_chain_n(const ChainArgs& a, int threads, size_t bytes, hipStream_t st, int bf) {
  const bool n3 = a.s.N == 3;
  if (bf) return n3 ? launch_chain_t<JU, 3, 1>(a, threads, bytes, st) : launch_chain_t<JU, 0, 1>(a, threads, bytes, st);
  return n3 ? launch_chain_t<JU, 3, 0>(a, threads, bytes, st) : launch_chain_t<JU, 0, 0>(a, threads, bytes, st);
}

template <int JU>
hipError_t launch_kruskal_n(const ChainArgs& a, int threads, size_t bytes, hipStream_t st, int f) {
  const bool n3 = a.s.N == 3;
  if (f == 3) return n3 ? launch_chain_t<JU, 3, 3>(a, threads, bytes, st) : launch_chain_t<JU, 0, 3>(a, threads, bytes, st);
  return n3 ? launch_chain_t<JU, 3, 2>(a, threads, bytes, st) : launch_chain_t<JU, 0, 2>(a, threads, bytes, st);
}

hipError_t launch_chain_queue(int n3, int bf, int mom, const ChainArgs* dev_args, const int* dev_list, int nslots,
                              int W, int threads, size_t bytes, hipStream_t st) {
  if (mom) return launch_chain_queue_mom(n3, bf, dev_args, dev_list, nslots, W, threads, bytes, st);
  if (bf) return n3 ? launch_queue_t<3, 1>(dev_args, dev_list, nslots, W, threads, bytes, st)
                    : launch_queue_t<0, 1>(dev_args, dev_list, nslots, W, threads, bytes, st);
  return n3 ? launch_queue_t<3, 0>(dev_args, dev_list, nslots, W, threads, bytes, st)
            : launch_queue_t<0, 0>(dev_args, dev_list, nslots, W, threads, bytes, st);
}

hipError_t launch_chain(const ChainArgs& a, int threads, hipStream_t st) {
  const int var = chain_variant(a.s);
  const size_t bytes = (size_t)a.lay.total * 4;
  {  // the plan must be the one these arguments produce
    ChainArgs chk = a;
    if (plan_chain_lds(chk, threads, a.bf16 != 0) != bytes || chk.lay.cbuf != a.lay.cbuf || chk.lay.row1 != a.lay.row1 ||
        chk.lay.ints != a.lay.ints || chk.lay.tmap != a.lay.tmap || chk.lay.aux_len != a.lay.aux_len ||
        chk.lay.hm_len != a.lay.hm_len || chk.lay.vg != a.lay.vg || !a.aux)
      return hipErrorInvalidValue;
    if (a.mom) {  // momentum: every velocity buffer
      if (!a.VG) return hipErrorInvalidValue;
      for (int n = 0; n < a.s.N; ++n)
        if (!a.VA[n]) return hipErrorInvalidValue;
    }
  }
  if (a.xid >= 0) {  // one XCC: the plain dense-core kernels only
    if (a.mom || a.R > 0) return hipErrorInvalidValue;
    return launch_chain_xcc(a, threads, bytes, st);
  }
  if (a.mom) return launch_chain_mom(a, threads, bytes, st);
  if (a.R > 0) {  // Kruskal core: kernels for equal ranks 5, 8, 10, else the generic-rank ones
    const int f = a.bf16 ? 3 : 2;
    switch (var) {
      case 5: return launch_kruskal_n<5>(a, threads, bytes, st, f);
      case 8: return launch_kruskal_n<8>(a, threads, bytes, st, f);
      case 10: return launch_kruskal_n<10>(a, threads, bytes, st, f);
      default: return launch_kruskal_n<0>(a, threads, bytes, st, f);
    }
  }
  hipError_t e = hipSuccess;
  if (a.bf16) {
    STDK_FOR_VARIANT(var, { e = launch_chain_n<JU>(a, threads, bytes, st, 1); });
  } else {
    STDK_FOR_VARIANT(var, { e = launch_chain_n<JU>(a, threads, bytes, st, 0); });
  }
  return e;
}

}  // namespace stdk
