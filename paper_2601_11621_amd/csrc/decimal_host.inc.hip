// Radix conversion to decimal text (the optional decimal output of Sec. 3.2):
// plan and C ABI.
//
// x (L limbs) is cut into n_0 = ceil(L/16) leaves of sixteen limbs, each turned
// into len_0 = 18 radix-10^9 digits.  Level j holds n_j nodes of len_j digits;
// node i is the value of limbs [i 16 2^j, (i+1) 16 2^j).  Two neighbours join as
// hi * P_j + lo with P_j = 2^(512 2^j) in radix 10^9 (t_j digits; P_{j+1} =
// P_j^2), giving len_{j+1} = len_j + t_j digits; a last node without a
// partner is carried up (copied and zero-padded).  All products of a level are
// one uniform batch.  The squarings that make the powers run on a second
// stream with their own scratch, level j waiting only for P_j.  A product too long for one transform (only the top one,
// beyond about 1.2e9 decimal digits) is cut in two along hi:
// T = hi_lo * P + lo, then c = hi_hi * P + T / B^m above the copied T mod B^m.

struct DecLevel {
  uint64_t nodes = 0, len = 0;   // n_j, len_j
  uint64_t t = 0;                // digits of P_j used as the operand
  uint64_t poff = 0;             // P_j in the power area
};

struct DecPlan {
  uint64_t L = 0;
  std::vector<DecLevel> lv;      // levels 0 .. h (level h: one node)
  std::vector<Stage> pw;         // P_j = P_{j-1}^2, j = 1 .. h-1
  std::vector<std::vector<Stage>> join;   // stages of level j -> j+1
  uint64_t x[2] = {0, 0}, xsize = 0, pbase = 0, psize = 0, tbase = 0, tsize = 0;   // uint32 offsets
  uint64_t res_len = 0, F_words = 0, nblk_max = 0;      // joins
  uint64_t res2_len = 0, F2_words = 0, nblk2_max = 0;   // squarings (second stream)
  size_t off_res = 0, off_F = 0, off_res2 = 0, off_F2 = 0, off_ctl = 0, ctl_words = 0, total = 0;   // bytes
  uint64_t products = 0, product_digits = 0;
};

// an upper bound on the radix-10^9 digits of 2^k (exact count + 1 at most)
uint64_t dec_digits_pow2(uint64_t k) { return (uint64_t)((long double)k * 0.30102999566398119521L / 9.0L) + 2; }

Stage dec_stage(uint64_t nmul, const UniDesc& u, uint64_t d0, uint64_t sd, uint64_t ld, bool* ok) {
  Stage s;
  s.dec = true;
  const uint64_t len = (uint64_t)u.la + u.lb;
  int k = ceil_log2(len - 1);
  if (k < 6) k = 6;
  *ok = k <= CAT_MAX_LOGN && nmul > 0 && u.la > 0 && u.lb > 0;
  if (!*ok) return s;
  s.logN = k;
  s.cls = g_tune.cls[k];
  s.logM = g_tune.log_row[k];
  s.maxL = g_tune.log_pass[k];
  s.nmul = nmul;
  s.limbs = nmul * len;
  s.dv = DescView{};
  s.dv.uni = 1;
  s.dv.u = u;
  s.sv = SegView{};
  s.sv.ubl = (uint32_t)((len + DEC_CRT_BLOCK - 1) / DEC_CRT_BLOCK);
  s.sv.nseg = (uint32_t)nmul;
  s.sv.iseg[0] = CrtSeg{u.c0, 0, len, d0, ld};
  s.sv.ustep[0] = u.sc;
  s.sv.ustep[1] = sd;
  const uint64_t nb = nmul * s.sv.ubl;
  *ok = nb < (1ull << 31);
  s.nblk = (uint32_t)nb;
  s.nseg = (uint32_t)nmul;
  return s;
}

cat_status make_dec_plan(uint64_t L, DecPlan* D) {
  DecPlan& P = *D;
  P = DecPlan{};
  P.L = L;
  if (L > (1ull << CAT_MAX_LOGN)) return CAT_ERANGE;
  // levels
  DecLevel l0;
  l0.nodes = std::max<uint64_t>(1, (L + DEC_LEAF_LIMBS - 1) / DEC_LEAF_LIMBS);
  l0.len = DEC_LEAF_DIGITS;
  P.lv.push_back(l0);
  uint64_t pcap = DEC_LEAF_DIGITS;   // capacity of P_j's slot
  uint64_t poff = 0;
  for (int j = 0; P.lv[j].nodes > 1; j++) {
    DecLevel& c = P.lv[j];
    c.poff = poff;
    c.t = j == 0 ? (uint64_t)DEC_LEAF_DIGITS
                 : std::min<uint64_t>(pcap, dec_digits_pow2((32ull * DEC_LEAF_LIMBS) << j));
    poff += pcap;
    pcap = 2 * c.t;   // P_{j+1} = P_j^2 as a product of 2 t_j digits
    DecLevel nx;
    nx.nodes = (c.nodes + 1) / 2;
    nx.len = c.len + c.t;
    P.lv.push_back(nx);
  }
  const int h = (int)P.lv.size() - 1;
  P.psize = poff;
  for (const DecLevel& l : P.lv) P.xsize = std::max<uint64_t>(P.xsize, l.nodes * l.len);
  // buffers (uint32 offsets): X0 | X1 | powers | split temporary
  uint64_t o = 0;
  auto take = [&](uint64_t words) {
    const uint64_t r = o;
    o = align_up(o + words, 64);
    return r;
  };
  P.x[0] = take(P.xsize);
  P.x[1] = take(P.xsize);
  P.pbase = take(P.psize);
  // squarings P_j = P_{j-1}^2 for j = 1 .. h-1
  for (int j = 1; j < h; j++) {
    const DecLevel& a = P.lv[j - 1];
    UniDesc u{P.pbase + a.poff, 0, P.pbase + a.poff, 0, P.pbase + P.lv[j].poff, 0, (uint32_t)a.t, (uint32_t)a.t};
    bool ok = false;
    P.pw.push_back(dec_stage(1, u, 0, 0, 0, &ok));
    if (!ok) return CAT_ERANGE;
  }
  // joins
  uint64_t tneed = 0;
  for (int j = 0; j < h; j++) {
    const DecLevel& c = P.lv[j];
    const DecLevel& nx = P.lv[j + 1];
    const uint64_t xin = P.x[j & 1], xout = P.x[(j + 1) & 1];
    const uint64_t np = c.nodes / 2;
    std::vector<Stage> v;
    UniDesc u{xin + c.len, 2 * c.len, P.pbase + c.poff, 0, xout, nx.len, (uint32_t)c.len, (uint32_t)c.t};
    bool ok = false;
    Stage s = dec_stage(np, u, xin, 2 * c.len, c.len, &ok);
    if (ok) {
      v.push_back(s);
    } else {
      // one product only, cut along hi
      if (np != 1) return CAT_ERANGE;
      const uint64_t m = (c.len + 1) / 2;
      if (m + c.t < c.len) return CAT_EINTERNAL;
      const uint64_t tb = 0;   // offset inside the temporary (set below)
      UniDesc ua{xin + c.len, 0, P.pbase + c.poff, 0, tb, 0, (uint32_t)m, (uint32_t)c.t};
      Stage sa = dec_stage(1, ua, xin, 0, c.len, &ok);
      if (!ok) return CAT_ERANGE;
      UniDesc ub{xin + c.len + m, 0, P.pbase + c.poff, 0, xout + m, 0, (uint32_t)(c.len - m), (uint32_t)c.t};
      Stage sb = dec_stage(1, ub, tb + m, 0, c.t, &ok);
      if (!ok) return CAT_ERANGE;
      sb.tails.n = 1;
      sb.tails.off[0] = 0;
      sb.tails.len[0] = m;
      sb.tail_out_base = xout;
      tneed = std::max<uint64_t>(tneed, m + c.t);
      v.push_back(sa);
      v.push_back(sb);
    }
    P.join.push_back(v);
  }
  P.tsize = tneed;
  P.tbase = take(P.tsize);
  // the split stages address the temporary relative to tbase
  for (auto& v : P.join) {
    if (v.size() != 2) continue;
    v[0].dv.u.c0 += P.tbase;
    v[0].sv.iseg[0].out_pos += P.tbase;
    v[1].sv.iseg[0].add_pos += P.tbase;
    v[1].tail_in_base = P.tbase;
  }
  // scratch of the products
  auto scratch = [&](const Stage& s, uint64_t* res_len, uint64_t* F_words, uint64_t* nblk_max) {
    *res_len = std::max<uint64_t>(*res_len, s.limbs);
    if (s.cls == CLS_LARGE) *F_words = std::max<uint64_t>(*F_words, s.nmul * 6ull << s.logN);
    // a join's common second operand, transformed once per prime
    if (s.cls == CLS_LDS && s.nmul > 1) *F_words = std::max<uint64_t>(*F_words, 3ull << s.logN);
    *nblk_max = std::max<uint64_t>(*nblk_max, s.nblk);
    P.products += s.nmul;
    P.product_digits += s.limbs;
  };
  for (const Stage& s : P.pw) scratch(s, &P.res2_len, &P.F2_words, &P.nblk2_max);
  for (const auto& v : P.join)
    for (const Stage& s : v) scratch(s, &P.res_len, &P.F_words, &P.nblk_max);
  size_t off = o * 4;
  auto takeb = [&](size_t bytes) {
    const size_t r = off;
    off = align_up(off + bytes, 256);
    return r;
  };
  P.off_res = takeb(3 * (P.res_len + 64) * 4);
  P.off_F = takeb(P.F_words * 4);
  P.off_res2 = takeb(3 * (P.res2_len + 64) * 4);
  P.off_F2 = takeb(P.F2_words * 4);
  // control block: error word | top index (8 bytes) | character count (8
  // bytes) | look-back flags of the joins | those of the squarings
  P.ctl_words = 6 + (P.nblk_max + 1) + (P.nblk2_max + 1);
  P.off_ctl = takeb(P.ctl_words * 4);
  P.total = off;
  return CAT_OK;
}

// P_0 = 2^(32 DEC_LEAF_LIMBS) in radix 10^9, least significant digit first
void dec_p0(uint32_t* d) {
  uint32_t w[DEC_LEAF_LIMBS + 1] = {0};   // as 32-bit limbs, by long division
  w[DEC_LEAF_LIMBS] = 1;
  for (int k = 0; k < DEC_LEAF_DIGITS; k++) {
    uint64_t r = 0;
    for (int i = DEC_LEAF_LIMBS; i >= 0; i--) {
      const uint64_t cur = (r << 32) | w[i];
      w[i] = (uint32_t)(cur / DEC_B);
      r = cur % DEC_B;
    }
    d[k] = (uint32_t)r;
  }
}

extern "C" {

cat_status decimal_sizes(size_t n_limbs, size_t* max_chars, size_t* work_bytes) {
  if (!max_chars || !work_bytes) return CAT_EINVAL;
  DecPlan P;
  STCHK(make_dec_plan(n_limbs, &P));
  // decimal digits of a number below 2^(32 L)
  *max_chars = (size_t)((long double)n_limbs * 32.0L * 0.30102999566398119521L) + 2;
  *work_bytes = P.total;
  return CAT_OK;
}

// The whole conversion on X.st (squarings on the second stream): clear the
// control block, P_0, the leaves, the joins, the top group and the text.
// Control block: error word, top (words 2-3), character count (words 4-5),
// look-back flags from word 6.
cat_status dec_record(const DecPlan& P, Exec X, const uint32_t* d_x, uint64_t n_limbs, char* d_out, uint64_t cap) {
  const hipStream_t st = X.st;
  unsigned long long* top = (unsigned long long*)(X.err + 2);
  unsigned long long* nc = (unsigned long long*)(X.err + 4);
  hipLaunchKernelGGL(k_fill, dim3((uint32_t)std::min<uint64_t>((P.ctl_words + 255) / 256, 1024)), dim3(256), 0, st,
                     X.err, (uint64_t)P.ctl_words, 0u);
  LAUNCHCHK();
  const int h = (int)P.lv.size() - 1;
  if (h > 0) {
    DecWords p0;
    dec_p0(p0.w);
    hipLaunchKernelGGL(k_dec_p0, dim3(1), dim3(64), 0, st, p0, X.W + P.pbase);
    LAUNCHCHK();
  }
  if (!P.pw.empty()) {
    // P_1 .. P_{h-1} on the second stream (after the fill and P_0); event j-1 marks P_j
    Exec S = X;
    S.st = g.side_stream;
    S.res = (uint32_t*)((char*)X.W + P.off_res2);
    S.res_stride = P.res2_len + 64;
    S.F = (uint32_t*)((char*)X.W + P.off_F2);
    S.flags = X.flags + P.nblk_max + 1;
    S.crt_epoch = 0;
    HIPCHK(hipEventRecord(g.dec_ev[0], st));
    HIPCHK(hipStreamWaitEvent(S.st, g.dec_ev[0], 0));
    for (size_t k = 0; k < P.pw.size(); k++) {
      STCHK(run_stage_batched(S, P.pw[k]));
      HIPCHK(hipEventRecord(g.dec_ev[k], S.st));
    }
  }
  const uint64_t n0 = P.lv[0].nodes;
  hipLaunchKernelGGL(k_dec_leaf, dim3((uint32_t)((n0 + 255) / 256)), dim3(256), 0, st, d_x, (uint64_t)n_limbs,
                     X.W + P.x[0], n0);
  LAUNCHCHK();
  for (int j = 0; j < h; j++) {
    if (j >= 1) HIPCHK(hipStreamWaitEvent(st, g.dec_ev[j - 1], 0));
    for (const Stage& s : P.join[j]) STCHK(run_stage_batched(X, s));
    const DecLevel& c = P.lv[j];
    if (c.nodes & 1) {
      const DecLevel& nx = P.lv[j + 1];
      const uint32_t* in = X.W + P.x[j & 1] + (c.nodes - 1) * c.len;
      uint32_t* out = X.W + P.x[(j + 1) & 1] + (nx.nodes - 1) * nx.len;
      const uint32_t blocks = (uint32_t)std::min<uint64_t>((nx.len + 255) / 256, 1024);
      hipLaunchKernelGGL(k_copy_pad, dim3(blocks), dim3(256), 0, st, in, c.len, out, nx.len);
      LAUNCHCHK();
    }
  }
  const uint32_t* dig = X.W + P.x[h & 1];
  const uint64_t nd = P.lv[h].len;
  hipLaunchKernelGGL(k_top_nonzero, dim3((uint32_t)std::min<uint64_t>((nd + 255) / 256, 512)), dim3(256), 0, st, dig,
                     nd, top, (uint32_t*)nullptr, (uint64_t)0);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_dec_ascii, dim3((uint32_t)((nd + 255) / 256)), dim3(256), 0, st, dig,
                     (const unsigned long long*)top, d_out ? cap : (uint64_t)0, d_out, nc);
  LAUNCHCHK();
  return CAT_OK;
}

// replayable conversions, keyed by (limbs, input, output, capacity, workspace)
std::map<std::vector<uintptr_t>, hipGraphExec_t> g_dec_graphs;
#define DEC_GRAPHS_MAX 32

cat_status bigint_to_decimal(const uint32_t* d_x, size_t n_limbs, char* d_out, size_t cap, size_t* n_chars,
                             void* d_work, size_t work_bytes, void* stream) {
  if (!n_chars || !d_work || (n_limbs && !d_x)) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  DecPlan P;
  STCHK(make_dec_plan(n_limbs, &P));
  if (work_bytes < P.total) return CAT_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  char* wb = (char*)d_work;
  Exec X;
  X.W = (uint32_t*)wb;
  X.res = (uint32_t*)(wb + P.off_res);
  X.res_stride = P.res_len + 64;
  X.F = (uint32_t*)(wb + P.off_F);
  X.err = (uint32_t*)(wb + P.off_ctl);
  X.flags = X.err + 6;
  X.st = st;
  const int h = (int)P.lv.size() - 1;
  while (g.dec_ev.size() < (size_t)std::max(h, 1)) {
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    g.dec_ev.push_back(e);
  }
  // one graph per key, replayed; direct launches while the kernel timer watches
  if (g.timer_name.empty()) {
    const std::vector<uintptr_t> key{(uintptr_t)n_limbs, (uintptr_t)d_x, (uintptr_t)d_out, (uintptr_t)cap,
                                     (uintptr_t)wb};
    auto it = g_dec_graphs.find(key);
    hipGraphExec_t ge = nullptr;
    if (it != g_dec_graphs.end()) {
      ge = it->second;
    } else {
      if (g_dec_graphs.size() >= DEC_GRAPHS_MAX) {
        for (auto& kv : g_dec_graphs) (void)hipGraphExecDestroy(kv.second);
        g_dec_graphs.clear();
      }
      STCHK(capture_graph(
          [&](hipStream_t cs) -> cat_status {
            Exec C = X;
            C.st = cs;
            return dec_record(P, C, d_x, n_limbs, d_out, cap);
          },
          &ge));
      g_dec_graphs[key] = ge;
    }
    HIPCHK(hipGraphLaunch(ge, st));
  } else {
    STCHK(dec_record(P, X, d_x, n_limbs, d_out, cap));
  }
  HIPCHK(hipMemcpyAsync(g.pin, X.err, 24, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  uint32_t derr = 0;
  uint64_t nch = 0;
  memcpy(&derr, g.pin, 4);
  memcpy(&nch, (char*)g.pin + 16, 8);
  cat_stats stats{};
  stats.products = P.products;
  stats.product_limbs = P.product_digits;
  stats.levels = (uint32_t)h;
  g.stats = stats;
  if (derr) return CAT_EINTERNAL;
  *n_chars = (size_t)nch;
  if (!d_out || cap < nch) return CAT_ERANGE;
  return CAT_OK;
}

}  // extern "C"
