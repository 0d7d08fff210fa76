// Factorial ratios N = prod_i a_i! / prod_j b_j! (Sec. 6.3): Phase 1 with the
// extended Legendre formula v_p(N) = sum_i v_p(a_i!) - sum_j v_p(b_j!) for every
// prime p <= A = max(a_i, b_j), then the Phase-2 reconstruction unchanged.
//
// Grouping.  Alg. 2 groups primes by their exponent value; a ratio can have
// far more distinct exponents than that table holds (v_p(n!) takes about
// 2 sqrt(n) values), so the primes are grouped by the bits of their exponents
// instead: group b holds, ascending, every prime whose exponent has bit b set
// and carries the exponent 2^b, so N = prod_b Q_b^(2^b) with at most 32 groups
// and the same product trees, power chains and outer product.
//
//  * k_rseeds: seeds q <= sqrt(A) (LDS byte map) and their exponents; also
//    clears the call's control block and the ratio counters.
//  * k_rsieve: one workgroup per segment of odd numbers in (sqrt(A), A]: bit
//    map of the primes with v_p(N) > 0 (a single division per argument, since
//    p^2 > A), and their count.
//  * k_rscan: exclusive scan of the segment counts; seeds with v_p(N) > 0 go
//    first.  k_rscatter: every prime and its exponent, ascending, into P / E.
//  * k_rbits: per chunk of 4096 entries, per bit: entries with the bit set and
//    the sum of their primes' bit lengths.  k_rbitscan: per bit, the chunk
//    offsets.  k_rtable: the group table.  k_rbitscatter: the grouped primes.

#define RATIO_MAX_TERMS 32
#define RATIO_CHUNK 4096u   // entries per workgroup of the bit-grouping kernels

struct RatioTerms {
  uint32_t k, m;                    // numerator / denominator argument counts
  uint32_t a[RATIO_MAX_TERMS];
  uint32_t b[RATIO_MAX_TERMS];
};

// Counters of one call (zeroed by k_rseeds)
struct RatioCounts {
  uint32_t np;                              // primes with v_p(N) > 0
  uint32_t pad;
  unsigned long long tot[32];               // entries per exponent bit
  unsigned long long bits[32];              // sum of bit lengths per exponent bit
};

// v_p(N), Legendre's sums by repeated division (every argument < 2^32)
__device__ __forceinline__ int64_t ratio_exp(const RatioTerms& rt, uint32_t p) {
  int64_t e = 0;
  for (uint32_t i = 0; i < rt.k; i++) e += legendre_dev(rt.a[i], p);
  for (uint32_t j = 0; j < rt.m; j++) e -= legendre_dev(rt.b[j], p);
  return e;
}

__global__ void __launch_bounds__(1024) k_rseeds(RatioTerms rt, uint32_t s, uint32_t* seeds, uint32_t* seed_e,
                                                 GroupTable* gt, uint32_t* __restrict__ ctl, uint64_t ctl_words,
                                                 RatioCounts* rc) {
  __shared__ uint8_t comp[65536];
  __shared__ uint32_t tmp[40];
  __shared__ uint32_t small[64];
  __shared__ uint32_t nsmall;
  const uint32_t T = blockDim.x, tid = threadIdx.x;
  for (uint64_t k = tid; k < ctl_words; k += T) ctl[k] = 0u;
  for (uint32_t k = tid; k < sizeof(RatioCounts) / 4; k += T) ((uint32_t*)rc)[k] = 0u;
  const uint32_t total = build_seeds(s, comp, tmp, small, &nsmall, seeds);
  if (tid == 0) gt->nseeds = total;
  for (uint32_t k = tid; k < total; k += T) {
    const int64_t e = ratio_exp(rt, seeds[k]);
    if (e < 0) atomicOr(&gt->err, CAT_DEVERR_NEG_EXP);
    if (e >= (1ll << 32)) atomicOr(&gt->err, CAT_DEVERR_RANGE);
    seed_e[k] = e > 0 && e < (1ll << 32) ? (uint32_t)e : 0u;
  }
}

// odd m = 2i+1 for i in [i0 + k*SEG, min(i0 + (k+1)*SEG, i_end)): primes in (s, A]
__global__ void __launch_bounds__(SIEVE_THREADS) k_rsieve(RatioTerms rt, uint64_t i0, uint64_t i_end,
                                                 const uint32_t* seeds, GroupTable* gt, uint32_t* bitmap,
                                                 uint32_t* seg_cnt) {
  __shared__ uint32_t bits[SIEVE_WORDS];
  __shared__ uint32_t tmp[40];
  const uint32_t T = blockDim.x, tid = threadIdx.x;
  const uint64_t i_lo = i0 + (uint64_t)blockIdx.x * SIEVE_SEG;
  const uint64_t i_hi = min(i_lo + SIEVE_SEG, i_end);
  const uint32_t len = (uint32_t)(i_hi - i_lo);
  mark_segment(bits, i_lo, len, seeds, gt->nseeds);
  uint32_t cnt = 0, err = 0;
  for (uint32_t w = tid; w < SIEVE_WORDS; w += T) {
    uint32_t v = bits[w], keep = 0;
    while (v) {
      const uint32_t b = __ffs(v) - 1;
      v &= v - 1;
      const uint32_t p = (uint32_t)(2 * (i_lo + w * 32 + b) + 1);
      const int64_t e = ratio_exp(rt, p);
      if (e < 0) err |= CAT_DEVERR_NEG_EXP;
      if (e >= (1ll << 32)) err |= CAT_DEVERR_RANGE;
      if (e > 0) keep |= 1u << b;
    }
    bitmap[(uint64_t)blockIdx.x * SIEVE_WORDS + w] = keep;
    cnt += __popc(keep);
  }
  if (err) atomicOr(&gt->err, err);
  uint32_t total;
  block_excl_scan_1024(cnt, tmp, &total);
  if (tid == 0) seg_cnt[blockIdx.x] = total;
}

// Segment offsets (after the seeds with v_p(N) > 0, which go first); P / E
// receive those seeds.  cap: capacity of P and E.
__global__ void __launch_bounds__(1024) k_rscan(uint32_t nseg, const uint32_t* seg_cnt, uint32_t* seg_off,
                                                const uint32_t* seeds, const uint32_t* seed_e, GroupTable* gt,
                                                uint32_t* P, uint32_t* E, uint64_t cap, RatioCounts* rc) {
  __shared__ uint32_t tmp[40];
  const uint32_t T = blockDim.x, tid = threadIdx.x;
  const uint32_t chunk = (nseg + T - 1) / T;
  const uint32_t lo = min(tid * chunk, nseg), hi = min(lo + chunk, nseg);
  uint32_t c = 0;
  for (uint32_t i = lo; i < hi; i++) c += seg_cnt[i];
  uint32_t total_large;
  uint32_t pos = block_excl_scan_1024(c, tmp, &total_large);
  for (uint32_t i = lo; i < hi; i++) { seg_off[i] = pos; pos += seg_cnt[i]; }
  // seeds with a positive exponent, ascending
  const uint32_t ns = gt->nseeds;
  const uint32_t sch = (ns + T - 1) / T;
  const uint32_t slo = min(tid * sch, ns), shi = min(slo + sch, ns);
  uint32_t cc = 0;
  for (uint32_t k = slo; k < shi; k++) cc += seed_e[k] > 0;
  uint32_t nse;
  uint32_t r = block_excl_scan_1024(cc, tmp, &nse);
  for (uint32_t k = slo; k < shi; k++)
    if (seed_e[k] > 0) {
      if (r < cap) {
        P[r] = seeds[k];
        E[r] = seed_e[k];
      }
      r++;
    }
  if (tid == 0) {
    gt->n_seed_e1 = nse;
    rc->np = nse + total_large;
    if ((uint64_t)nse + total_large > cap) atomicOr(&gt->err, CAT_DEVERR_BOUNDS);
  }
}

__global__ void __launch_bounds__(SIEVE_THREADS) k_rscatter(RatioTerms rt, uint64_t i0, const uint32_t* bitmap,
                                                   const uint32_t* seg_off, const GroupTable* gt, uint32_t* P,
                                                   uint32_t* E, uint64_t cap) {
  __shared__ uint32_t tmp[40];
  const uint32_t tid = threadIdx.x;
  constexpr uint32_t WPT = SIEVE_WORDS / SIEVE_THREADS;   // words per thread
  const uint64_t i_lo = i0 + (uint64_t)blockIdx.x * SIEVE_SEG;
  const uint32_t* bm = bitmap + (uint64_t)blockIdx.x * SIEVE_WORDS;
  uint32_t w[WPT];
  uint32_t c = 0;
#pragma unroll
  for (uint32_t k = 0; k < WPT; k++) {
    w[k] = bm[tid * WPT + k];
    c += __popc(w[k]);
  }
  const uint32_t r = block_excl_scan_1024(c, tmp, nullptr);
  uint64_t at = (uint64_t)gt->n_seed_e1 + seg_off[blockIdx.x] + r;
#pragma unroll
  for (uint32_t k = 0; k < WPT; k++) {
    uint32_t v = w[k];
    while (v) {
      const uint32_t b = __ffs(v) - 1;
      v &= v - 1;
      const uint32_t p = (uint32_t)(2 * (i_lo + (tid * WPT + k) * 32 + b) + 1);
      if (at < cap) {
        P[at] = p;
        E[at] = (uint32_t)ratio_exp(rt, p);
      }
      at++;
    }
  }
}

// Entry range of chunk c, each thread owning 16 consecutive entries.
__global__ void __launch_bounds__(256) k_rbits(const uint32_t* P, const uint32_t* E, const RatioCounts* rcin,
                                               uint32_t* chunk_cnt, RatioCounts* rc) {
  __shared__ uint32_t cnt[32];
  __shared__ uint32_t bsum[32];
  const uint32_t tid = threadIdx.x;
  if (tid < 32) {
    cnt[tid] = 0;
    bsum[tid] = 0;
  }
  __syncthreads();
  const uint64_t np = rcin->np;
  const uint64_t base = (uint64_t)blockIdx.x * RATIO_CHUNK + 16ull * tid;
  uint32_t mask[32] = {};   // per bit: which of the thread's entries have it
  uint32_t blen[16];
#pragma unroll
  for (int i = 0; i < 16; i++) {
    const uint64_t at = base + i;
    const uint32_t e = at < np ? E[at] : 0u;
    blen[i] = at < np ? 32 - __clz(P[at]) : 0u;
#pragma unroll
    for (int b = 0; b < 32; b++) mask[b] |= ((e >> b) & 1u) << i;
  }
#pragma unroll
  for (int b = 0; b < 32; b++) {
    if (mask[b]) {
      uint32_t bl = 0;
#pragma unroll
      for (int i = 0; i < 16; i++) bl += ((mask[b] >> i) & 1u) ? blen[i] : 0u;
      atomicAdd(&cnt[b], (uint32_t)__popc(mask[b]));
      atomicAdd(&bsum[b], bl);
    }
  }
  __syncthreads();
  if (tid < 32) {
    chunk_cnt[(uint64_t)blockIdx.x * 32 + tid] = cnt[tid];
    if (cnt[tid]) {
      atomicAdd(&rc->tot[tid], (unsigned long long)cnt[tid]);
      atomicAdd(&rc->bits[tid], (unsigned long long)bsum[tid]);
    }
  }
}

// per bit (one workgroup each): exclusive scan of the chunk counts
__global__ void __launch_bounds__(1024) k_rbitscan(uint32_t nchunks, const uint32_t* chunk_cnt, uint32_t* chunk_off) {
  __shared__ uint32_t tmp[40];
  const uint32_t b = blockIdx.x, T = blockDim.x, tid = threadIdx.x;
  const uint32_t chunk = (nchunks + T - 1) / T;
  const uint32_t lo = min(tid * chunk, nchunks), hi = min(lo + chunk, nchunks);
  uint32_t c = 0;
  for (uint32_t i = lo; i < hi; i++) c += chunk_cnt[(uint64_t)i * 32 + b];
  uint32_t pos = block_excl_scan_1024(c, tmp, nullptr);
  for (uint32_t i = lo; i < hi; i++) {
    chunk_off[(uint64_t)i * 32 + b] = pos;
    pos += chunk_cnt[(uint64_t)i * 32 + b];
  }
}

// group table: one group per exponent bit that occurs, bit ascending
__global__ void k_rtable(const RatioCounts* rc, GroupTable* gt, uint64_t cap) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t g = 0;
  uint64_t o = 0;
  for (uint32_t b = 0; b < 32; b++) {
    if (rc->tot[b] == 0) continue;
    gt->exps[g] = 1u << b;
    gt->off[g] = o;
    gt->gbits[g] = rc->bits[b];
    o += rc->tot[b];
    g++;
  }
  gt->off[g] = o;
  gt->ngroups = g;
  if (o > cap) atomicOr(&gt->err, CAT_DEVERR_BOUNDS);
}

// grouped primes: chunk c writes, per group, its entries with the group's bit
__global__ void __launch_bounds__(256) k_rbitscatter(const uint32_t* P, const uint32_t* E, const RatioCounts* rc,
                                                     const uint32_t* chunk_off, const GroupTable* gt, uint32_t* out,
                                                     uint64_t cap) {
  __shared__ uint32_t tmp[40];
  const uint32_t tid = threadIdx.x;
  const uint64_t np = rc->np;
  const uint64_t base = (uint64_t)blockIdx.x * RATIO_CHUNK + 16ull * tid;
  uint32_t pv[16], ev[16];
#pragma unroll
  for (int i = 0; i < 16; i++) {
    const uint64_t at = base + i;
    pv[i] = at < np ? P[at] : 0u;
    ev[i] = at < np ? E[at] : 0u;
  }
  const uint32_t ng = gt->ngroups;
  for (uint32_t g = 0; g < ng; g++) {
    const uint32_t b = 31 - __clz(gt->exps[g]);
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < 16; i++) c += (ev[i] >> b) & 1u;
    uint32_t r = block_excl_scan_1024(c, tmp, nullptr);
    uint64_t at = gt->off[g] + chunk_off[(uint64_t)blockIdx.x * 32 + b] + r;
#pragma unroll
    for (int i = 0; i < 16; i++)
      if ((ev[i] >> b) & 1u) {
        if (at < cap) out[at] = pv[i];
        at++;
      }
  }
}
