// Phase 1 of the method (Sec. 3.1, Alg. 1): all primes p <= 2n with their
// exponents e_p = v_p((2n)!) - 2 v_p(n!) - v_p(n+1) (Sec. 2), grouped by e.
//
// Device design (gfx950):
//  * k_seeds: one workgroup sieves the seed primes q <= s = isqrt(2n) in a
//    64 KB LDS byte map and computes their exponents with Legendre's sums.
//  * k_sieve: one workgroup per segment of SEG odd numbers in (s, 2n]; the
//    segment is a bit map in LDS (SEG/8 bytes), marked by the odd seeds
//    (cooperatively for small q, one thread per prime for large q).  For a
//    prime p > s we have p^2 > 2n, so Legendre's sums have one term and
//    v_p(n+1) <= 1; with r = n mod p the exponent is
//        e_p = [2r >= p] - [r == p-1]   (in {0, 1}).
//    Only primes with e_p = 1 stay in the bit map written to HBM; the
//    workgroup also writes its count.
//  * k_groups: one workgroup scans the segment counts, places the seeds in
//    their groups and writes the group table (exponent ascending).
//  * k_scatter: one workgroup per segment writes its primes in ascending
//    order to their final place inside G_1.
// Every group ends up with its primes ascending; G_1 = {seeds with e = 1}
// followed by the large primes with e = 1.

// Segments of 2^14 odd numbers (2 KB bit maps) by default; ranges of at
// least 2^10 segments of 2^16 (n above about 6.7e7) use 2^16, and ranges of
// at least 2^10 segments of 2^17 (n above about 1.3e8) use 2^17: the
// per-seed start computations of a segment are spread over 4 or 8 times the
// numbers.
#define SIEVE_SEG_LOG 14
#define SIEVE_SEG_LOG_BIG 16
#define SIEVE_SEG_LOG_HUGE 17
#define SIEVE_SEG (1u << SIEVE_SEG_LOG)        // odd numbers per segment (default)
#define SIEVE_WORDS (SIEVE_SEG / 32)
#define SIEVE_THREADS 256
#define SEED_MAX 6544                           // pi(65535) = 6542

struct GroupTable {
  uint32_t ngroups;
  uint32_t n_seed_e1;         // seeds with e = 1 (they open G_1)
  uint32_t nseeds;
  uint32_t err;
  uint32_t exps[CAT_MAX_GROUPS];
  uint64_t off[CAT_MAX_GROUPS + 1];
  // upper bound on the bit length of Q_g (sum of the bit lengths of its
  // primes; 32 per prime where not summed), which bounds the power chains
  uint64_t gbits[CAT_MAX_GROUPS];
};

// Exclusive scan over a block of up to 16 wave64s.  tmp: >= 40 words.
__device__ __forceinline__ uint32_t block_excl_scan_1024(uint32_t v, uint32_t* tmp, uint32_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (int)(blockDim.x >> 6);
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[wid] = x;
  __syncthreads();
  if (wid == 0) {
    uint32_t w = lane < nw ? tmp[lane] : 0;
    uint32_t t = w;
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
      uint32_t y = __shfl_up(t, d, 64);
      if (lane >= d) t += y;
    }
    if (lane < 16) tmp[16 + lane] = t - w;    // exclusive wave offsets
    if (lane == nw - 1) tmp[32] = t;
  }
  __syncthreads();
  uint32_t r = tmp[16 + wid] + x - v;
  if (total) *total = tmp[32];
  __syncthreads();
  return r;
}

// Legendre's sum v_p(m!) = sum_k floor(m / p^k) by repeated division; m < 2^32.
__device__ __forceinline__ uint32_t legendre_dev(uint32_t m, uint32_t p) {
  uint32_t s = 0;
  while (m) { m /= p; s += m; }
  return s;
}

// ---------------------------------------------------------------------------
// The primes q <= s (s < 2^16) in ascending order, by a workgroup of up to 1024
// threads sieving a byte map in LDS (comp: s+1 bytes); returns their count.
__device__ uint32_t build_seeds(uint32_t s, uint8_t* comp, uint32_t* tmp, uint32_t* small, uint32_t* nsmall,
                                uint32_t* seeds) {
  const uint32_t T = blockDim.x, tid = threadIdx.x;
  for (uint32_t i = tid; i <= s; i += T) comp[i] = (i < 2) ? 1 : 0;
  // primes up to isqrt(s) <= 255 by trial division, one thread per candidate
  uint32_t r = 0;
  while ((r + 1) * (r + 1) <= s) r++;
  if (tid == 0) *nsmall = 0;
  __syncthreads();
  if (tid >= 2 && tid <= r) {
    bool isq = true;
    for (uint32_t d = 2; d * d <= tid; d++)
      if (tid % d == 0) { isq = false; break; }
    if (isq) small[atomicAdd(nsmall, 1u)] = tid;
  }
  __syncthreads();
  for (uint32_t k = 0; k < *nsmall; k++) {
    const uint32_t q = small[k];
    for (uint32_t m = q * q + tid * q; m <= s; m += T * q) comp[m] = 1;
  }
  __syncthreads();
  // compaction, ascending: thread t owns numbers [t*chunk, (t+1)*chunk)
  const uint32_t chunk = (s + 1 + T - 1) / T;
  uint32_t lo = tid * chunk, hi = min(lo + chunk, s + 1);
  uint32_t cnt = 0;
  for (uint32_t i = lo; i < hi; i++) cnt += comp[i] ? 0 : 1;
  uint32_t total;
  uint32_t pos = block_excl_scan_1024(cnt, tmp, &total);
  for (uint32_t i = lo; i < hi; i++)
    if (!comp[i]) seeds[pos++] = i;
  return total;
}

// Bit map of the odd numbers 2i+1, i in [i_lo, i_lo + len), that no odd seed
// divides (seeds[0] = 2 is skipped; every seed q has q*q above the segment's
// composites it must strike, so what stays is prime).  bits: SIEVE_WORDS words.
template <int SL = SIEVE_SEG_LOG>
__device__ void mark_segment(uint32_t* bits, uint64_t i_lo, uint32_t len, const uint32_t* seeds, uint32_t nseeds) {
  constexpr uint32_t SEG = 1u << SL, WORDS = SEG / 32;
  constexpr int NPRE = 17;   // odd primes below 64
  __shared__ uint32_t pre_q[NPRE], pre_r[NPRE], pre_d[NPRE];
  __shared__ uint64_t pre_pat[NPRE];
  __shared__ uint32_t pre_n;
  const uint32_t T = blockDim.x, tid = threadIdx.x;
  // m_lo = 2 i_lo + 1 <= 2n + 1 < 2^32: the first odd multiple q t >= m_lo
  // (t >= q) comes from one 32-bit division (a 64-bit one is a long software
  // sequence on the GPU); the product q t may reach 2^32 and stays 64-bit
  const uint32_t m_lo = (uint32_t)(2 * i_lo + 1);
  auto first_index = [&](uint32_t q) -> uint64_t {
    uint32_t t = m_lo / q;
    if (t * q != m_lo) t++;   // ceil(m_lo / q); before the increment t q <= m_lo
    if (t < q) t = q;
    if (!(t & 1)) t++;
    return ((uint64_t)q * t - 1) / 2 - i_lo;
  };
  // Odd seeds q < 64 with q^2 <= m_lo (every odd multiple of q in the segment
  // is marked, at the positions idx, idx + q, ...) are cleared word by word
  // with a periodic bit pattern instead of one LDS atomic per multiple: word w
  // loses the bits r, r + q, ... < 32 with r = (idx - 32 w) mod q, i.e. the
  // pattern sum_k 2^(k q) shifted left by r.
  if (tid == 0) {
    uint32_t c = 0;
    for (uint32_t k = 1; k < nseeds && c < NPRE; k++) {
      const uint32_t q = seeds[k];
      if (q >= 64 || (uint64_t)q * q > m_lo) break;
      pre_q[c++] = q;
    }
    pre_n = c;
  }
  __syncthreads();
  const uint32_t npre = pre_n;
  if (tid < npre) {
    const uint32_t q = pre_q[tid];
    pre_r[tid] = (uint32_t)(first_index(q) % q);
    pre_d[tid] = (32u * T) % q;   // the step of r between a thread's words
    uint64_t pat = 0;
    for (uint32_t b = 0; b < 64; b += q) pat |= 1ull << b;
    pre_pat[tid] = pat;
  }
  __syncthreads();
  uint32_t rr[NPRE];
#pragma unroll
  for (int j = 0; j < NPRE; j++) {
    if (j < (int)npre) {
      const uint32_t q = pre_q[j];
      const uint32_t s0 = (32u * tid) % q;
      rr[j] = pre_r[j] >= s0 ? pre_r[j] - s0 : pre_r[j] + q - s0;
    }
  }
  for (uint32_t w = tid; w < WORDS; w += T) {
    uint32_t b0 = w * 32;
    uint32_t v = 0;
    if (b0 + 32 <= len) v = 0xFFFFFFFFu;
    else if (b0 < len) v = (1u << (len - b0)) - 1u;
#pragma unroll
    for (int j = 0; j < NPRE; j++) {
      if (j < (int)npre) {
        v &= ~(uint32_t)(pre_pat[j] << rr[j]);
        const uint32_t q = pre_q[j], d = pre_d[j];
        rr[j] = rr[j] >= d ? rr[j] - d : rr[j] + q - d;
      }
    }
    bits[w] = v;
  }
  __syncthreads();
  // small odd seeds: every thread marks a share of the multiples of q
  uint32_t k = 1 + npre;
  for (; k < nseeds; k++) {
    const uint32_t q = seeds[k];
    if ((uint64_t)q * SIEVE_THREADS > 2 * SEG) break;   // fewer multiples than 2 per thread
    const uint64_t idx = first_index(q);
    for (uint64_t x = idx + (uint64_t)tid * q; x < len; x += (uint64_t)T * q)
      atomicAnd(&bits[x >> 5], ~(1u << (x & 31)));
  }
  // large seeds: one thread per prime
  for (uint32_t kk = k + tid; kk < nseeds; kk += T) {
    const uint32_t q = seeds[kk];
    const uint64_t idx = first_index(q);
    for (uint64_t x = idx; x < len; x += q)
      atomicAnd(&bits[x >> 5], ~(1u << (x & 31)));
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// ctl: the call's control block (group table first), ctl_words words, cleared
// here before anything else of the call writes to it.
__global__ void __launch_bounds__(1024) k_seeds(uint64_t n, uint32_t s, uint32_t* seeds, int32_t* seed_e,
                                                GroupTable* gt, uint32_t* __restrict__ ctl, uint64_t ctl_words) {
  __shared__ uint8_t comp[65536];
  __shared__ uint32_t tmp[40];
  __shared__ uint32_t small[64];
  __shared__ uint32_t nsmall;
  const uint32_t T = blockDim.x, tid = threadIdx.x;
  for (uint64_t k = tid; k < ctl_words; k += T) ctl[k] = 0u;
  __threadfence_block();
  const uint32_t total = build_seeds(s, comp, tmp, small, &nsmall, seeds);
  if (tid == 0) gt->nseeds = total;
  __syncthreads();
  __threadfence_block();
  // exponents by Legendre's sums; 2n < 2^32 and n + 1 < 2^32
  const uint32_t n2 = (uint32_t)(2 * n), n1 = (uint32_t)n, np1 = (uint32_t)(n + 1);
  for (uint32_t k = tid; k < total; k += T) {
    const uint32_t q = seeds[k];
    const int32_t a = (int32_t)legendre_dev(n2, q);
    const int32_t b = (int32_t)legendre_dev(n1, q);
    uint32_t m = np1;
    int32_t c = 0;
    while (m % q == 0) { m /= q; c++; }
    const int32_t e = a - 2 * b - c;
    if (e < 0) atomicOr(&gt->err, CAT_DEVERR_NEG_EXP);
    seed_e[k] = e;
  }
}

// ---------------------------------------------------------------------------
// Segment k covers odd indices i in [i0 + k*SEG, min(i0 + (k+1)*SEG, i_end)),
// i.e. odd numbers m = 2i+1 in (s, 2n].
template <int SL>
__global__ void __launch_bounds__(SIEVE_THREADS) k_sieve(uint64_t n, uint64_t i0, uint64_t i_end,
                                                const uint32_t* seeds, const GroupTable* gt,
                                                uint32_t* bitmap, uint32_t* seg_cnt) {
  constexpr uint32_t SEG = 1u << SL, WORDS = SEG / 32;
  __shared__ uint32_t bits[WORDS];
  __shared__ uint32_t tmp[40];
  const uint32_t T = blockDim.x, tid = threadIdx.x;
  const uint64_t i_lo = i0 + (uint64_t)blockIdx.x * SEG;
  const uint64_t i_hi = min(i_lo + SEG, i_end);
  const uint32_t len = (uint32_t)(i_hi - i_lo);
  mark_segment<SL>(bits, i_lo, len, seeds, gt->nseeds);
  // keep primes with e_p = 1, count them
  uint32_t cnt = 0;
  const uint32_t n32 = (uint32_t)n;   // n < 2^31
  for (uint32_t w = tid; w < WORDS; w += T) {
    uint32_t v = bits[w], keep = 0;
    while (v) {
      uint32_t b = __ffs(v) - 1;
      v &= v - 1;
      uint32_t p = (uint32_t)(2 * (i_lo + w * 32 + b) + 1);
      uint32_t r = n32 % p;
      uint32_t e = ((uint64_t)2 * r >= p ? 1u : 0u) - (r == p - 1 ? 1u : 0u);
      if (e == 1) keep |= 1u << b;
    }
    bitmap[(uint64_t)blockIdx.x * WORDS + w] = keep;
    cnt += __popc(keep);
  }
  uint32_t total;
  block_excl_scan_1024(cnt, tmp, &total);
  if (tid == 0) seg_cnt[blockIdx.x] = total;
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_groups(uint32_t nseg, const uint32_t* seg_cnt, uint32_t* seg_off,
                                                 const uint32_t* seeds, const int32_t* seed_e,
                                                 uint32_t* primes, uint64_t cap, GroupTable* gt) {
  __shared__ uint32_t tmp[40];
  __shared__ uint32_t cnt_e[CAT_MAX_GROUPS + 1];
  __shared__ unsigned long long bits_e[CAT_MAX_GROUPS + 1];
  __shared__ uint64_t goff[CAT_MAX_GROUPS + 2];
  const uint32_t T = blockDim.x, tid = threadIdx.x;
  // the thread's seeds (a contiguous chunk, ascending) and their exponents,
  // loaded once, with the segment counts below, all in flight
  constexpr int SCH = (SEED_MAX + 1023) / 1024;
  const uint32_t ns = gt->nseeds;
  const uint32_t sch = (ns + T - 1) / T;   // <= SCH
  const uint32_t slo = min(tid * sch, ns), shi = min(slo + sch, ns);
  uint32_t sd[SCH];
  int32_t se[SCH];
#pragma unroll
  for (int i = 0; i < SCH; i++) {
    const uint32_t k = slo + i < shi ? slo + i : 0;
    sd[i] = seeds[k];
    se[i] = slo + i < shi ? seed_e[k] : 0;
  }
  // 1. exclusive scan of the segment counts
  const uint32_t chunk = (nseg + T - 1) / T;
  uint32_t lo = min(tid * chunk, nseg), hi = min(lo + chunk, nseg);
  uint32_t c = 0;
  for (uint32_t i = lo; i < hi; i++) c += seg_cnt[i];
  uint32_t total_large;
  uint32_t pos = block_excl_scan_1024(c, tmp, &total_large);
  for (uint32_t i = lo; i < hi; i++) { seg_off[i] = pos; pos += seg_cnt[i]; }
  // 2. seed counts per exponent
  if (tid <= CAT_MAX_GROUPS) {
    cnt_e[tid] = 0;
    bits_e[tid] = 0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < SCH; i++) {
    const int32_t e = se[i];
    if (e > 0 && e <= CAT_MAX_GROUPS) {
      atomicAdd(&cnt_e[e], 1u);
      atomicAdd(&bits_e[e], (unsigned long long)(32 - __clz(sd[i])));
    }
  }
  __syncthreads();
  // 3. group table (exponent ascending, empty groups dropped)
  if (tid == 0) {
    uint32_t g = 0;
    uint64_t o = 0;
    for (uint32_t e = 1; e <= CAT_MAX_GROUPS; e++) {
      uint64_t cnt = cnt_e[e] + (e == 1 ? (uint64_t)total_large : 0);
      goff[e] = o;
      if (cnt == 0) continue;
      gt->exps[g] = e;
      gt->off[g] = o;
      // G_1 holds the large primes: no tighter bound is needed for it
      gt->gbits[g] = e == 1 ? 32 * cnt : (uint64_t)bits_e[e];
      o += cnt;
      g++;
    }
    gt->off[g] = o;
    gt->ngroups = g;
    gt->n_seed_e1 = cnt_e[1];
    if (o > cap) atomicOr(&gt->err, CAT_DEVERR_BOUNDS);
    goff[0] = o;  // total
  }
  __syncthreads();
  // 4. seeds into their groups, stable (seeds ascending)
  for (uint32_t e = 1; e <= CAT_MAX_GROUPS; e++) {
    if (cnt_e[e] == 0) continue;   // uniform
    uint32_t cc = 0;
#pragma unroll
    for (int i = 0; i < SCH; i++) cc += (se[i] == (int32_t)e);
    uint32_t r = block_excl_scan_1024(cc, tmp, nullptr);
    const uint64_t base = goff[e];
#pragma unroll
    for (int i = 0; i < SCH; i++)
      if (se[i] == (int32_t)e) {
        const uint64_t at = base + r++;
        if (at < cap) primes[at] = sd[i];
      }
  }
}

// ---------------------------------------------------------------------------
template <int SL>
__global__ void __launch_bounds__(SIEVE_THREADS) k_scatter(uint64_t i0, const uint32_t* bitmap, const uint32_t* seg_off,
                                                  const GroupTable* gt, uint32_t* primes, uint64_t cap) {
  __shared__ uint32_t tmp[40];
  const uint32_t tid = threadIdx.x;
  constexpr uint32_t SEG = 1u << SL, WORDS = SEG / 32;
  constexpr uint32_t WPT = WORDS / SIEVE_THREADS;   // words per thread
  const uint64_t i_lo = i0 + (uint64_t)blockIdx.x * SEG;
  const uint32_t* bm = bitmap + (uint64_t)blockIdx.x * WORDS;
  uint32_t w[WPT];
  uint32_t c = 0;
#pragma unroll
  for (uint32_t k = 0; k < WPT; k++) { w[k] = bm[tid * WPT + k]; c += __popc(w[k]); }
  uint32_t total;
  uint32_t r = block_excl_scan_1024(c, tmp, &total);
  const uint64_t base = (uint64_t)gt->n_seed_e1 + seg_off[blockIdx.x];
  // primes of a segment staged in LDS: 32 KB, 64 KB for segments of 2^17
  // (about 12,000 primes near 4e9)
  constexpr uint32_t STAGE = SL >= SIEVE_SEG_LOG_HUGE ? 16384 : 8192;
  if (total <= STAGE) {
    // the segment's primes are one contiguous run: staged in LDS in order,
    // then written by consecutive threads to consecutive words
    __shared__ uint32_t stage[STAGE];
#pragma unroll
    for (uint32_t k = 0; k < WPT; k++) {
      uint32_t v = w[k];
      while (v) {
        uint32_t b = __ffs(v) - 1;
        v &= v - 1;
        stage[r++] = (uint32_t)(2 * (i_lo + (tid * WPT + k) * 32 + b) + 1);
      }
    }
    __syncthreads();
    for (uint32_t j = tid; j < total; j += SIEVE_THREADS)
      if (base + j < cap) primes[base + j] = stage[j];
    return;
  }
  uint64_t at = base + r;
#pragma unroll
  for (uint32_t k = 0; k < WPT; k++) {
    uint32_t v = w[k];
    while (v) {
      uint32_t b = __ffs(v) - 1;
      v &= v - 1;
      if (at < cap) primes[at] = (uint32_t)(2 * (i_lo + (tid * WPT + k) * 32 + b) + 1);
      at++;
    }
  }
}
