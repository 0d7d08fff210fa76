// Radix conversion to decimal (the optional decimal text output of Sec. 3.2):
// device kernels.  The integer is converted bottom-up in radix B = 10^9:
// leaves of sixteen 32-bit limbs become eighteen radix-B digits, and each level
// joins two neighbours as hi * 2^(512 * 2^j) + lo, where the power of two is
// itself held in radix B.  The product is the NTT product of the library with a
// radix-B carry step that also adds lo.
#define DEC_B 1000000000u
#define DEC_LEAF_LIMBS 16
#define DEC_LEAF_DIGITS 18         // 2^512 < 10^162
// digits per thread of the radix-B carry step (>= 4: a thread's first sum
// reaches four positions back), threads and digits per workgroup (128
// threads: its look-back recomputes a neighbour block half the size of the
// binary CRT's, 7-18 % less time than 256 threads, 512 was slower still)
#define DEC_CRT_E 4
#define DEC_CRT_THREADS 128
#define DEC_CRT_BLOCK (DEC_CRT_E * DEC_CRT_THREADS)

// floor((r * 2^32 + w) / 10^9) and its remainder, for r < 10^9 (so the
// quotient fits 32 bits): two-by-one division with a precomputed reciprocal
// of the normalised divisor d = 4 * 10^9 (Moller and Granlund, "Improved
// division by invariant integers", IEEE TC 2011, Algorithm 4).
#define DEC_D 4000000000u
#define DEC_V ((uint32_t)(0xFFFFFFFFFFFFFFFFull / DEC_D - (1ull << 32)))
__device__ __forceinline__ uint32_t div_b(uint32_t r, uint32_t w, uint32_t* rem) {
  const uint32_t u1 = (r << 2) | (w >> 30), u0 = w << 2;
  const uint64_t q = (uint64_t)DEC_V * u1 + ((((uint64_t)u1 + 1) << 32) | u0);
  uint32_t q1 = (uint32_t)(q >> 32);
  const uint32_t q0 = (uint32_t)q;
  uint32_t rr = u0 - q1 * DEC_D;
  if (rr > q0) {
    q1--;
    rr += DEC_D;
  }
  if (rr >= DEC_D) {
    q1++;
    rr -= DEC_D;
  }
  *rem = rr >> 2;
  return q1;
}

// Column value V = conv + addend (< 2^96) split into radix-B components
// V = c0 + c1 B + c2 B^2 + c3 B^3 (c3 < 80).
__device__ __forceinline__ void dec_split(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t add, uint32_t* c) {
  uint32_t v0, v1, v2;
  garner3(r0, r1, r2, v0, v1, v2);
  const uint64_t lo = ((uint64_t)v1 << 32 | v0) + add;
  if (lo < add) v2++;
  v0 = (uint32_t)lo;
  v1 = (uint32_t)(lo >> 32);
  uint32_t r;
  const uint32_t q2 = div_b(0, v2, &r);
  const uint32_t q1 = div_b(r, v1, &r);
  const uint32_t q0 = div_b(r, v0, &r);
  c[0] = r;
  // (q2, q1, q0) = floor(V / B) < 2^96 / B < 2^67, so q2 < 8 < B: the
  // division of the top word is q2 = 0 B + q2
  r = q2;
  const uint32_t p1 = div_b(r, q1, &r);
  const uint32_t p0 = div_b(r, q0, &r);
  c[1] = r;
  // (p1, p0) < 2^67 / B < 2^38, so p1 < 2^6 < B likewise
  r = p1;
  const uint32_t s0 = div_b(r, p0, &r);
  c[2] = r;
  c[3] = s0;
}


// Radix-B digit k of a segment: s_k = c0(k) + c1(k-1) + c2(k-2) + c3(k-3) <
// 3B + 80, so s_k = x_k + B y_k with y_k <= 3, u_k = x_k + y_{k-1} <= B + 2 and
// the carries left are binary: generate u_k >= B, propagate u_k = B - 1.
// Thread positions k0 .. k0+E-1; the four components of the positions
// k0-4 .. k0-1 that enter these sums (10 words) come from the left neighbour
// (thread 0: recomputed from the residues by the first DEC_CTX lanes, one
// position kb-DEC_CTX+l each).  As in the binary carry step, the u of those
// positions decide the carry into the block unless all of them propagate:
// *spec gets that carry, or 2 when undecided.
#define DEC_XV 10
#define DEC_CTX 16
__device__ __forceinline__ void crt_local10(const CrtSeg& sg, const uint32_t* __restrict__ r0,
                                            const uint32_t* __restrict__ r1, const uint32_t* __restrict__ r2,
                                            const uint32_t* __restrict__ add, uint64_t kb, uint32_t (*xv)[DEC_XV],
                                            uint32_t* tmp, uint64_t* u, bool* Gt, bool* Pt, uint32_t* spec) {
  const uint32_t tid = threadIdx.x;
  const uint64_t k0 = kb + (uint64_t)tid * DEC_CRT_E;
  // c[i][.] for positions k0-4+i (i < 4 from the neighbour, own from i = 4)
  uint32_t c[DEC_CRT_E + 4][4];
  // the first DEC_CTX lanes also fetch the block's left context
  // kb-DEC_CTX .. kb-1, one position each, with their own loads
  const int64_t kl = (int64_t)kb - DEC_CTX + (int64_t)tid;
  const bool lctx = tid < DEC_CTX && kl >= 0 && (uint64_t)kl < sg.len;
  uint32_t y0 = 0, y1 = 0, y2 = 0, ya = 0;
  {
    uint32_t x0[DEC_CRT_E], x1[DEC_CRT_E], x2[DEC_CRT_E], xa[DEC_CRT_E];
#pragma unroll
    for (int i = 0; i < DEC_CRT_E; i++) {
      const uint64_t k = k0 + i;
      const uint64_t kc = k < sg.len ? k : 0;
      x0[i] = r0[kc];
      x1[i] = r1[kc];
      x2[i] = r2[kc];
      xa[i] = add[sg.add_pos + (k < sg.add_len ? k : 0)];
    }
    if (tid < DEC_CTX) {
      const uint64_t kc = lctx ? (uint64_t)kl : 0;
      y0 = r0[kc];
      y1 = r1[kc];
      y2 = r2[kc];
      ya = add[sg.add_pos + (kc < sg.add_len ? kc : 0)];
    }
#pragma unroll
    for (int i = 0; i < DEC_CRT_E; i++) {
      const uint64_t k = k0 + i;
      if (k < sg.len) {
        dec_split(x0[i], x1[i], x2[i], k < sg.add_len ? xa[i] : 0u, c[i + 4]);
      } else {
        c[i + 4][0] = c[i + 4][1] = c[i + 4][2] = c[i + 4][3] = 0;
      }
    }
  }
  __syncthreads();   // xv may still be read by a previous call
  {
    uint32_t* o = xv[tid + 1];
    const int e = DEC_CRT_E;
    o[0] = c[e + 3][0]; o[1] = c[e + 3][1]; o[2] = c[e + 3][2]; o[3] = c[e + 3][3];
    o[4] = c[e + 2][1]; o[5] = c[e + 2][2]; o[6] = c[e + 2][3];
    o[7] = c[e + 1][2]; o[8] = c[e + 1][3];
    o[9] = c[e][3];
  }
  if (tid < 64) {
    // lane l < DEC_CTX recomputes position kb-DEC_CTX+l (zero outside the
    // segment); the last lane gathers the block's context, and the u of the
    // lanes from 4 on decide the carry in when one of them does not propagate
    uint32_t q[4] = {0, 0, 0, 0};
    if (lctx) dec_split(y0, y1, y2, (uint64_t)kl < sg.add_len ? ya : 0u, q);
    const uint32_t q1a = __shfl_up(q[1], 1, 64), q2a = __shfl_up(q[2], 1, 64), q3a = __shfl_up(q[3], 1, 64);
    const uint32_t q2b = __shfl_up(q[2], 2, 64), q3b = __shfl_up(q[3], 2, 64), q3c = __shfl_up(q[3], 3, 64);
    const uint32_t sl = q[0] + q1a + q2b + q3c;   // digit sum of the lane's position (lanes >= 3)
    const uint32_t yl = (sl >= DEC_B) + (sl >= 2 * DEC_B) + (sl >= 3 * DEC_B);
    const uint32_t yp = __shfl_up(yl, 1, 64);
    const uint32_t ul = sl - yl * DEC_B + yp;     // u of the lane's position (lanes >= 4)
    const bool valid = tid >= 4 && tid < DEC_CTX;
    const uint64_t gm = __ballot(valid && ul >= DEC_B);
    const uint64_t dm = gm | __ballot(valid && ul < DEC_B - 1);
    if (tid == 0) *spec = dm ? (uint32_t)((gm >> (63 - __builtin_clzll(dm))) & 1ull) : 2u;
    if (tid == DEC_CTX - 1) {
      uint32_t* o = xv[0];
      o[0] = q[0]; o[1] = q[1]; o[2] = q[2]; o[3] = q[3];
      o[4] = q1a; o[5] = q2a; o[6] = q3a;
      o[7] = q2b; o[8] = q3b;
      o[9] = q3c;
    }
  }
  __syncthreads();
  {
    const uint32_t* o = xv[tid];
    c[3][0] = o[0]; c[3][1] = o[1]; c[3][2] = o[2]; c[3][3] = o[3];
    c[2][0] = 0;    c[2][1] = o[4]; c[2][2] = o[5]; c[2][3] = o[6];
    c[1][0] = 0;    c[1][1] = 0;    c[1][2] = o[7]; c[1][3] = o[8];
    c[0][0] = 0;    c[0][1] = 0;    c[0][2] = 0;    c[0][3] = o[9];
  }
  // position k0 - 1 gives y_{k0-1}
  uint32_t s = c[3][0] + c[2][1] + c[1][2] + c[0][3];
  uint32_t yprev = (s >= DEC_B) + (s >= 2 * DEC_B) + (s >= 3 * DEC_B);
  bool G = false, P = true;
#pragma unroll
  for (int i = 0; i < DEC_CRT_E; i++) {
    s = c[i + 4][0] + c[i + 3][1] + c[i + 2][2] + c[i + 1][3];
    const uint32_t y = (s >= DEC_B) + (s >= 2 * DEC_B) + (s >= 3 * DEC_B);
    u[i] = (uint64_t)(s - y * DEC_B) + yprev;
    yprev = y;
    const bool g = u[i] >= DEC_B, pr = u[i] == DEC_B - 1;
    G = g || (pr && G);
    P = P && pr;
  }
  *Gt = G;
  *Pt = P;
  uint32_t cout;
  bool ap;
  wave_carry(G, P, 0, &cout, &ap);
  if ((tid & 63) == 0) tmp[tid >> 6] = cout | (ap ? 2u : 0u);
  __syncthreads();
}

// CRT + radix-B carry + addend, with the look-back of k_crt (same flags,
// epochs and recompute fallback); the blocks from nblk on copy tail ranges.
__global__ void __launch_bounds__(DEC_CRT_THREADS)
k_crt10(SegView sv, const uint32_t* __restrict__ res, uint64_t res_stride, uint32_t* __restrict__ out,
        const uint32_t* __restrict__ add, uint32_t nblk, uint32_t* __restrict__ flags, uint32_t epoch,
        uint32_t polls, CopyList tails, const uint32_t* __restrict__ tin, uint32_t* __restrict__ tout,
        uint32_t* __restrict__ err) {
  __shared__ uint32_t tmp[16], tmp2[16];
  __shared__ uint32_t xv[DEC_CRT_THREADS + 1][DEC_XV];
  __shared__ uint32_t s_state, s_pair, s_spec, s_spec2;
  const uint32_t b = blockIdx.x, tid = threadIdx.x;
  if (b >= nblk) {
    copy_tail_block(tails, tin, tout, b - nblk);
    return;
  }
  CrtSeg sg;
  uint32_t first, end;
  sv.find(b, &sg, &first, &end);
  const uint32_t* r0 = res + sg.res_pos;
  const uint32_t* r1 = r0 + res_stride;
  const uint32_t* r2 = r1 + res_stride;
  const uint64_t kb = (uint64_t)(b - first) * DEC_CRT_BLOCK;
  uint64_t u[DEC_CRT_E];
  bool G, P;
  crt_local10(sg, r0, r1, r2, add, kb, xv, tmp, u, &G, &P, &s_spec);
  const uint32_t own = crt_block_pair(tmp);
  if (tid == 0)
    __hip_atomic_store(flags + b, (epoch << 3) | (own << 1) | 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t cin = 0, k = b;
  bool done = (b == first);
  if (!done && s_spec < 2u) {
    cin = s_spec;
    done = true;
  }
  while (!done) {
    k--;
    if (tid == 0) {
      uint32_t f = 0;
      for (uint32_t i = 0; i < polls; i++) {
        f = __hip_atomic_load(flags + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((f & 1u) && (f >> 3) == epoch) break;
        f = 0;
        __builtin_amdgcn_s_sleep(2);
      }
      s_state = f ? 1u : 2u;
      s_pair = (f >> 1) & 3u;
    }
    __syncthreads();
    const uint32_t state = s_state;
    uint32_t pair = s_pair;
    __syncthreads();
    if (state == 2u) {
      uint64_t u2[DEC_CRT_E];
      bool G2, P2;
      crt_local10(sg, r0, r1, r2, add, (uint64_t)(k - first) * DEC_CRT_BLOCK, xv, tmp2, u2, &G2, &P2, &s_spec2);
      pair = crt_block_pair(tmp2);
    }
    if (pair & 1u) { cin = 1; done = true; }
    else if (!(pair & 2u)) done = true;
    else if (k == first) done = true;
  }
  if (tid == 0 && b + 1 == end && ((own & 1u) | ((own >> 1) & cin))) atomicOr(err, CAT_DEVERR_CARRY_OUT);
  const uint32_t wid = tid >> 6;
  uint32_t wc = cin;
  for (uint32_t w = 0; w < wid; w++) {
    const uint32_t x = tmp[w];
    wc = (x & 1u) | ((x >> 1) & wc);
  }
  uint32_t cout;
  bool ap;
  uint32_t c = wave_carry(G, P, wc, &cout, &ap);
  uint32_t* o = out + sg.out_pos;
  const uint64_t k0 = kb + (uint64_t)tid * DEC_CRT_E;
#pragma unroll
  for (int i = 0; i < DEC_CRT_E; i++) {
    const uint64_t kk = k0 + i;
    const uint32_t t = (uint32_t)u[i] + c;
    c = t >= DEC_B;
    if (kk < sg.len) o[kk] = c ? t - DEC_B : t;
  }
}

// Leaves: limbs [16i, 16i+16) of x (zero past L) as eighteen radix-B digits
// at out[18i .. 18i+18), least significant first (schoolbook division).
__global__ void __launch_bounds__(256) k_dec_leaf(const uint32_t* __restrict__ x, uint64_t L,
                                                  uint32_t* __restrict__ out, uint64_t nleaves) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nleaves) return;
  uint32_t w[DEC_LEAF_LIMBS];
#pragma unroll
  for (int k = 0; k < DEC_LEAF_LIMBS; k++) {
    const uint64_t at = i * DEC_LEAF_LIMBS + k;
    w[k] = at < L ? x[at] : 0u;
  }
#pragma unroll
  for (int d = 0; d < DEC_LEAF_DIGITS; d++) {
    uint32_t r = 0;
#pragma unroll
    for (int k = DEC_LEAF_LIMBS - 1; k >= 0; k--) w[k] = div_b(r, w[k], &r);
    out[i * DEC_LEAF_DIGITS + d] = r;
  }
}

// out[k] = k < nin ? in[k] : 0 for k < nout (a node carried up a level).
__global__ void k_copy_pad(const uint32_t* __restrict__ in, uint64_t nin, uint32_t* __restrict__ out,
                           uint64_t nout) {
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nout; k += (uint64_t)gridDim.x * blockDim.x)
    out[k] = k < nin ? in[k] : 0u;
}

// Text: radix-B digits dig[0 .. top] (dig[top] != 0, or top = 0) as
// D = width(dig[top]) + 9 top characters, most significant first.
// ASCII text, most significant digit first.  top (device) is one past the
// highest nonzero radix-10^9 group (0 for x = 0); the leading group takes
// `width` characters, every other group nine.  The character count goes to
// *nc; nothing is written when it exceeds cap.  Grid: one thread per group
// that can exist.
__global__ void __launch_bounds__(256) k_dec_ascii(const uint32_t* __restrict__ dig,
                                                   const unsigned long long* __restrict__ top, uint64_t cap,
                                                   char* __restrict__ out, unsigned long long* __restrict__ nc) {
  const unsigned long long t = *top;
  const uint64_t ti = t ? t - 1 : 0;
  const uint32_t vt = dig[ti];
  uint32_t width = 1;
  for (uint32_t q = vt; q >= 10u; q /= 10u) width++;
  const uint64_t n = width + 9 * ti;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *nc = n;
  if (n > cap || i > ti) return;
  uint32_t v = dig[i];
  if (i == ti) {
    for (int k = (int)width - 1; k >= 0; k--) {
      out[k] = (char)('0' + v % 10u);
      v /= 10u;
    }
    return;
  }
  char* o = out + width + 9 * (ti - 1 - i);
#pragma unroll
  for (int k = 8; k >= 0; k--) {
    o[k] = (char)('0' + v % 10u);
    v /= 10u;
  }
}

// P_0 (the leaf power in radix 10^9), written by a kernel so that a captured
// conversion carries it as an argument
struct DecWords {
  uint32_t w[DEC_LEAF_DIGITS];
};
__global__ void k_dec_p0(DecWords p0, uint32_t* __restrict__ out) {
  if (threadIdx.x < DEC_LEAF_DIGITS) out[threadIdx.x] = p0.w[threadIdx.x];
}
