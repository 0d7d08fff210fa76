// Small products of the reconstruction tree (Sec. 3.2, Alg. 2: the lower
// levels of BalancedProductTree(G_e)), plus utility kernels.
//
//  * k_leaf<LF>: one thread forms a node of tree level LF directly from its
//    (up to) 2^LF consecutive primes, by multiplying a register accumulator by
//    one 32-bit prime at a time.  The node is the same integer the pairwise
//    tree gives (a product of the same leaves), in the same 2^LF-limb slot.
//  * k_school: one wave per product of la, lb <= 128 limbs: column sums (a
//    lane holds up to four consecutive columns, a 64-bit sum and a carry
//    count each), then the ballot carry-lookahead.

// ---------------------------------------------------------------------------
// Leaf packing.  Tree view: level LF, node i of group g is written at
// base[g] + i*2^LF; `tl.mpref` is the prefix count of NODES per group.
// The leaves and the nodes pass through LDS (row t of the tile holds thread
// t's node, padded to 2^LF + 1 words so that the row-wise reads of the
// threads hit distinct banks), so that the global loads and stores of a wave
// cover whole runs of consecutive words.
template <int LF>
__global__ void __launch_bounds__(256)
k_leaf(TreeLevel tl, uint64_t nnodes, const uint32_t* __restrict__ primes, uint32_t* __restrict__ out) {
  constexpr int W = 1 << LF;
  constexpr int RW = W + 1;
  constexpr int NT = 256;
  __shared__ uint32_t tile[NT * RW];
  __shared__ uint64_t noff[NT];
  __shared__ uint32_t ncnt[NT];
  const uint32_t tid = threadIdx.x;
  const uint64_t i0 = (uint64_t)blockIdx.x * NT;
  {
    const uint64_t i = i0 + tid;
    uint64_t off = 0;
    uint32_t cnt = 0;
    if (i < nnodes) {
      uint32_t g = 0;
      while (g + 1 < tl.ngroups && i >= tl.mpref[g + 1]) g++;
      const uint64_t il = i - tl.mpref[g];
      off = tl.base[g] + il * W;
      const uint64_t rem = tl.K[g] - il * W;
      cnt = (uint32_t)(rem < (uint64_t)W ? rem : (uint64_t)W);
    }
    noff[tid] = off;
    ncnt[tid] = cnt;
  }
  __syncthreads();
  // leaf k of node t at tile[t RW + k]: lane group of W threads per node,
  // every load in flight before the first LDS store
  constexpr int NPR = NT / W;     // nodes per round
  {
    uint32_t v[W];
#pragma unroll
    for (int r = 0; r < W; r++) {
      const uint32_t t = r * NPR + tid / W, k = tid % W, c = ncnt[t];
      v[r] = c ? primes[noff[t] + (k < c ? k : c - 1)] : 0u;
    }
#pragma unroll
    for (int r = 0; r < W; r++) tile[(r * NPR + tid / W) * RW + tid % W] = v[r];
  }
  __syncthreads();
  const uint32_t cnt = ncnt[tid];
  uint32_t acc[W];
  {
    acc[0] = tile[tid * RW];
#pragma unroll
    for (int k = 1; k < W; k++) acc[k] = 0;
#pragma unroll
    for (int k = 1; k < W; k++) {
      if ((uint32_t)k < cnt) {
        const uint32_t q = tile[tid * RW + k];
        uint32_t carry = 0;
#pragma unroll
        for (int l = 0; l < k; l++) {
          const uint64_t t = (uint64_t)acc[l] * q + carry;
          acc[l] = (uint32_t)t;
          carry = (uint32_t)(t >> 32);
        }
        acc[k] = carry;
      }
    }
  }
  // each thread rewrites only its own row: no barrier between its reads and
  // its writes
#pragma unroll
  for (int k = 0; k < W; k++) tile[tid * RW + k] = acc[k];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < W; r++) {
    const uint32_t t = r * NPR + tid / W, k = tid % W;
    if (k < ncnt[t]) out[noff[t] + k] = tile[t * RW + k];
  }
}

// ---------------------------------------------------------------------------
// Schoolbook products, la, lb <= 128.  4 waves per block, one product each;
// blocks from ceil(nmul / 4) on copy the tail ranges.
#define SCHOOL_MAX 128
// ---------------------------------------------------------------------------
// Long times short (the shorter operand <= COLSUM_MAX_LB limbs): the exact
// column sums V(k) = sum_j a[k-j] b[j] (< 2^74) for k < la + lb, written as
// three words to the residue rows (v0, v1, v2 at r[k], r[stride + k],
// r[2 stride + k]); the raw mode of the CRT kernel then propagates the carries.
// Workgroup b covers the CRT block b (COLSUM_COLS = CAT_CRT_BLOCK columns of
// one product, found with the stage's segment map); it stages the window
// a[kb - lb, kb + COLSUM_COLS) and b in LDS, and each thread slides a window of
// COLSUM_E values of a down j.  Each column keeps a 64-bit sum and a count of
// its carries out of bit 64 (at most lb), one multiply-add and one add-carry
// per 32x32 product.
#define COLSUM_MAX_LB 1024
#define COLSUM_E CAT_CRT_E
#define COLSUM_T CAT_CRT_THREADS
#define COLSUM_COLS (COLSUM_E * COLSUM_T)
static_assert(COLSUM_COLS == CAT_CRT_BLOCK, "column-sum blocks are the CRT blocks");
__device__ __forceinline__ uint32_t uni32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
  return ((uint64_t)uni32((uint32_t)(x >> 32)) << 32) | uni32((uint32_t)x);
}
// acc_e += w_e * bj (64-bit, carry out of bit 64 counted in top_e) for three
// columns: the carry of each multiply-add goes to a mask of its own and is
// added two instructions after it was written
__device__ __forceinline__ void colsum_mac3(uint64_t& a0, uint64_t& a1, uint64_t& a2, uint32_t& t0, uint32_t& t1,
                                            uint32_t& t2, uint32_t w0, uint32_t w1, uint32_t w2, uint32_t bj) {
  uint64_t c0, c1, c2;
  asm("v_mad_u64_u32 %0, %6, %9, %12, %0\n\t"
      "v_mad_u64_u32 %1, %7, %10, %12, %1\n\t"
      "v_mad_u64_u32 %2, %8, %11, %12, %2\n\t"
      "v_addc_co_u32_e64 %3, %6, 0, %3, %6\n\t"
      "v_addc_co_u32_e64 %4, %7, 0, %4, %7\n\t"
      "v_addc_co_u32_e64 %5, %8, 0, %5, %8"
      : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(t0), "+v"(t1), "+v"(t2), "=&s"(c0), "=&s"(c1), "=&s"(c2)
      : "v"(w0), "v"(w1), "v"(w2), "v"(bj));
}
static_assert(COLSUM_E == 3, "colsum_mac3 covers three columns");
// the same for one, two and four columns (one and two with wait states
// between a carry's write and its read)
__device__ __forceinline__ void colsum_mac1(uint64_t& a0, uint32_t& t0, uint32_t w0, uint32_t bj) {
  uint64_t c0;
  asm("v_mad_u64_u32 %0, %2, %3, %4, %0\n\t"
      "s_nop 1\n\t"
      "v_addc_co_u32_e64 %1, %2, 0, %1, %2"
      : "+v"(a0), "+v"(t0), "=&s"(c0)
      : "v"(w0), "v"(bj));
}
__device__ __forceinline__ void colsum_mac2(uint64_t& a0, uint64_t& a1, uint32_t& t0, uint32_t& t1, uint32_t w0,
                                            uint32_t w1, uint32_t bj) {
  uint64_t c0, c1;
  asm("v_mad_u64_u32 %0, %4, %6, %8, %0\n\t"
      "v_mad_u64_u32 %1, %5, %7, %8, %1\n\t"
      "s_nop 0\n\t"
      "v_addc_co_u32_e64 %2, %4, 0, %2, %4\n\t"
      "v_addc_co_u32_e64 %3, %5, 0, %3, %5"
      : "+v"(a0), "+v"(a1), "+v"(t0), "+v"(t1), "=&s"(c0), "=&s"(c1)
      : "v"(w0), "v"(w1), "v"(bj));
}
__device__ __forceinline__ void colsum_mac4(uint64_t& a0, uint64_t& a1, uint64_t& a2, uint64_t& a3, uint32_t& t0,
                                            uint32_t& t1, uint32_t& t2, uint32_t& t3, uint32_t w0, uint32_t w1,
                                            uint32_t w2, uint32_t w3, uint32_t bj) {
  uint64_t c0, c1, c2, c3;
  asm("v_mad_u64_u32 %0, %8, %12, %16, %0\n\t"
      "v_mad_u64_u32 %1, %9, %13, %16, %1\n\t"
      "v_mad_u64_u32 %2, %10, %14, %16, %2\n\t"
      "v_mad_u64_u32 %3, %11, %15, %16, %3\n\t"
      "v_addc_co_u32_e64 %4, %8, 0, %4, %8\n\t"
      "v_addc_co_u32_e64 %5, %9, 0, %5, %9\n\t"
      "v_addc_co_u32_e64 %6, %10, 0, %6, %10\n\t"
      "v_addc_co_u32_e64 %7, %11, 0, %7, %11"
      : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(t0), "+v"(t1), "+v"(t2), "+v"(t3), "=&s"(c0), "=&s"(c1),
        "=&s"(c2), "=&s"(c3)
      : "v"(w0), "v"(w1), "v"(w2), "v"(w3), "v"(bj));
}
template <int E>
__device__ __forceinline__ void mac_cols(uint64_t* acc, uint32_t* top, const uint32_t* w, uint32_t bj) {
  if constexpr (E == 1) colsum_mac1(acc[0], top[0], w[0], bj);
  if constexpr (E == 2) colsum_mac2(acc[0], acc[1], top[0], top[1], w[0], w[1], bj);
  if constexpr (E == 3) colsum_mac3(acc[0], acc[1], acc[2], top[0], top[1], top[2], w[0], w[1], w[2], bj);
  if constexpr (E == 4)
    colsum_mac4(acc[0], acc[1], acc[2], acc[3], top[0], top[1], top[2], top[3], w[0], w[1], w[2], w[3], bj);
}
__global__ void __launch_bounds__(COLSUM_T) k_colsum(DescView dv, SegView sv, const uint32_t* __restrict__ ain,
                                                const uint32_t* __restrict__ bin, uint32_t* __restrict__ res,
                                                uint64_t stride, uint32_t* __restrict__ err) {
  // lb rounded up to even (b padded with a zero limb); sw[t] = a[kb - lbe + t]
  __shared__ uint32_t sw[COLSUM_COLS + COLSUM_MAX_LB];
  __shared__ __align__(8) uint32_t sbv[COLSUM_MAX_LB];
  CrtSeg sg;
  uint32_t first, end, si;
  sv.find(blockIdx.x, &sg, &first, &end, &si);
  const MulDesc d = dv.get(uni32(si));
  // the longer operand slides, the shorter one is the kernel of the sums
  const uint32_t da = uni32(d.la), db = uni32(d.lb);
  const bool sw_ab = da < db;
  const uint32_t* a = sw_ab ? bin + uni64(d.b_off) : ain + uni64(d.a_off);
  const uint32_t* b = sw_ab ? ain + uni64(d.a_off) : bin + uni64(d.b_off);
  const uint32_t la = sw_ab ? db : da, lb = sw_ab ? da : db;
  const uint32_t tid = threadIdx.x;
  if (lb > COLSUM_MAX_LB) {
    if (tid == 0) atomicOr(err, CAT_DEVERR_BOUNDS);
    return;
  }
  const uint32_t L = la + lb;
  const uint32_t kb = (uni32(blockIdx.x) - uni32(first)) * COLSUM_COLS;
  const uint32_t lbe = (lb + 1) & ~1u;
  const uint32_t wn = COLSUM_COLS + lbe;
  for (uint32_t i = tid; i < wn; i += COLSUM_T) {
    const int64_t idx = (int64_t)kb - (int64_t)lbe + i;
    sw[i] = (idx >= 0 && idx < (int64_t)la) ? a[idx] : 0u;
  }
  for (uint32_t i = tid; i < lbe; i += COLSUM_T) sbv[i] = i < lb ? b[i] : 0u;
  __syncthreads();
  // column k = kb + COLSUM_E tid + e takes a[k - j] = sw[c0 + e - j]; the
  // reads for j + 1 and j + 2 at the last pair (down to sw[COLSUM_E tid])
  // stay in the window
  const uint32_t c0 = COLSUM_E * tid + lbe;
  uint32_t w[COLSUM_E];
#pragma unroll
  for (int e = 0; e < COLSUM_E; e++) w[e] = sw[c0 + e];
  uint64_t acc[COLSUM_E];
  uint32_t top[COLSUM_E];
#pragma unroll
  for (int e = 0; e < COLSUM_E; e++) {
    acc[e] = 0;
    top[e] = 0;
  }
  for (uint32_t j = 0; j < lbe; j += 2) {
    const uint2 bj = *(const uint2*)&sbv[j];
    const uint32_t wn1 = sw[c0 - j - 1], wn2 = sw[c0 - j - 2];
    colsum_mac3(acc[0], acc[1], acc[2], top[0], top[1], top[2], w[0], w[1], w[2], bj.x);
    // j + 1: every column moves one position down a
    colsum_mac3(acc[0], acc[1], acc[2], top[0], top[1], top[2], wn1, w[0], w[1], bj.y);
    w[2] = w[0];
    w[1] = wn1;
    w[0] = wn2;
  }
  uint32_t* r = res + sg.res_pos;
  const uint32_t k0 = kb + COLSUM_E * tid;
#pragma unroll
  for (int e = 0; e < COLSUM_E; e++) {
    if (k0 + e >= L) break;
    r[k0 + e] = (uint32_t)acc[e];
    r[stride + k0 + e] = (uint32_t)(acc[e] >> 32);
    r[2 * stride + k0 + e] = top[e];
  }
}

#define SCHOOL_WAVES 4
#define SCHOOL_WIN (3 * SCHOOL_MAX)
// Column sums of one product in one wave: lane owns the E consecutive columns
// k = E lane + e (64 E >= la + lb - 1) and runs over j < lbe (the shorter
// operand rounded up to even, padded with a zero limb): V(k) = sum_j
// a[k - j] b[j], with sa[t] = a[t - lbe] (zero outside [0, la)).  Each column
// keeps a 64-bit sum and its count of carries out of bit 64; the three words
// go to sv[.][k + 3].
template <int E>
__device__ __forceinline__ void school_cols(const uint32_t* sa, const uint32_t* sbv, uint32_t lbe, uint32_t lane,
                                            uint32_t (*sv)[2 * SCHOOL_MAX + 4]) {
  const uint32_t c0 = E * lane + lbe;
  uint32_t w[E];
#pragma unroll
  for (int e = 0; e < E; e++) w[e] = sa[c0 + e];
  uint64_t acc[E];
  uint32_t top[E];
#pragma unroll
  for (int e = 0; e < E; e++) {
    acc[e] = 0;
    top[e] = 0;
  }
  for (uint32_t j = 0; j < lbe; j += 2) {
    const uint2 bj = *(const uint2*)&sbv[j];
    const uint32_t wn1 = sa[c0 - j - 1], wn2 = sa[c0 - j - 2];
    mac_cols<E>(acc, top, w, bj.x);
    // j + 1: every column one position further down a
    uint32_t w1[E];
    w1[0] = wn1;
#pragma unroll
    for (int e = 1; e < E; e++) w1[e] = w[e - 1];
    mac_cols<E>(acc, top, w1, bj.y);
#pragma unroll
    for (int e = E - 1; e >= 2; e--) w[e] = w[e - 2];
    if constexpr (E >= 2) w[1] = wn1;
    w[0] = wn2;
  }
#pragma unroll
  for (int e = 0; e < E; e++) {
    const uint32_t k = E * lane + e;
    sv[0][k + 3] = (uint32_t)acc[e];
    sv[1][k + 3] = (uint32_t)(acc[e] >> 32);
    sv[2][k + 3] = top[e];
  }
  for (uint32_t k = 64 * E + lane; k < 2 * SCHOOL_MAX; k += 64) {
    sv[0][k + 3] = 0;
    sv[1][k + 3] = 0;
    sv[2][k + 3] = 0;
  }
}

__global__ void __launch_bounds__(64 * SCHOOL_WAVES)
k_school(DescView dv, uint64_t nmul, const uint32_t* __restrict__ ain, const uint32_t* __restrict__ bin,
         uint32_t* __restrict__ out, uint32_t* __restrict__ err, uint32_t prod_blocks, CopyList tails,
         const uint32_t* __restrict__ tin, uint32_t* __restrict__ tout) {
  __shared__ uint32_t sa[SCHOOL_WAVES][SCHOOL_WIN];
  __shared__ __align__(8) uint32_t sb[SCHOOL_WAVES][SCHOOL_MAX];
  __shared__ uint32_t sv[SCHOOL_WAVES][3][2 * SCHOOL_MAX + 4];
  if (blockIdx.x >= prod_blocks) {
    copy_tail_block(tails, tin, tout, blockIdx.x - prod_blocks);
    return;
  }
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t mi = (uint64_t)blockIdx.x * SCHOOL_WAVES + w;
  if (mi >= nmul) return;   // whole wave leaves together; no block barrier below
  const MulDesc d = dv.get(uni64(mi));
  // the longer operand slides (la), the shorter one is summed over (lb)
  const uint32_t da = uni32(d.la), db = uni32(d.lb);
  const bool swp = da < db;
  const uint32_t* a = swp ? bin + uni64(d.b_off) : ain + uni64(d.a_off);
  const uint32_t* b = swp ? ain + uni64(d.a_off) : bin + uni64(d.b_off);
  const uint32_t la = swp ? db : da, lb = swp ? da : db, L = la + lb;
  const uint32_t lbe = (lb + 1) & ~1u;
  {
    // every load of the lane in flight together: clamped addresses, masks
    uint32_t xa[SCHOOL_WIN / 64], xb[2];
#pragma unroll
    for (int i = 0; i < SCHOOL_WIN / 64; i++) {
      const uint32_t idx = lane + 64 * i - lbe;    // wraps when t < lbe
      xa[i] = idx < la ? a[idx] : 0u;
    }
#pragma unroll
    for (int i = 0; i < 2; i++) {
      const uint32_t t = lane + 64 * i;
      xb[i] = t < lb ? b[t] : 0u;
    }
#pragma unroll
    for (int i = 0; i < SCHOOL_WIN / 64; i++) sa[w][lane + 64 * i] = xa[i];
#pragma unroll
    for (int i = 0; i < 2; i++) sb[w][lane + 64 * i] = xb[i];
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  const uint32_t ncol = (L - 1 + 63) / 64;   // columns per lane; k < L - 1 carry the sums
  if (ncol <= 1)
    school_cols<1>(sa[w], sb[w], lbe, lane, sv[w]);
  else if (ncol == 2)
    school_cols<2>(sa[w], sb[w], lbe, lane, sv[w]);
  else if (ncol == 3)
    school_cols<3>(sa[w], sb[w], lbe, lane, sv[w]);
  else
    school_cols<4>(sa[w], sb[w], lbe, lane, sv[w]);
  if (lane < 3) { sv[w][0][lane] = 0; sv[w][1][lane] = 0; sv[w][2][lane] = 0; }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  // lane owns limbs 4*lane .. 4*lane+3 (position k stored at index k+3)
  constexpr int E = 4;
  const uint32_t k0 = lane * E;
  uint64_t u[E];
  uint32_t yprev = (uint32_t)(((uint64_t)sv[w][0][k0 + 2] + sv[w][1][k0 + 1] + sv[w][2][k0]) >> 32);
  bool G = false, P = true;
#pragma unroll
  for (int i = 0; i < E; i++) {
    const uint32_t k = k0 + i;
    uint64_t s = 0;
    if (k < L) s = (uint64_t)sv[w][0][k + 3] + sv[w][1][k + 2] + sv[w][2][k + 1];
    u[i] = (s & 0xFFFFFFFFull) + yprev;
    yprev = (uint32_t)(s >> 32);
    const bool g = u[i] >= (1ull << 32), pr = u[i] == 0xFFFFFFFFull;
    G = g || (pr && G);
    P = P && pr;
  }
  uint32_t cout;
  bool ap;
  uint32_t c = wave_carry(G, P, 0, &cout, &ap);
#pragma unroll
  for (int i = 0; i < E; i++) {
    const uint32_t k = k0 + i;
    const uint64_t t = u[i] + c;
    c = (uint32_t)(t >> 32);
    if (k < L) out[d.c_off + k] = (uint32_t)t;
  }
  if (lane == 0 && cout) atomicOr(err, CAT_DEVERR_CARRY_OUT);
}

// ---------------------------------------------------------------------------
// Copy of up to CAT_MAX_GROUPS ranges (the odd nodes carried up a level).
__global__ void k_copy_ranges(CopyList cl, const uint32_t* __restrict__ in, uint32_t* __restrict__ out) {
  const uint32_t r = blockIdx.y;
  if (r >= cl.n) return;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < cl.len[r];
       k += (uint64_t)gridDim.x * blockDim.x)
    out[cl.off[r] + k] = in[cl.off[r] + k];
}

// Copies of up to CAT_MAX_GROUPS ranges from one array to another, each to
// an offset of its own (the primes of the requests of a batch, compacted).
struct MoveList {
  uint32_t n;
  uint64_t src[CAT_MAX_GROUPS], dst[CAT_MAX_GROUPS], len[CAT_MAX_GROUPS];
};
__global__ void k_move_ranges(MoveList ml, const uint32_t* __restrict__ in, uint32_t* __restrict__ out) {
  const uint32_t r = blockIdx.y;
  if (r >= ml.n) return;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ml.len[r];
       k += (uint64_t)gridDim.x * blockDim.x)
    out[ml.dst[r] + k] = in[ml.src[r] + k];
}

__global__ void k_fill(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x)
    p[k] = v;
}

// Highest index with a nonzero limb, +1 (0 if all zero) -> *top; limbs below
// ncopy are also copied to dst (the caller's output).  Each block reduces in
// LDS and issues one atomicMax.
__global__ void __launch_bounds__(256) k_top_nonzero(const uint32_t* __restrict__ x, uint64_t n,
                                                     unsigned long long* top, uint32_t* __restrict__ dst,
                                                     uint64_t ncopy) {
  __shared__ unsigned long long part[4];
  unsigned long long best = 0;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t v = x[k];
    if (v) best = k + 1;
    if (k < ncopy) dst[k] = v;
  }
  for (int d = 32; d >= 1; d >>= 1) {
    unsigned long long o = __shfl_xor(best, d, 64);
    best = o > best ? o : best;
  }
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); w++) best = part[w] > best ? part[w] : best;
    if (best) atomicMax(top, best);
  }
}

// Limb k of floor(x / 2^s) for x[0..lx) (zero past the top).
__device__ __forceinline__ uint32_t shifted_limb(const uint32_t* __restrict__ x, uint64_t lx, uint64_t s, uint64_t k) {
  const uint64_t w = k + (s >> 5);
  const uint32_t r = (uint32_t)(s & 31);
  const uint32_t lo = w < lx ? x[w] : 0u;
  if (r == 0) return lo;
  const uint32_t hi = w + 1 < lx ? x[w + 1] : 0u;
  return (lo >> r) | (hi << (32 - r));
}

// 1 + the highest index where X = floor(x / 2^s) and Y = y differ (0 if X = Y),
// limbs past the ends being zero -> *top (atomicMax; zero it before).  n: the
// limbs to scan (at least the longer of X and Y).
__global__ void __launch_bounds__(256) k_diff_top(const uint32_t* __restrict__ x, uint64_t lx, uint64_t s,
                                                  const uint32_t* __restrict__ y, uint64_t ly, uint64_t n,
                                                  unsigned long long* top) {
  __shared__ unsigned long long part[4];
  unsigned long long best = 0;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t a = shifted_limb(x, lx, s, k), b = k < ly ? y[k] : 0u;
    if (a != b) best = k + 1;
  }
  for (int d = 32; d >= 1; d >>= 1) {
    unsigned long long o = __shfl_xor(best, d, 64);
    best = o > best ? o : best;
  }
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); w++) best = part[w] > best ? part[w] : best;
    if (best) atomicMax(top, best);
  }
}

// Sum of the bit lengths of the entries of each group (bounds on log2 Q_g).
__global__ void __launch_bounds__(256) k_group_bits(const uint32_t* __restrict__ x, const uint64_t* __restrict__ off,
                                                    uint32_t ngroups, unsigned long long* __restrict__ gbits) {
  const uint32_t g = blockIdx.y;
  if (g >= ngroups) return;
  unsigned long long s = 0;
  for (uint64_t k = off[g] + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < off[g + 1];
       k += (uint64_t)gridDim.x * blockDim.x)
    s += (unsigned long long)(32 - __clz(x[k]));
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(&gbits[g], s);
}

// Fingerprints of a limb vector: x mod (2^32 - 5), x mod (2^32 + 1), x mod
// (2^32 - 1).  Workgroup b reduces the 4096 limbs [4096 b, 4096 b + 4096):
// thread t holds the RES_C limbs at 4096 b + 256 i + t (coalesced loads) and
// the block's partial is sum_k x_k (2^32)^(k - 4096 b) mod q; the library
// combines the partials with the weights (2^32)^(4096 b) on the host.  With
// 2^32 = 5, -1 and 1 modulo the three moduli, the weight of limb 256 i + t
// is 5^(256 i + t), (-1)^t and 1: a Horner pass over i with the constant
// 5^256 (two folds of 2^32 = 5 per step) for the first, plain 64-bit sums
// for the others.
#define RES_T 256
#define RES_C 16
#define RES_BLOCK (RES_T * RES_C)
#define RES_Q0 4294967291ull   // 2^32 - 5
#define RES_Q1 4294967297ull   // 2^32 + 1
#define RES_Q2 4294967295ull   // 2^32 - 1
// y mod (2^32 - 5) for any 64-bit y: fold 2^32 = 5 twice, then one subtraction
__device__ __forceinline__ uint32_t mod_q0(uint64_t y) {
  const uint64_t r = (y >> 32) * 5ull + (y & 0xFFFFFFFFull);   // < 6 * 2^32
  const uint64_t r2 = (r >> 32) * 5ull + (r & 0xFFFFFFFFull);  // < 2^32 + 30
  return (uint32_t)(r2 >= RES_Q0 ? r2 - RES_Q0 : r2);
}
__global__ void __launch_bounds__(RES_T) k_residues(const uint32_t* __restrict__ x, uint64_t n, uint32_t w256,
                                                    uint64_t* __restrict__ part) {
  __shared__ uint64_t red[3][RES_T / 64];
  const uint32_t t = threadIdx.x;
  const uint64_t base = (uint64_t)blockIdx.x * RES_BLOCK;
  uint32_t v[RES_C];
#pragma unroll
  for (int i = 0; i < RES_C; i++) {
    const uint64_t k = base + (uint64_t)i * RES_T + t;
    v[i] = k < n ? x[k] : 0u;
  }
  uint32_t h = 0;
  uint64_t s = 0;
#pragma unroll
  for (int i = RES_C - 1; i >= 0; i--) {
    h = mod_q0((uint64_t)h * w256 + v[i]);
    s += v[i];
  }
  // lane weight 5^t mod q0 by square-and-multiply over the bits of t < 256
  uint32_t w = 1, b5 = 5;
  for (uint32_t e = t; e; e >>= 1) {
    if (e & 1) w = mod_q0((uint64_t)w * b5);
    b5 = mod_q0((uint64_t)b5 * b5);
  }
  uint64_t a0 = mod_q0((uint64_t)h * w);      // < 2^32: 256 of them sum below 2^40
  uint64_t ap = (t & 1) ? 0 : s, am = (t & 1) ? s : 0;   // s < 2^36
  for (int d = 32; d >= 1; d >>= 1) {
    a0 += __shfl_xor(a0, d, 64);
    ap += __shfl_xor(ap, d, 64);
    am += __shfl_xor(am, d, 64);
  }
  if ((t & 63) == 0) {
    red[0][t >> 6] = a0;
    red[1][t >> 6] = ap;
    red[2][t >> 6] = am;
  }
  __syncthreads();
  if (t == 0) {
    uint64_t s0 = 0, sp = 0, sm = 0;
    for (int k = 0; k < RES_T / 64; k++) {
      s0 += red[0][k];
      sp += red[1][k];
      sm += red[2][k];
    }
    part[3 * (uint64_t)blockIdx.x + 0] = s0 % RES_Q0;
    part[3 * (uint64_t)blockIdx.x + 1] = (sp % RES_Q1 + RES_Q1 - sm % RES_Q1) % RES_Q1;
    part[3 * (uint64_t)blockIdx.x + 2] = (sp + sm) % RES_Q2;
  }
}

// ---------------------------------------------------------------------------
// Twiddle tables.  roots[prime][s] = omega_{2^s} in Montgomery form, for
// each prime set (the second set has roots up to 2^CAT_LAZY_MAX_LOGN).
struct RootsC {
  uint32_t r[CAT_NPRIMES][CAT_MAX_LOGN + 1];     // forward, Montgomery form
  uint32_t ir[CAT_NPRIMES][CAT_MAX_LOGN + 1];    // inverse
  uint32_t one[CAT_NPRIMES];                     // R mod p
};
__constant__ RootsC c_roots;
__constant__ RootsC c_roots1;
template <int AS>
__device__ __forceinline__ const RootsC& rootsc() {
  if constexpr (AS == 0) return c_roots;
  else return c_roots1;
}

__device__ __forceinline__ uint32_t mont_pow(uint32_t b, uint64_t e, uint32_t one, uint32_t p, uint32_t pinv) {
  uint32_t r = one;
  while (e) {
    if (e & 1) r = mont_mul(r, b, p, pinv);
    b = mont_mul(b, b, p, pinv);
    e >>= 1;
  }
  return r;
}
__device__ __forceinline__ uint2 tw_pair(uint32_t w, uint32_t pinv) { return make_uint2(w, w * pinv); }
// Shoup pair of the value whose Montgomery form is w: (W, floor(W 2^32 / p))
__device__ __forceinline__ uint2 shoup_pair(uint32_t w, uint32_t p, uint32_t pinv) {
  const uint32_t W = mont_mul(w, 1u, p, pinv);
  return make_uint2(W, (uint32_t)(((uint64_t)W << 32) / p));
}

// Pass tables: for s = 1..14, S = 2^s, radix R = 2^pass_logr(s), entry
// (k1, j2) at tws_off(s) + (k1 << (s - r)) + j2 = omega_S^{+-j2*k1}:
// Montgomery pairs (set 0) or Shoup pairs (set 1).
template <int AS>
__global__ void k_build_tws(uint2* __restrict__ tws, uint2* __restrict__ itws) {
  const uint32_t prime = blockIdx.y;
  const PrimeC& pc = primec<AS>(prime);
  const RootsC& rc = rootsc<AS>();
  const uint32_t p = pc.p, pinv = pc.pinv;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < TWS_ENTRIES; i += gridDim.x * blockDim.x) {
    int s = 1;
    while (tws_off(s + 1) <= i) s++;
    const uint32_t li = i - tws_off(s);
    const int r = pass_logr(s);
    const uint32_t k1 = li >> (s - r), j2 = li & ((1u << (s - r)) - 1);
    const uint64_t e = (uint64_t)j2 * k1;
    const uint32_t w = mont_pow(rc.r[prime][s], e, rc.one[prime], p, pinv);
    const uint32_t iw = mont_pow(rc.ir[prime][s], e, rc.one[prime], p, pinv);
    tws[(size_t)prime * TWS_ENTRIES + i] = AS == 0 ? tw_pair(w, pinv) : shoup_pair(w, p, pinv);
    itws[(size_t)prime * TWS_ENTRIES + i] = AS == 0 ? tw_pair(iw, pinv) : shoup_pair(iw, p, pinv);
  }
}

// Two-level tables of omega = omega_{2^tw_logn}: lo[i] = omega^i (i < 2^14,
// Montgomery pairs), hi[i] = omega^{i*2^14} (i < 2^(tw_logn - 14), Montgomery
// form); and the inverse.
template <int AS>
__global__ void k_build_tw2(uint2* __restrict__ lo, uint32_t* __restrict__ hi, uint2* __restrict__ ilo,
                            uint32_t* __restrict__ ihi) {
  const uint32_t prime = blockIdx.y;
  const PrimeC& pc = primec<AS>(prime);
  const RootsC& rc = rootsc<AS>();
  const uint32_t p = pc.p, pinv = pc.pinv;
  const uint32_t one = rc.one[prime];
  const uint32_t r = rc.r[prime][tw_logn<AS>()], ir = rc.ir[prime][tw_logn<AS>()];
  const uint32_t nhi = 1u << (tw_logn<AS>() - TW2_LO_BITS);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < TW2_LO; i += gridDim.x * blockDim.x) {
    lo[(size_t)prime * TW2_LO + i] = tw_pair(mont_pow(r, i, one, p, pinv), pinv);
    ilo[(size_t)prime * TW2_LO + i] = tw_pair(mont_pow(ir, i, one, p, pinv), pinv);
    if (i < nhi) {
      hi[(size_t)prime * TW2_HI + i] = mont_pow(r, (uint64_t)i << TW2_LO_BITS, one, p, pinv);
      ihi[(size_t)prime * TW2_HI + i] = mont_pow(ir, (uint64_t)i << TW2_LO_BITS, one, p, pinv);
    }
  }
}
