// Several lower levels of the product trees in one launch (Sec. 3.2: the
// levels of BalancedProductTree, batched across all groups G_e).
//
// A workgroup owns a tile of FT_SLOTS = 4096 consecutive leaves of one group.
// A node of level j covers 2^j leaves, and 2^j divides 4096 for j <= 12, so
// every node of the levels j0..j1 (j1 <= 11) that touches the tile lies inside
// it: the workgroup carries its tile from level j0 to level j1 + 1 without
// leaving LDS.  At each level it multiplies the adjacent node pairs with the
// three-prime transform -- one 256-thread part per prime, each holding both
// operands of every product of the tile in LDS, exactly the per-prime work of
// a one-workgroup product tile -- then recombines the three residues of every
// coefficient by Garner's method and propagates the carries inside each
// product (products never cross the tile, so no other workgroup is involved)
// and writes the product limbs back over the tile's limb array, where the
// next level reads them.  The odd last node of a level stays where it is.
// Only the first level's limbs are read from HBM and only the last level's
// are written: 8 bytes per leaf limb for all the fused levels together,
// against 4 B in + 12 B of residues out and back + 4 B out per level when
// every level is a transform launch followed by a carry launch.
#define FT_LOGT 12
#define FT_SLOTS (1u << FT_LOGT)
#define FT_PART 256                               // threads per prime (FT_SLOTS / 16)
#define FT_THREADS (CAT_NPRIMES * FT_PART)
#define FT_CRT_E 8                                // positions per thread of the carry step
#define FT_CRT_THREADS (FT_SLOTS / FT_CRT_E)      // 512: waves 0..7
#define FT_MAX_LEVELS 12
static_assert(FT_CRT_THREADS <= FT_THREADS, "the carry step runs on a part of the workgroup");

struct FusedTree {
  uint32_t ngroups;                          // groups with products in the fused levels
  uint32_t j0, j1;                           // first and last fused level (input node sizes 2^j)
  uint64_t base[CAT_MAX_GROUPS];             // arena offset of the group's first leaf
  uint64_t K[CAT_MAX_GROUPS];                // leaves of the group
  uint32_t tpref[CAT_MAX_GROUPS + 1];        // tiles before the group
  uint2 scale[FT_MAX_LEVELS][CAT_NPRIMES];   // 2^32 N^-1 (Montgomery pair) for N = 2^(j+1), j = j0 + index
};

// One prime's part of a fused tile (FT_PART threads, local index lt): both
// operand tiles in lds (A at [0, T), B at [T, 2T)) transformed, multiplied
// pointwise and the product transformed back into A.
__device__ __forceinline__ void fused_transform(uint32_t* lds, int logN, uint2 sc, const PrimeC& pc,
                                                const uint2* __restrict__ tws, const uint2* __restrict__ itws,
                                                uint32_t lt) {
  const uint32_t p = pc.p;
  ntt_fwd_tile<true>(lds, logN, 2 * FT_SLOTS, 0, tws, pc, lt, FT_PART);
  // pointwise on the 16 positions of A and of B this thread wrote last (the
  // last radix-16 pass gives it groups lt and lt + 256), which the first
  // inverse pass reads back in the same thread
#pragma unroll
  for (int k = 0; k < 16; k++) {
    const uint32_t t = 16 * lt + k;
    const uint32_t x = lds[lds_pad(t)], y = lds[lds_pad(FT_SLOTS + t)];
    lds[lds_pad(t)] = mul_tw(mont_mul(x, y, p, pc.pinv), sc.x, sc.y, p);
  }
  ntt_inv_tile<true>(lds, logN, FT_SLOTS, 0, itws, pc, lt, FT_PART);   // ends with a barrier
}

// Garner + carries over a fused tile whose products occupy the segments
// [m N, m N + len(m)) (len(m) = 0: no product).  Thread t < 512 owns
// positions [8 t, 8 t + 8), all in product m = 8 t / N; it recomputes the
// values of the three positions before its first (zero before the product's
// first position), which enter its first column sums.  The same carry scheme
// as the carry kernel: column values V(k) = v0 + v1 2^32 + v2 2^64,
// s_k = v0(k) + v1(k-1) + v2(k-2) < 3 2^32, binary generate / propagate per
// limb.  The last thread of a product passes no carry on (its pair is
// masked), so one unsegmented scan over the tile resolves every product at
// once.  put(m, k, limb) stores limb k of product m; a product of
// len(m) = N + 1 limbs (la + lb - 1 = N coefficients) gets its top limb
// (position N, where only the high words of the last two coefficients and
// the carry arrive) from the segment's last thread; *bad is set when a
// product would exceed its len(m) limbs.  Every thread of the workgroup
// calls this (one barrier inside).
template <class LEN, class PUT>
__device__ __forceinline__ void fused_carry(uint32_t (*buf)[lds_pad(2 * FT_SLOTS)], int logN, uint32_t tid,
                                            LEN len, PUT put, uint32_t* wpair, uint32_t* bad) {
  const uint32_t N = 1u << logN;
  const uint32_t k0 = tid * FT_CRT_E;
  const uint32_t m = k0 >> logN;
  const uint32_t kp = k0 & (N - 1);                        // position in the product
  const uint32_t L = tid < FT_CRT_THREADS ? len(m) : 0u;   // la + lb (0: no product)
  const bool live = L > 0;
  uint32_t v0[FT_CRT_E + 3], v1[FT_CRT_E + 3], v2[FT_CRT_E + 3];
#pragma unroll
  for (int i = 0; i < FT_CRT_E + 3; i++) {
    v0[i] = v1[i] = v2[i] = 0;
    const bool here = live && (i >= 3 || kp + i >= 3);
    if (here) {
      const uint32_t k = k0 + i - 3;
      garner3(buf[0][lds_pad(k)], buf[1][lds_pad(k)], buf[2][lds_pad(k)], v0[i], v1[i], v2[i]);
    }
  }
  uint64_t u[FT_CRT_E];
  uint32_t yprev = (uint32_t)(((uint64_t)v0[2] + v1[1] + v2[0]) >> 32);
  bool G = false, P = true;
#pragma unroll
  for (int i = 0; i < FT_CRT_E; i++) {
    const uint64_t s = (uint64_t)v0[i + 3] + v1[i + 2] + v2[i + 1];
    u[i] = (s & 0xFFFFFFFFull) + yprev;
    yprev = (uint32_t)(s >> 32);
    const bool gg = u[i] >= (1ull << 32), pp = u[i] == 0xFFFFFFFFull;
    G = gg || (pp && G);
    P = P && pp;
  }
  const bool seg_end = ((k0 + FT_CRT_E) & (N - 1)) == 0;   // last thread of its product
  const bool Gm = live && G && !seg_end, Pm = live && P && !seg_end;
  uint32_t cout;
  bool ap;
  wave_carry(Gm, Pm, 0, &cout, &ap);
  if (tid < FT_CRT_THREADS && (tid & 63) == 0) wpair[tid >> 6] = cout | (ap ? 2u : 0u);
  __syncthreads();
  uint32_t wc = 0;
  for (uint32_t w = 0; w < (tid >> 6) && w < FT_CRT_THREADS / 64; w++) {
    const uint32_t x = wpair[w];
    wc = (x & 1u) | ((x >> 1) & wc);
  }
  uint32_t c = wave_carry(Gm, Pm, wc, &cout, &ap);
  if (live) {
#pragma unroll
    for (int i = 0; i < FT_CRT_E; i++) {
      const uint64_t t = u[i] + c;
      c = (uint32_t)(t >> 32);
      const uint32_t limb = (uint32_t)t;
      if (kp + i < L) put(m, kp + i, limb);
      else if (limb) *bad = 1;                       // the product exceeds la + lb limbs
    }
    if (seg_end) {
      // what the segment passes on, position N: V(N) = 0, so the column sum
      // there is v1(N-1) + v2(N-2), plus the binary carry and the spill of
      // position N - 1; it is the top limb of an (N + 1)-limb product and
      // zero for every other, and nothing may reach position N + 1
      const uint64_t sN = (uint64_t)v1[FT_CRT_E + 2] + v2[FT_CRT_E + 1];
      const uint64_t uN = (sN & 0xFFFFFFFFull) + yprev + c;
      const uint64_t beyond = (uN >> 32) + (sN >> 32) + v2[FT_CRT_E + 2];
      if (L > N) {
        put(m, N, (uint32_t)uN);
        if (beyond) *bad = 1;
      } else if (uN || beyond) {
        *bad = 1;
      }
    }
  }
}

// Products of a generic batch whose transforms fit one workgroup (N <= 2^12),
// every such bucket in one launch: one 768-thread workgroup per tile of up to
// 2^12 / N products of one bucket (a tile table built by the plan), the
// three primes' transforms in LDS, Garner and the carries in the workgroup,
// the limbs written straight to the products' outputs.
struct FusedMul {
  const uint2* tiles;                  // per tile: x = first descriptor, y = logN | count << 8
  const MulDesc* desc;                 // descriptors, bucket by bucket
  uint2 scale[FT_LOGT + 1][CAT_NPRIMES];
};

__global__ void __launch_bounds__(FT_THREADS)
k_mul_fused(FusedMul fm, const uint32_t* __restrict__ ain, const uint32_t* __restrict__ bin,
            uint32_t* __restrict__ out, NttTables tb, uint32_t* __restrict__ err) {
  __shared__ uint32_t buf[CAT_NPRIMES][lds_pad(2 * FT_SLOTS)];
  __shared__ MulDesc ds[64];
  __shared__ uint32_t wpair[FT_CRT_THREADS / 64];
  const uint32_t tid = threadIdx.x;
  const uint2 tl = fm.tiles[blockIdx.x];
  const int logN = (int)(tl.y & 0xFFu);
  const uint32_t cnt = tl.y >> 8, N = 1u << logN;
  for (uint32_t i = tid; i < cnt; i += FT_THREADS) ds[i] = fm.desc[tl.x + i];
  __syncthreads();
  // FT_PART is a multiple of the wave size: the prime is uniform per wave
  const uint32_t prime = __builtin_amdgcn_readfirstlane(tid / FT_PART), lt = tid % FT_PART;
  const PrimeC& pc = c_primes[prime];
  const uint32_t p = pc.p;
  uint32_t* lds = buf[prime];
  {
    // every load of the thread in flight before the first use: clamped
    // in-bounds addresses and masks
    uint32_t xa[16], xb[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const uint32_t s = lt + i * FT_PART;
      const uint32_t m = s >> logN, q = s & (N - 1);
      const uint32_t mc = m < cnt ? m : cnt - 1;
      const MulDesc d = ds[mc];
      const uint32_t ka = (m < cnt && q < d.la) ? 0xFFFFFFFFu : 0u, kb = (m < cnt && q < d.lb) ? 0xFFFFFFFFu : 0u;
      xa[i] = ain[d.a_off + (q & ka)] & ka;
      xb[i] = bin[d.b_off + (q & kb)] & kb;
    }
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const uint32_t s = lt + i * FT_PART;
      lds[lds_pad(s)] = reduce_limb(xa[i], p);
      lds[lds_pad(FT_SLOTS + s)] = reduce_limb(xb[i], p);
    }
  }
  __syncthreads();
  fused_transform(lds, logN, fm.scale[logN][prime], pc, tb.tws + (size_t)prime * TWS_ENTRIES,
                  tb.itws + (size_t)prime * TWS_ENTRIES, lt);
  uint32_t bad = 0;
  fused_carry(
      buf, logN, tid, [&](uint32_t m) -> uint32_t { return m < cnt ? ds[m].la + ds[m].lb : 0u; },
      [&](uint32_t m, uint32_t k, uint32_t limb) { out[ds[m].c_off + k] = limb; }, wpair, &bad);
  if (bad) atomicOr(err, CAT_DEVERR_CARRY_OUT);
}

__global__ void __launch_bounds__(FT_THREADS)
k_tree_fused(FusedTree ft, const uint32_t* __restrict__ in, uint32_t* __restrict__ out, NttTables tb,
             uint32_t* __restrict__ err) {
  __shared__ uint32_t buf[CAT_NPRIMES][lds_pad(2 * FT_SLOTS)];   // per prime: A [0, T), B [T, 2T)
  __shared__ uint32_t X[FT_SLOTS];                              // limbs of the current level
  __shared__ uint32_t wpair[FT_CRT_THREADS / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t b = blockIdx.x;
  uint32_t g = 0;
  while (g + 1 < ft.ngroups && b >= ft.tpref[g + 1]) g++;
  const uint64_t t0 = (uint64_t)(b - ft.tpref[g]) * FT_SLOTS;
  const uint32_t Kt = (uint32_t)min((uint64_t)FT_SLOTS, ft.K[g] - t0);   // leaves in this tile
  const uint64_t gofs = ft.base[g] + t0;
  for (uint32_t k = tid; k < Kt; k += FT_THREADS) X[k] = in[gofs + k];
  __syncthreads();

  // FT_PART is a multiple of the wave size: the prime is uniform per wave
  const uint32_t prime = __builtin_amdgcn_readfirstlane(tid / FT_PART), lt = tid % FT_PART;
  const PrimeC& pc = c_primes[prime];
  const uint32_t p = pc.p;
  uint32_t* lds = buf[prime];
  const uint2* tws = tb.tws + (size_t)prime * TWS_ENTRIES;
  const uint2* itws = tb.itws + (size_t)prime * TWS_ENTRIES;
  uint32_t bad = 0;

  for (uint32_t j = ft.j0; j <= ft.j1; j++) {
    const uint32_t half = 1u << j;
    const int logN = (int)j + 1;
    const uint32_t N = 2u * half;
    const uint32_t nodes = (Kt + half - 1) >> j;
    const uint32_t np = nodes / 2;                 // products: node pairs (2m, 2m + 1)
    if (np == 0) continue;                         // uniform over the workgroup
    // operands into this prime's tile: product m takes slots [m N, m N + N)
    // of A (node 2m, zero-padded) and of B (node 2m + 1, zero-padded)
    {
      uint32_t xa[16], xb[16];
#pragma unroll
      for (int i = 0; i < 16; i++) {
        const uint32_t s = lt + i * FT_PART;
        const uint32_t m = s >> logN, q = s & (N - 1);
        const uint32_t lb = m < np ? min(half, Kt - (2 * m + 1) * half) : 0u;
        const bool ina = m < np && q < half, inb = m < np && q < lb;
        const uint32_t ia = ina ? m * N + q : 0u, ib = inb ? m * N + half + q : 0u;
        xa[i] = ina ? X[ia] : 0u;
        xb[i] = inb ? X[ib] : 0u;
      }
#pragma unroll
      for (int i = 0; i < 16; i++) {
        const uint32_t s = lt + i * FT_PART;
        lds[lds_pad(s)] = reduce_limb(xa[i], p);
        lds[lds_pad(FT_SLOTS + s)] = reduce_limb(xb[i], p);
      }
    }
    __syncthreads();
    fused_transform(lds, logN, ft.scale[j - ft.j0][prime], pc, tws, itws, lt);
    fused_carry(
        buf, logN, tid,
        [&](uint32_t m) -> uint32_t { return m < np ? half + min(half, Kt - (2 * m + 1) * half) : 0u; },
        [&](uint32_t m, uint32_t k, uint32_t limb) { X[m * N + k] = limb; }, wpair, &bad);
    __syncthreads();   // X complete; the tiles are free for the next level
  }
  if (bad) atomicOr(err, CAT_DEVERR_CARRY_OUT);
  for (uint32_t k = tid; k < Kt; k += FT_THREADS) out[gofs + k] = X[k];
}
