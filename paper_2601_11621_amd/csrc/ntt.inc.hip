// Exact big-integer products for the reconstruction phase (Sec. 3.2, Alg. 2):
// cyclic convolution modulo three 32-bit primes by number-theoretic transforms.
//
// Transform structure (all integer, in LDS):
//  * A length-S transform is split as S = R * (S/R) (R = 2^r <= 16): each
//    work item loads R elements at stride S/R, does a radix-R DFT in registers
//    (radix-2 decimation-in-frequency network with constant roots omega_16^i),
//    multiplies output k1 by omega_S^{j2*k1} and writes it back in place; the
//    R blocks of size S/R are then transformed the same way.  The first pass
//    takes radix 2^(log2 S mod 4) when that is not 0, every later pass radix 16.
//    Outputs come out in a fixed digit-reversed order, which the pointwise
//    product does not care about; the inverse runs the passes backwards with
//    inverse roots (decimation-in-time networks), which undoes the order.
//  * Products with N up to 2^14 can run entirely in one workgroup
//    (k_ntt_lds: tiles of 2^12, 2^13 or 2^14 slots per operand, one thread per
//    16 slots; small products share a 2^12 tile).
//  * Larger N = L_0 ... L_{P-1} * M with M = 2^8 .. 2^14 use Bailey's four-step
//    split (1990) applied recursively: k_pass_fwd transforms the strided
//    columns of one level of the split (packing limbs on the fly in the first)
//    and applies its twiddles; k_row transforms each M-point row of both
//    operands, multiplies them pointwise and inverse-transforms the row;
//    k_pass_inv undoes the column levels, the outermost writing exact residues.
//    Which form a length bucket takes, and its row and column-pass lengths,
//    come from the per-bucket schedule (defaults, or the autotuner's table).
//  * In-pass twiddles are (w, wq) Montgomery pairs in tables laid out so that
//    neighbouring lanes read neighbouring entries; the column-level twiddles
//    omega_S^{j*f} come from two small tables of omega_{2^27} powers.
// The residues of the three primes are then recombined by k_crt (Garner's
// method) into 96-bit coefficient values, summed into limbs and carried with
// a wave64 ballot carry-lookahead; blocks of one product are joined by a
// look-back over the preceding blocks inside the same launch.

__constant__ PrimeC c_primes[CAT_NPRIMES];
__constant__ CrtC c_crt;
// The second (lazy) prime set; its w16 / iw16 entries are Shoup pairs.
__constant__ PrimeC c_primes1[CAT_NPRIMES];
__constant__ CrtC c_crt1;
// AS: the prime set of a kernel (0: p in (2^31, 2^32), values reduced after
// every operation; 1: q < 2^30, lazy ranges as described in common.hpp)
template <int AS>
__device__ __forceinline__ const PrimeC& primec(uint32_t i) {
  if constexpr (AS == 0) return c_primes[i];
  else return c_primes1[i];
}
template <int AS>
__device__ __forceinline__ const CrtC& crtc() {
  if constexpr (AS == 0) return c_crt;
  else return c_crt1;
}
// largest transform of a prime set (log2): the column twiddles are powers of
// omega_{2^tw_logn}
template <int AS>
__host__ __device__ constexpr int tw_logn() { return AS == 0 ? CAT_MAX_LOGN : CAT_LAZY_MAX_LOGN; }
// twiddle product: Montgomery pair (set 0, exact) or Shoup pair (set 1, [0, 2q))
template <int AS>
__device__ __forceinline__ uint32_t tw_mul(uint32_t a, uint32_t w, uint32_t ws, uint32_t p) {
  if constexpr (AS == 0) return mul_tw(a, w, ws, p);
  else return shoup(a, w, ws, p);
}

// bit reversal of an r-bit index, compile-time
__host__ __device__ constexpr int brev_c(int x, int r) {
  int y = 0;
  for (int i = 0; i < r; i++) y |= ((x >> i) & 1) << (r - 1 - i);
  return y;
}

__host__ __device__ constexpr uint32_t lds_pad(uint32_t i) { return i + (i >> 4); }

// Radix-R DFT on registers, decimation in frequency: natural input, output
// y[k] in v[brev(k)].  Set 1: inputs and outputs in [0, 2q); a butterfly
// gives red(a + b) and (a - b + 2q) * w (the sum below 4q, the Shoup product
// below 2q).  TW (set 1): every output but v[0] is multiplied next by a
// twiddle (Shoup, any 32-bit input), so the last stage leaves those in
// [0, 4q) unreduced.
template <int LOGR, int AS = 0, bool TW = false, bool ZHI = false>
__device__ __forceinline__ void dft_fwd(uint32_t* v, const PrimeC& pc) {
  constexpr int R = 1 << LOGR;
  const uint32_t p = pc.p;
  const uint32_t p2 = 2 * p;
#pragma unroll
  for (int h = R / 2; h >= 1; h /= 2) {
#pragma unroll
    for (int s = 0; s < R; s += 2 * h) {
#pragma unroll
      for (int i = 0; i < h; i++) {
        uint32_t a = v[s + i], b = v[s + i + h];
        const int wi = i * (8 / h);   // omega_{2h}^i = omega_16^{i*8/h}
        if constexpr (ZHI) {
          if (h == R / 2) {
            // ZHI: the upper half of the input is zero (a zero-padded
            // operand), so the first stage gives a and a * w
            v[s + i + h] = (i == 0) ? a : tw_mul<AS>(a, pc.w16[wi], pc.w16q[wi], p);
            continue;
          }
        }
        if constexpr (AS == 0) {
          v[s + i] = add_mod(a, b, p);
          uint32_t d = sub_mod(a, b, p);
          if (i == 0) v[s + i + h] = d;
          else v[s + i + h] = mul_tw(d, pc.w16[wi], pc.w16q[wi], p);
        } else {
          const bool keep = TW && h == 1;   // the twiddle that follows reduces it
          v[s + i] = (keep && s + i != 0) ? a + b : red2(a + b, p2);
          const uint32_t t = a + (p2 - b);
          if (i == 0) v[s + i + h] = keep ? t : red2(t, p2);
          else v[s + i + h] = shoup(t, pc.w16[wi], pc.w16q[wi], p);
        }
      }
    }
  }
}

// Inverse: input y[k] in v[brev(k)], decimation in time with inverse roots,
// output x[j] (times R) in v[j].  Set 1: inputs and outputs in [0, 4q); a
// butterfly reduces a to [0, 2q), takes t = w b in [0, 2q) and gives a + t and
// a - t + 2q.  TW (set 1): every input but v[0] comes from a twiddle (Shoup,
// in [0, 2q)), so the first stage does not reduce those again.
template <int LOGR, int AS = 0, bool TW = false>
__device__ __forceinline__ void dft_inv(uint32_t* v, const PrimeC& pc) {
  constexpr int R = 1 << LOGR;
  const uint32_t p = pc.p;
  const uint32_t p2 = 2 * p;
#pragma unroll
  for (int h = 1; h < R; h *= 2) {
#pragma unroll
    for (int s = 0; s < R; s += 2 * h) {
#pragma unroll
      for (int i = 0; i < h; i++) {
        uint32_t a = v[s + i], b = v[s + i + h];
        const int wi = i * (8 / h);
        if constexpr (AS == 0) {
          uint32_t t = (i == 0) ? b : mul_tw(b, pc.iw16[wi], pc.iw16q[wi], p);
          v[s + i] = add_mod(a, t, p);
          v[s + i + h] = sub_mod(a, t, p);
        } else {
          const bool fresh = TW && h == 1;   // inputs straight from the twiddles
          if (!(fresh && s + i != 0)) a = red2(a, p2);
          const uint32_t t = (i == 0) ? (fresh ? b : red2(b, p2)) : shoup(b, pc.iw16[wi], pc.iw16q[wi], p);
          v[s + i] = a + t;
          v[s + i + h] = a + (p2 - t);
        }
      }
    }
  }
}

// One forward pass of radix R over an LDS tile of `ngroups*R` elements laid out
// as element e of column c at (e << logC) + c (logC = 0: a plain vector).
// The elements form consecutive sub-problems of size S = R << logSR.
// tw: table of this pass, tw[(k1 << logSR) + j2] = omega_S^{j2*k1}.
// A thread handles U groups at once (g, g + blockDim, ...) so that the loads
// of one overlap the arithmetic of the other.
//
// Addressing: element j1 of a group sits at base + j1 * stride with a stride
// that is the same for the whole pass.  Unpadded, stride = 2^(logSR + logC).
// Padded (PAD, used with logC = 0 only), index i sits at i + i/16; every pass
// has logSR = 0 or a multiple of 4 (the passes after the first have radix 16
// and the first takes logS mod 4), so i/16 grows by 2^logSR/16 per step of j1
// (or by 0 when logSR = 0 and the 16 elements are one aligned run) and the
// padded index is linear in j1 as well.  The twiddle of (k1, j2) is read at a
// per-pass base (k1 << logSR), uniform across the workgroup, plus the lane's
// j2: one 32-bit offset per group serves all R - 1 reads.
__device__ __forceinline__ uint32_t pass_stride(bool pad, uint32_t logSR, uint32_t logC) {
  return pad ? (1u << logSR) + ((1u << logSR) >> 4) : (1u << (logSR + logC));
}

template <int LOGR, bool PAD>
__device__ __forceinline__ uint32_t group_base(uint32_t g, uint32_t logSR, uint32_t logC, uint32_t* jj) {
  const uint32_t h = g >> logC;
  const uint32_t j = h & ((1u << logSR) - 1);
  *jj = j;
  const uint32_t e0 = ((h >> logSR) << (logSR + LOGR)) + j;
  return PAD ? lds_pad(e0) : (e0 << logC) + (g & ((1u << logC) - 1));
}

// The twiddle reads go through a raw buffer resource over the pass table
// (kept in scalar registers: the table pointer is the same for a whole wave),
// with the uniform part (k1 << logSR) as the scalar offset and the lane's j2
// as the vector offset, so no per-read 64-bit address arithmetic is spent.
// Word 3 of the gfx9 descriptor: 32-bit data format, which untyped loads use
// for nothing but the range check against the table size.
#define CAT_BUF_DW3 0x00020000
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tw_rsrc(const uint2* tw, uint32_t entries) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)tw, (short)0, (int)(entries * (uint32_t)sizeof(uint2)), CAT_BUF_DW3);
}
__device__ __forceinline__ uint2 tw_at(__amdgpu_buffer_rsrc_t rs, uint32_t k1, uint32_t logSR, uint32_t jo) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, jo, (int)((k1 << logSR) * (uint32_t)sizeof(uint2)), 0);
  return make_uint2(v[0], v[1]);
}

// Word arrays read and written through raw buffer resources with byte
// offsets in one VGPR: loads past the array's end return 0 and stores there
// are dropped (the range check of an unswizzled buffer), which the column
// kernels use for the zero padding of their operands and the end of a product.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t words_rsrc(const uint32_t* p, uint64_t words) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(uint32_t)(words * 4u), CAT_BUF_DW3);
}
__device__ __forceinline__ uint32_t buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t byte_off, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)byte_off, 0, 0);
}

template <int LOGR, bool PAD, int U, int AS, bool ZHI = false>
__device__ __forceinline__ void groups_fwd(uint32_t* lds, uint32_t g0, uint32_t nthr, uint32_t logSR, uint32_t logC,
                                           const uint2* __restrict__ tw, const PrimeC& pc) {
  constexpr int R = 1 << LOGR;
  const uint32_t stride = pass_stride(PAD, logSR, logC);
  uint32_t v[U][R];
  uint32_t b[U], jj[U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    b[u] = group_base<LOGR, PAD>(g0 + u * nthr, logSR, logC, &jj[u]);
#pragma unroll
    for (int j1 = 0; j1 < R; j1++) v[u][j1] = (ZHI && j1 >= R / 2) ? 0u : lds[b[u] + j1 * stride];
  }
  // (j2 = 0 reads the pair of 1, which multiplies exactly: no divergent
  // branch around the twiddles)
#pragma unroll
  for (int u = 0; u < U; u++) {
    if (logSR > 0) {
      dft_fwd<LOGR, AS, true, ZHI>(v[u], pc);
      const uint32_t jo = jj[u] * (uint32_t)sizeof(uint2);
      const __amdgpu_buffer_rsrc_t rs = tw_rsrc(tw, (uint32_t)R << logSR);
#pragma unroll
      for (int k1 = 1; k1 < R; k1++) {
        const uint2 t = tw_at(rs, (uint32_t)k1, logSR, jo);
        const int r = brev_c(k1, LOGR);
        v[u][r] = tw_mul<AS>(v[u][r], t.x, t.y, pc.p);
      }
    } else {
      dft_fwd<LOGR, AS, false, ZHI>(v[u], pc);
    }
  }
#pragma unroll
  for (int u = 0; u < U; u++) {
#pragma unroll
    for (int k1 = 0; k1 < R; k1++) lds[b[u] + k1 * stride] = v[u][brev_c(k1, LOGR)];
  }
}

template <int LOGR, bool PAD, int U, int AS>
__device__ __forceinline__ void groups_inv(uint32_t* lds, uint32_t g0, uint32_t nthr, uint32_t logSR, uint32_t logC,
                                           const uint2* __restrict__ itw, const PrimeC& pc) {
  constexpr int R = 1 << LOGR;
  const uint32_t stride = pass_stride(PAD, logSR, logC);
  uint32_t v[U][R];
  uint32_t b[U], jj[U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    b[u] = group_base<LOGR, PAD>(g0 + u * nthr, logSR, logC, &jj[u]);
#pragma unroll
    for (int k1 = 0; k1 < R; k1++) v[u][brev_c(k1, LOGR)] = lds[b[u] + k1 * stride];
  }
#pragma unroll
  for (int u = 0; u < U; u++) {
    if (logSR > 0) {
      const uint32_t jo = jj[u] * (uint32_t)sizeof(uint2);
      const __amdgpu_buffer_rsrc_t rs = tw_rsrc(itw, (uint32_t)R << logSR);
#pragma unroll
      for (int k1 = 1; k1 < R; k1++) {
        const uint2 t = tw_at(rs, (uint32_t)k1, logSR, jo);
        const int r = brev_c(k1, LOGR);
        v[u][r] = tw_mul<AS>(v[u][r], t.x, t.y, pc.p);
      }
      dft_inv<LOGR, AS, true>(v[u], pc);
    } else {
      dft_inv<LOGR, AS, false>(v[u], pc);
    }
  }
#pragma unroll
  for (int u = 0; u < U; u++) {
#pragma unroll
    for (int j1 = 0; j1 < R; j1++) lds[b[u] + j1 * stride] = v[u][j1];
  }
}

// Thread `tid` of the `nthr` threads that share the tile (the workgroup, or
// one prime's part of a workgroup that holds several tiles).
template <int LOGR, bool PAD, int AS, bool ZHI = false>
__device__ __forceinline__ void pass_fwd(uint32_t* lds, uint32_t ngroups, uint32_t logSR, uint32_t logC,
                                         const uint2* __restrict__ tw, const PrimeC& pc, uint32_t tid,
                                         uint32_t nthr) {
  uint32_t g = tid;
  for (; g + nthr < ngroups; g += 2 * nthr) groups_fwd<LOGR, PAD, 2, AS, ZHI>(lds, g, nthr, logSR, logC, tw, pc);
  for (; g < ngroups; g += nthr) groups_fwd<LOGR, PAD, 1, AS, ZHI>(lds, g, nthr, logSR, logC, tw, pc);
}

template <int LOGR, bool PAD, int AS>
__device__ __forceinline__ void pass_inv(uint32_t* lds, uint32_t ngroups, uint32_t logSR, uint32_t logC,
                                         const uint2* __restrict__ itw, const PrimeC& pc, uint32_t tid,
                                         uint32_t nthr) {
  uint32_t g = tid;
  for (; g + nthr < ngroups; g += 2 * nthr) groups_inv<LOGR, PAD, 2, AS>(lds, g, nthr, logSR, logC, itw, pc);
  for (; g < ngroups; g += nthr) groups_inv<LOGR, PAD, 1, AS>(lds, g, nthr, logSR, logC, itw, pc);
}

// radix of the pass at sub-problem size 2^logS
__host__ __device__ constexpr int pass_logr(int logS) { return (logS % 4) ? (logS % 4) : 4; }
// offset of the table of size 2^s inside a per-prime pass-table block
__host__ __device__ constexpr uint32_t tws_off(int s) { return (1u << s) - 2u; }
#define CAT_LDS_MAX_LOGT 14  // largest transform held by one workgroup (both operands, 2^14 each)
#define TWS_ENTRIES 32766u   // sum over s = 1..14 of 2^s

// Synchronisation between two radix-16 passes.  Both have total/16 groups,
// and the 2^logSmall elements of a sub-problem of the smaller size are written
// and read by the same 2^logSmall consecutive groups, i.e. consecutive
// threads; in a plain vector (logC = 0) with 2^logSmall <= 64 those sit in one
// wave, which orders its own LDS traffic, so no workgroup barrier is needed.
// (Next to a pass of smaller radix the group counts differ: full barrier.)
__device__ __forceinline__ void pass_sync(int logSmall, uint32_t logC) {
  if (logC == 0 && logSmall <= 6) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Full forward transform of size 2^logS on every sub-problem of an LDS tile
// with `total` elements (all columns), passes from size 2^logS down.  On
// return (logC = 0) thread g of the last pass holds the outputs at
// [16 g, 16 g + 16) of its groups; the caller synchronises before other
// threads read them.
// zhi: the upper half of every sub-problem is zero (zero-padded operands):
// the first pass reads only the lower half and its first stage multiplies.
template <bool PAD, int AS = 0>
__device__ __forceinline__ void ntt_fwd_tile(uint32_t* lds, int logS, uint32_t total, uint32_t logC,
                             const uint2* __restrict__ tws, const PrimeC& pc, uint32_t tid = threadIdx.x,
                             uint32_t nthr = blockDim.x, bool zhi = false, int stop = 0) {
  // stop = 4: the last pass (sub-problems of 16) is left to the caller, after
  // the synchronisation before it
  bool firstp = true;
  while (logS > stop) {
    const int lr = pass_logr(logS);
    const uint32_t ng = total >> lr;
    const uint32_t logSR = (uint32_t)(logS - lr);
    const uint2* tw = tws + tws_off(logS);
    if (firstp && zhi) {
      switch (lr) {
        case 1: pass_fwd<1, PAD, AS, true>(lds, ng, logSR, logC, tw, pc, tid, nthr); break;
        case 2: pass_fwd<2, PAD, AS, true>(lds, ng, logSR, logC, tw, pc, tid, nthr); break;
        case 3: pass_fwd<3, PAD, AS, true>(lds, ng, logSR, logC, tw, pc, tid, nthr); break;
        default: pass_fwd<4, PAD, AS, true>(lds, ng, logSR, logC, tw, pc, tid, nthr); break;
      }
    } else {
      switch (lr) {
        case 1: pass_fwd<1, PAD, AS>(lds, ng, logSR, logC, tw, pc, tid, nthr); break;
        case 2: pass_fwd<2, PAD, AS>(lds, ng, logSR, logC, tw, pc, tid, nthr); break;
        case 3: pass_fwd<3, PAD, AS>(lds, ng, logSR, logC, tw, pc, tid, nthr); break;
        default: pass_fwd<4, PAD, AS>(lds, ng, logSR, logC, tw, pc, tid, nthr); break;
      }
    }
    firstp = false;
    logS -= lr;
    if (logS > 0) {
      if (lr == 4) pass_sync(logS, logC);   // every later pass has radix 16
      else __syncthreads();
    }
  }
}

// Inverse; the caller synchronises before the first pass as needed (with
// logC = 0 the first pass reads [16 g, 16 g + 16) in thread g) and the
// transform ends with a workgroup barrier.
template <bool PAD, int AS = 0>
__device__ __forceinline__ void ntt_inv_tile(uint32_t* lds, int logS, uint32_t total, uint32_t logC,
                             const uint2* __restrict__ itws, const PrimeC& pc, uint32_t tid = threadIdx.x,
                             uint32_t nthr = blockDim.x, int ls0 = 4) {
  // passes in the reverse order of ntt_fwd_tile: the radix-16 passes of sizes
  // 2^4, 2^8, ... first, the (possibly smaller-radix) pass of size 2^logS last
  // (ls0 = 8: the caller did the pass of size 2^4 and synchronised after it)
  const int lr0 = pass_logr(logS);
  for (int ls = ls0; ls <= logS - lr0; ls += 4) {
    pass_inv<4, PAD, AS>(lds, total >> 4, (uint32_t)(ls - 4), logC, itws + tws_off(ls), pc, tid, nthr);
    if (ls + 4 <= logS - lr0 || lr0 == 4) pass_sync(ls, logC);   // the next pass has radix 16
    else __syncthreads();
  }
  if (logS > 0) {
    const uint32_t ng = total >> lr0;
    const uint32_t logSR = (uint32_t)(logS - lr0);
    const uint2* tw = itws + tws_off(logS);
    switch (lr0) {
      case 1: pass_inv<1, PAD, AS>(lds, ng, logSR, logC, tw, pc, tid, nthr); break;
      case 2: pass_inv<2, PAD, AS>(lds, ng, logSR, logC, tw, pc, tid, nthr); break;
      case 3: pass_inv<3, PAD, AS>(lds, ng, logSR, logC, tw, pc, tid, nthr); break;
      default: pass_inv<4, PAD, AS>(lds, ng, logSR, logC, tw, pc, tid, nthr); break;
    }
  }
  __syncthreads();
}

// frequency held at output position q of the pass-structured transform of size 2^logS
__device__ __forceinline__ uint32_t out_freq(uint32_t q, int logS) {
  uint32_t f = 0, mult = 1;
  while (logS > 0) {
    const int r = pass_logr(logS);
    const int rest = logS - r;
    const uint32_t k1 = q >> rest;
    f += k1 * mult;
    mult <<= r;
    q &= (1u << rest) - 1;
    logS = rest;
  }
  return f;
}

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2) in
// the order of their linear index.  Neighbouring column tiles share cache
// lines (a tile row is C words), so block b of a grid of G is renumbered to
// put consecutive tiles on one XCD: XCD x gets the tiles
// [x ceil(G/8), ...) in order (a bijection of [0, G) for any G).
#define CAT_XCDS 8
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t G) {
  const uint32_t q = G / CAT_XCDS, r = G % CAT_XCDS;
  const uint32_t x = b % CAT_XCDS, k = b / CAT_XCDS;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

struct NttTables {
  const uint2* tws;       // [prime][TWS_ENTRIES] forward pass tables
  const uint2* itws;      // [prime][TWS_ENTRIES] inverse
  const uint2* tw2lo;     // [prime][2^14] omega_{2^27}^i, Montgomery pairs
  const uint32_t* tw2hi;  // [prime][2^13] omega_{2^27}^{i*2^14}, Montgomery form
  const uint2* itw2lo;    // inverse roots
  const uint32_t* itw2hi;
};

// A limb entering a transform: reduced (set 0) or brought into [0, 2q) (set 1).
template <int AS>
__device__ __forceinline__ uint32_t in_limb(uint32_t x, uint32_t p) {
  if constexpr (AS == 0) return reduce_limb(x, p);
  else return limb_lazy(x, p);
}
// Pointwise product of two forward outputs times the scale pair sc (2^32/N):
// exact (set 0) or in (0, 2q) (set 1).
template <int AS>
__device__ __forceinline__ uint32_t pointwise(uint32_t x, uint32_t y, uint2 sc, const PrimeC& pc) {
  if constexpr (AS == 0) return mul_tw(mont_mul(x, y, pc.p, pc.pinv), sc.x, sc.y, pc.p);
  else return mont_lazy(mont_mul_lazy(x, y, pc.p, pc.pinv), sc.x, sc.y, pc.p);
}
// Data times a computed twiddle (Montgomery pair, fully reduced): exact
// (set 0) or in (0, 2q) for any 32-bit input (set 1).
template <int AS>
__device__ __forceinline__ uint32_t data_tw(uint32_t x, uint2 w, uint32_t p) {
  if constexpr (AS == 0) return mul_tw(x, w.x, w.y, p);
  else return mont_lazy(x, w.x, w.y, p);
}
// Pointwise product without the scale (the row kernel applies it with the
// inverse twiddles): x y / 2^32, exact (set 0) or in (0, 2q) (set 1).
template <int AS>
__device__ __forceinline__ uint32_t pointwise_raw(uint32_t x, uint32_t y, const PrimeC& pc) {
  if constexpr (AS == 0) return mont_mul(x, y, pc.p, pc.pinv);
  else return mont_mul_lazy(x, y, pc.p, pc.pinv);
}

// The innermost passes around the pointwise product on registers: thread g
// holds the forward sub-problems of 16 at [16 g, 16 g + 16) of A and of B
// (the groups of the last forward pass, logSR = 0), takes both DFTs, the
// pointwise product (in the outputs' bit-reversed order, which both share)
// and the inverse DFT of the first inverse pass, and writes that group back:
// the two passes and the product without their LDS round trips.  SCALED:
// pointwise with the scale pair (the one-workgroup kernel), else the raw
// product (the row kernel, whose inverse twiddles carry the scale).
template <int AS, bool SCALED>
__device__ __forceinline__ void mid_passes(uint32_t* lds, uint32_t a0, uint32_t b0, uint2 sc, const PrimeC& pc) {
  uint32_t x[16], y[16];
#pragma unroll
  for (int k = 0; k < 16; k++) {
    x[k] = lds[a0 + k];
    y[k] = lds[b0 + k];
  }
  dft_fwd<4, AS, false, false>(x, pc);
  dft_fwd<4, AS, false, false>(y, pc);
#pragma unroll
  for (int k = 0; k < 16; k++) x[k] = SCALED ? pointwise<AS>(x[k], y[k], sc, pc) : pointwise_raw<AS>(x[k], y[k], pc);
  dft_inv<4, AS, false>(x, pc);
#pragma unroll
  for (int k = 0; k < 16; k++) lds[a0 + k] = x[k];
}

// An inverse-transform output leaving as a residue in [0, p).
template <int AS>
__device__ __forceinline__ uint32_t out_residue(uint32_t x, uint32_t p) {
  if constexpr (AS == 0) return x;
  else return red4(x, p);
}

// ---------------------------------------------------------------------------
// Whole product in one workgroup, N = 2^logN <= 2^LOGT <= 2^14.
// Writes res[prime][r_off + j] = (a*b)_j mod p for j < la+lb.
// Tile of 2^LOGT coefficient slots (T/N products), 2^LOGT/16 threads, so every
// radix-16 pass gives each thread two groups over the two operands.
// BMODE 0: both operands per product.  BMODE 1 and 2 serve a stage whose
// second operand is one array for every product: mode 1, launched with one
// workgroup per prime, leaves its transform in fb[prime][0 .. N); mode 2
// loads that beside each first operand and transforms only the latter.  The
// grid
// is 3 x tiles workgroups; workgroup ids are renumbered so that each XCD takes
// a contiguous run of (tile, prime) pairs: the three primes of a tile run one
// after another on one XCD and read the operands once from HBM into its L2.
// First forward and last inverse pass of a packed tile on registers: the
// tile's products lie back to back as a then b (N/2 words each), and thread
// t of the NT loaded the words t + NT i, i < 16.  With a first pass of radix
// 2^LR = 2^pass_logr(logN) over positions j + 2^logSR k (logSR = logN - LR,
// 2^logSR = D NT), the lower half of its group (block b = 2 m + o, j = t +
// NT d) is the loaded words i = b 2^(LR-1) D + d + D k, the upper half zero;
// of the last inverse pass it holds the groups (product m, j = t + NT d),
// whose outputs k are its stored words i = m 2^LR D + d + D k.  Same
// arithmetic as groups_fwd (with ZHI) and groups_inv.
template <int LR, int D, int AS>
__device__ __forceinline__ void lds_first_fwd(uint32_t* lds, const uint32_t* x, uint32_t NT, uint32_t N, uint32_t TT,
                                              uint32_t cnt, const uint2* __restrict__ tw, const PrimeC& pc) {
  constexpr int R = 1 << LR, H = R / 2, NB = 16 / (H * D);
  const uint32_t SR = NT * D, stride = SR + SR / 16, logSR = 31 - __builtin_clz(SR);
  const __amdgpu_buffer_rsrc_t rt = tw_rsrc(tw, (uint32_t)R << logSR);
#pragma unroll
  for (int b = 0; b < NB; b++) {
    if ((uint32_t)(b >> 1) >= cnt) continue;
#pragma unroll
    for (int d = 0; d < D; d++) {
      uint32_t v[R];
#pragma unroll
      for (int k = 0; k < R; k++) v[k] = k < H ? x[b * H * D + d + D * k] : 0u;
      dft_fwd<LR, AS, true, true>(v, pc);
      const uint32_t j = threadIdx.x + NT * d;
      const uint32_t jo = j * (uint32_t)sizeof(uint2);
#pragma unroll
      for (int k1 = 1; k1 < R; k1++) {
        const uint2 t = tw_at(rt, (uint32_t)k1, logSR, jo);
        const int r = brev_c(k1, LR);
        v[r] = tw_mul<AS>(v[r], t.x, t.y, pc.p);
      }
      const uint32_t base = lds_pad(((b & 1) ? TT : 0u) + (uint32_t)(b >> 1) * N + j);
#pragma unroll
      for (int k1 = 0; k1 < R; k1++) lds[base + k1 * stride] = v[brev_c(k1, LR)];
    }
  }
}
template <int LR, int D, int AS>
__device__ __forceinline__ void lds_last_inv(const uint32_t* lds, uint32_t* dst, uint32_t NT, uint32_t N, uint32_t T,
                                             const uint2* __restrict__ itw, const PrimeC& pc) {
  constexpr int R = 1 << LR, NP = 16 / (R * D);
  const uint32_t SR = NT * D, stride = SR + SR / 16, logSR = 31 - __builtin_clz(SR);
  const __amdgpu_buffer_rsrc_t rt = tw_rsrc(itw, (uint32_t)R << logSR);
#pragma unroll
  for (int m = 0; m < NP; m++) {
    if ((uint32_t)m * N >= T) continue;
#pragma unroll
    for (int d = 0; d < D; d++) {
      const uint32_t j = threadIdx.x + NT * d;
      const uint32_t base = lds_pad((uint32_t)m * N + j);
      uint32_t v[R];
#pragma unroll
      for (int k1 = 0; k1 < R; k1++) v[brev_c(k1, LR)] = lds[base + k1 * stride];
      const uint32_t jo = j * (uint32_t)sizeof(uint2);
#pragma unroll
      for (int k1 = 1; k1 < R; k1++) {
        const uint2 t = tw_at(rt, (uint32_t)k1, logSR, jo);
        const int r = brev_c(k1, LR);
        v[r] = tw_mul<AS>(v[r], t.x, t.y, pc.p);
      }
      dft_inv<LR, AS, true>(v, pc);
#pragma unroll
      for (int k = 0; k < R; k++) dst[threadIdx.x + NT * (m * R * D + d + D * k)] = out_residue<AS>(v[k], pc.p);
    }
  }
}

template <int LOGT, int BMODE, int AS>
__global__ void __launch_bounds__((1 << LOGT) / 16)
k_ntt_lds(DescView dv, uint64_t nmul, int logN, const uint32_t* __restrict__ ain, const uint32_t* __restrict__ bin,
          uint32_t* __restrict__ res, uint64_t res_stride, NttTables tb, uint2 scale0, uint2 scale1, uint2 scale2,
          uint32_t* __restrict__ fb) {
  constexpr uint32_t TT = 1u << LOGT;
  __shared__ uint32_t lds[lds_pad(2 * TT)];
  __shared__ MulDesc ds[64];
  const uint32_t wid = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t prime = wid % CAT_NPRIMES;
  const PrimeC& pc = primec<AS>(prime);
  const uint32_t p = pc.p;
  const uint32_t N = 1u << logN;
  const uint32_t per = TT >> logN;                 // products per tile (<= 64)
  const uint64_t m0 = (uint64_t)(wid / CAT_NPRIMES) * per;
  const uint32_t cnt = (uint32_t)min((uint64_t)per, nmul - m0);
  for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) ds[i] = dv.get(m0 + i);
  __syncthreads();
  const uint32_t T = cnt << logN;                  // live slots
  const uint2* tws = tb.tws + (size_t)prime * TWS_ENTRIES;
  const uint2* itws = tb.itws + (size_t)prime * TWS_ENTRIES;
  // A second operand that is the same for every product (the power P_j of a
  // decimal join): BMODE 1 (one workgroup per prime) transforms it once and
  // stores the N words as they stand in LDS to fb[prime][.]; BMODE 2 loads
  // them into every product's slot and transforms only the first operands.
  if constexpr (BMODE == 1) {
    const MulDesc d = ds[0];
    for (uint32_t t = threadIdx.x; t < N; t += blockDim.x)
      lds[lds_pad(t)] = in_limb<AS>(t < d.lb ? bin[d.b_off + t] : 0u, p);
    __syncthreads();
    ntt_fwd_tile<true, AS>(lds, logN, N, 0, tws, pc);
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < N; t += blockDim.x) fb[(size_t)prime * N + t] = lds[lds_pad(t)];
    return;
  }
  // Packed tiles (every tree level): the tile's products have la = lb = N/2
  // and lie back to back, a then b, in one array, with their residues at the
  // same relative positions, so the tile reads T consecutive words and writes
  // T consecutive residues
  bool packed = false;
  if constexpr (BMODE == 0) {
    bool ok = true;
    if (threadIdx.x < cnt) {
      const MulDesc d = ds[threadIdx.x], d0 = ds[0];
      const uint64_t rel = (uint64_t)threadIdx.x << logN;
      ok = d.la == (N >> 1) && d.lb == (N >> 1) && d.a_off == d0.a_off + rel && d.b_off == d.a_off + (N >> 1) &&
           d.r_off == d0.r_off + rel;
    }
    packed = __syncthreads_and(ok ? 1 : 0) != 0 && ain == bin;
  }
  // 2^12-slot packed tiles of transforms of 2^9 .. 2^12 points: the first
  // forward pass (radix 2^lr, groups of positions j + 256 k) and the last
  // inverse pass run on registers, since a thread's loaded and stored words
  // are exactly its groups of those passes
  constexpr uint32_t NTL = TT / 16;                // blockDim.x
  // (2^12 tiles: transforms of 2^9 .. 2^12 points; 2^13: 2^13; 2^14: 2^13
  // and 2^14, where 2^(logN - pass_logr(logN)) is a multiple of the thread
  // count)
  const bool regp = BMODE == 0 && packed &&
                    (LOGT == 12 ? logN >= 9 : LOGT == 13 ? logN == 13 : LOGT == 14 ? logN >= 13 : false);
  const int logSR1 = logN - pass_logr(logN);
  if (regp) {
    const uint32_t* src = ain + ds[0].a_off;
    uint32_t x[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const uint32_t w = threadIdx.x + i * NTL;
      x[i] = in_limb<AS>(src[w < T ? w : T - 1], p);
    }
    const uint2* tw1 = tws + tws_off(logN);
    if constexpr (LOGT == 12) {
      switch (logN) {
        case 9: lds_first_fwd<1, 1, AS>(lds, x, NTL, N, TT, cnt, tw1, pc); break;
        case 10: lds_first_fwd<2, 1, AS>(lds, x, NTL, N, TT, cnt, tw1, pc); break;
        case 11: lds_first_fwd<3, 1, AS>(lds, x, NTL, N, TT, cnt, tw1, pc); break;
        default: lds_first_fwd<4, 1, AS>(lds, x, NTL, N, TT, cnt, tw1, pc); break;
      }
    } else if constexpr (LOGT == 13) {
      lds_first_fwd<1, 8, AS>(lds, x, NTL, N, TT, cnt, tw1, pc);
    } else if constexpr (LOGT == 14) {
      if (logN == 13) lds_first_fwd<1, 4, AS>(lds, x, NTL, N, TT, cnt, tw1, pc);
      else lds_first_fwd<2, 4, AS>(lds, x, NTL, N, TT, cnt, tw1, pc);
    }
  } else if (packed) {
    constexpr uint32_t NT = TT / 16;               // blockDim.x
    const uint32_t* src = ain + ds[0].a_off;
    const uint32_t half = N >> 1;
    uint32_t x[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const uint32_t w = threadIdx.x + i * NT;
      x[i] = src[w < T ? w : T - 1];
    }
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const uint32_t w = threadIdx.x + i * NT;
      if (w < T) {
        // word w: product w / N, operand bit logN - 1 of w, position w mod N/2
        const uint32_t dst = ((w >> (logN - 1)) & 1u ? TT : 0u) + (w & ~(N - 1)) + (w & (half - 1));
        lds[lds_pad(dst)] = in_limb<AS>(x[i], p);
        lds[lds_pad(dst + half)] = 0u;
      }
    }
  } else {
    // every load of the thread is issued before the first is used: clamped,
    // in-bounds addresses and masks instead of branches around the loads
    constexpr uint32_t NT = TT / 16;               // blockDim.x
    uint32_t xa[16], xb[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const uint32_t t = threadIdx.x + i * NT;
      const uint32_t tc = t < T ? t : T - 1;
      const uint32_t m = tc >> logN, j = tc & (N - 1);
      const MulDesc d = ds[m];
      const uint32_t ka = j < d.la ? 0xFFFFFFFFu : 0u, kb = j < d.lb ? 0xFFFFFFFFu : 0u;
      xa[i] = ain[d.a_off + (j & ka)] & ka;
      if constexpr (BMODE == 2)
        xb[i] = fb[(size_t)prime * N + j];
      else
        xb[i] = bin[d.b_off + (j & kb)] & kb;
    }
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const uint32_t t = threadIdx.x + i * NT;
      lds[lds_pad(t)] = in_limb<AS>(xa[i], p);
      lds[lds_pad(TT + t)] = BMODE == 2 ? xb[i] : in_limb<AS>(xb[i], p);
    }
  }
  // slots past T of a partial tile repeat the last live slot; their
  // sub-problems are independent and never read back
  __syncthreads();
  // A occupies [0, T), B [TT, TT + T); transform both as one tile
  if constexpr (BMODE == 2) {
    ntt_fwd_tile<true, AS>(lds, logN, T, 0, tws, pc);
  } else if (regp) {
    // the passes after the first but the last
    if (T == TT) {
      ntt_fwd_tile<true, AS>(lds, logSR1, 2 * TT, 0, tws, pc, threadIdx.x, blockDim.x, false, 4);
    } else {
      ntt_fwd_tile<true, AS>(lds, logSR1, T, 0, tws, pc, threadIdx.x, blockDim.x, false, 4);
      ntt_fwd_tile<true, AS>(lds + lds_pad(TT), logSR1, T, 0, tws, pc, threadIdx.x, blockDim.x, false, 4);
    }
  } else if (T == TT) {
    ntt_fwd_tile<true, AS>(lds, logN, 2 * TT, 0, tws, pc, threadIdx.x, blockDim.x, packed);
  } else {
    ntt_fwd_tile<true, AS>(lds, logN, T, 0, tws, pc, threadIdx.x, blockDim.x, packed);
    ntt_fwd_tile<true, AS>(lds + lds_pad(TT), logN, T, 0, tws, pc, threadIdx.x, blockDim.x, packed);
  }
  // pointwise product on the 16 positions whose forward outputs this thread
  // wrote last (A and B alike), which the first inverse pass reads back in the
  // same thread: no barrier on either side
  const uint2 sc = prime == 0 ? scale0 : (prime == 1 ? scale1 : scale2);
  if (regp) {
    // with the last forward pass and the first inverse pass on registers
    if (16 * threadIdx.x < T) mid_passes<AS, true>(lds, lds_pad(16 * threadIdx.x), lds_pad(TT + 16 * threadIdx.x), sc, pc);
    pass_sync(4, 0);
  } else if (16 * threadIdx.x < T) {
#pragma unroll
    for (int k = 0; k < 16; k++) {
      const uint32_t t = 16 * threadIdx.x + k;
      const uint32_t x = lds[lds_pad(t)], y = lds[lds_pad(TT + t)];
      lds[lds_pad(t)] = pointwise<AS>(x, y, sc, pc);
    }
  }
  uint32_t* out = res + (size_t)prime * res_stride;
  if (regp) {
    // every pass but the first and the last
    ntt_inv_tile<true, AS>(lds, logSR1, T, 0, itws, pc, threadIdx.x, blockDim.x, 8);
    uint32_t* dst = out + ds[0].r_off;
    const uint2* itw1 = itws + tws_off(logN);
    if constexpr (LOGT == 12) {
      switch (logN) {
        case 9: lds_last_inv<1, 1, AS>(lds, dst, NTL, N, T, itw1, pc); break;
        case 10: lds_last_inv<2, 1, AS>(lds, dst, NTL, N, T, itw1, pc); break;
        case 11: lds_last_inv<3, 1, AS>(lds, dst, NTL, N, T, itw1, pc); break;
        default: lds_last_inv<4, 1, AS>(lds, dst, NTL, N, T, itw1, pc); break;
      }
    } else if constexpr (LOGT == 13) {
      lds_last_inv<1, 8, AS>(lds, dst, NTL, N, T, itw1, pc);
    } else if constexpr (LOGT == 14) {
      if (logN == 13) lds_last_inv<1, 4, AS>(lds, dst, NTL, N, T, itw1, pc);
      else lds_last_inv<2, 4, AS>(lds, dst, NTL, N, T, itw1, pc);
    }
    return;
  }
  ntt_inv_tile<true, AS>(lds, logN, T, 0, itws, pc);
  if (packed) {
    constexpr uint32_t NT = TT / 16;
    uint32_t* dst = out + ds[0].r_off;
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const uint32_t t = threadIdx.x + i * NT;
      if (t < T) dst[t] = out_residue<AS>(lds[lds_pad(t)], p);
    }
    return;
  }
  for (uint32_t m = 0; m < cnt; m++) {
    const MulDesc d = ds[m];
    const uint32_t L = d.la + d.lb;
    for (uint32_t j = threadIdx.x; j < L; j += blockDim.x)
      out[d.r_off + j] = j < N ? out_residue<AS>(lds[lds_pad((m << logN) + j)], p) : 0u;
  }
}

// ---------------------------------------------------------------------------
// Large N: N = L_0 * L_1 * ... * L_{P-1} * M, M = 2^12 (Bailey's four-step,
// applied recursively).  Pass p works on contiguous sub-problems of size S_p
// (S_0 = N, S_{p+1} = S_p / L_p): the L_p-point DFT along the outermost
// dimension (stride sigma = S_p / L_p) of each sub-problem, then the twiddle
// omega_{S_p}^{j * f(q)} (j < sigma the inner index, f(q) the frequency at
// output position q).  The last M-point transforms (k_row) run on rows.
// A workgroup holds an L x C tile (C consecutive inner indices) in LDS.
// Scratch F: per product, per prime, per operand N words:
//   F[((m*3 + prime)*2 + op)*N + position]
#define NTT_COL_THREADS 256
// Column tiles hold 2^NTT_COL_LOGT words (32 KB, 4 workgroups per CU) on large
// stages and 2^NTT_COL_LOGT_SMALL on stages too small to fill the GPU (twice
// the workgroups, twice as many resident).
#define NTT_COL_LOGT 13
#define NTT_COL_LOGT_SMALL 12
#define NTT_COL_MAXL 10         // longest column DFT: 2^10 points
#define COL_BATCH 16            // global loads a thread keeps in flight in the column kernels
#define TW2_LO_BITS 14u
#define TW2_LO (1u << TW2_LO_BITS)
#define TW2_HI (1u << (CAT_MAX_LOGN - TW2_LO_BITS))

// omega_{2^27}^y (or its inverse) as a Montgomery pair from the two-level
// tables lo[y mod 2^14] (pairs) and hi[y >> 14] (Montgomery form).
__device__ __forceinline__ uint2 tw2(const uint2* __restrict__ lo, const uint32_t* __restrict__ hi, uint32_t y,
                                     const PrimeC& pc) {
  const uint2 l = lo[y & (TW2_LO - 1)];
  const uint32_t w = mul_tw(hi[y >> TW2_LO_BITS], l.x, l.y, pc.p);
  return make_uint2(w, w * pc.pinv);
}


struct PassGeom {
  int logN, logS, logL, logC;
  __device__ __forceinline__ void locate(uint64_t bx, uint64_t* m, uint64_t* base, uint32_t* j0) const {
    const int logSig = logS - logL;
    const uint64_t tiles = 1ull << (logSig - logC);          // tiles per sub-problem
    const uint64_t blocks = 1ull << (logN - logS);           // sub-problems per product
    *m = bx / (blocks * tiles);
    const uint64_t r = bx - *m * blocks * tiles;
    const uint64_t blk = r / tiles;
    *base = blk << logS;
    *j0 = (uint32_t)((r - blk * tiles) << logC);
  }
};

// The innermost column pass (sub-problems of 16 rows, logSR = 0) on
// registers: group threadIdx.x + 256 u of a tile of NV * 256 words (C =
// 2^logC <= 256 columns) holds rows 16 h .. 16 h + 15 of column c (h = g >>
// logC, c = g mod C).  Forward: the pass's outputs go straight to F, with the
// pass's own twiddles omega_S^(j f(q)) when tw (q the row, j = j0 + c);
// inverse: the pass's inputs come straight from F.  Same arithmetic as
// groups_fwd / groups_inv at logSR = 0.
template <int AS, int NV>
__device__ __forceinline__ void col_last_fwd_store(const uint32_t* lds, __amdgpu_buffer_rsrc_t rf, uint32_t cbase,
                                                   uint32_t rowB, uint32_t logC, int tw, uint32_t j0, int logL,
                                                   uint32_t ysh, const uint2* __restrict__ lo,
                                                   const uint32_t* __restrict__ hi, const PrimeC& pc) {
  const uint32_t C = 1u << logC;
#pragma unroll
  for (int u = 0; u < NV / 16; u++) {
    const uint32_t g = threadIdx.x + 256u * u;
    const uint32_t h = g >> logC, c = g & (C - 1);
    const uint32_t b = (h << (4 + logC)) + c;
    uint32_t x[16];
#pragma unroll
    for (int j1 = 0; j1 < 16; j1++) x[j1] = lds[b + j1 * C];
    dft_fwd<4, AS, false, false>(x, pc);
    const uint32_t ob = (cbase + c) * 4u;
#pragma unroll
    for (int k1 = 0; k1 < 16; k1++) {
      const uint32_t q = 16 * h + k1;
      uint32_t val = x[brev_c(k1, 4)];
      if (tw) {
        const uint32_t y = (((j0 + c) * out_freq(q, logL)) << ysh) & ((1u << tw_logn<AS>()) - 1);
        const uint2 l = lo[y & (TW2_LO - 1)];
        const uint32_t w = mul_tw(hi[y >> TW2_LO_BITS], l.x, l.y, pc.p);
        val = data_tw<AS>(val, make_uint2(w, w * pc.pinv), pc.p);
      }
      buf_st(rf, ob + q * rowB, val);
    }
  }
}
template <int AS, int NV>
__device__ __forceinline__ void col_first_inv_load(uint32_t* lds, __amdgpu_buffer_rsrc_t rf, uint32_t cbase,
                                                   uint32_t rowB, uint32_t logC, const PrimeC& pc) {
  const uint32_t C = 1u << logC;
  uint32_t v[NV / 16][16];
#pragma unroll
  for (int u = 0; u < NV / 16; u++) {
    const uint32_t g = threadIdx.x + 256u * u;
    const uint32_t h = g >> logC, c = g & (C - 1);
    const uint32_t ob = (cbase + c) * 4u + 16 * h * rowB;
#pragma unroll
    for (int k1 = 0; k1 < 16; k1++) v[u][brev_c(k1, 4)] = buf_ld(rf, ob + k1 * rowB);
  }
#pragma unroll
  for (int u = 0; u < NV / 16; u++) {
    const uint32_t g = threadIdx.x + 256u * u;
    const uint32_t h = g >> logC, c = g & (C - 1);
    const uint32_t b = (h << (4 + logC)) + c;
    dft_inv<4, AS, false>(v[u], pc);
#pragma unroll
    for (int j1 = 0; j1 < 16; j1++) lds[b + j1 * C] = v[u][j1];
  }
}

// The first forward column pass on registers for an operand of at most N/2
// words: in a tile of NV * 256 words and at most 256 columns, group
// threadIdx.x + 256 u of that pass (radix 2^LR) has its lower half at the
// elements threadIdx.x + 256 (u + j1 NV / 2^LR), j1 < 2^LR / 2, which are the
// thread's loaded values v[u + j1 NV / 2^LR]; the upper half is zero.  Same
// arithmetic as groups_fwd with ZHI.
template <int LR, int AS, int NV>
__device__ __forceinline__ void col_first_fwd(uint32_t* lds, const uint32_t* v, uint32_t logL, uint32_t logC,
                                              const uint2* __restrict__ tw, const PrimeC& pc) {
  constexpr int R = 1 << LR;
  constexpr int U = NV >> LR;
  const uint32_t logSR = logL - LR;
  const uint32_t stride = 1u << (logSR + logC);
#pragma unroll
  for (int u = 0; u < U; u++) {
    uint32_t jj;
    const uint32_t b = group_base<LR, false>(threadIdx.x + 256u * u, logSR, logC, &jj);
    uint32_t x[R];
#pragma unroll
    for (int j1 = 0; j1 < R; j1++) x[j1] = j1 < R / 2 ? v[u + j1 * U] : 0u;
    if (logSR > 0) {
      dft_fwd<LR, AS, true, true>(x, pc);
      const uint32_t jo = jj * (uint32_t)sizeof(uint2);
      const __amdgpu_buffer_rsrc_t rt = tw_rsrc(tw, (uint32_t)R << logSR);
#pragma unroll
      for (int k1 = 1; k1 < R; k1++) {
        const uint2 t = tw_at(rt, (uint32_t)k1, logSR, jo);
        const int r = brev_c(k1, LR);
        x[r] = tw_mul<AS>(x[r], t.x, t.y, pc.p);
      }
    } else {
      dft_fwd<LR, AS, false, true>(x, pc);
    }
#pragma unroll
    for (int k1 = 0; k1 < R; k1++) lds[b + k1 * stride] = x[brev_c(k1, LR)];
  }
}

template <int LOGT, int AS>
__global__ void __launch_bounds__(NTT_COL_THREADS)
k_pass_fwd(DescView dv, PassGeom pg, int first, int tw, int pre, int plogS, int plogL, int op_base,
           const uint32_t* __restrict__ ain, const uint32_t* __restrict__ bin, uint32_t* __restrict__ F,
           NttTables tb) {
  __shared__ uint32_t lds[1u << LOGT];
  // x: (tile, prime) pairs, XCD-contiguous; the three primes of a tile of the
  // first pass read the same operand words
  const uint32_t wid = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t prime = wid % CAT_NPRIMES, op = op_base + blockIdx.z;
  const PrimeC& pc = primec<AS>(prime);
  const uint32_t p = pc.p;
  uint64_t m, base;
  uint32_t j0;
  pg.locate(wid / CAT_NPRIMES, &m, &base, &j0);
  const int logSig = pg.logS - pg.logL;
  const uint32_t C = 1u << pg.logC;
  const uint64_t N = 1ull << pg.logN;
  const uint32_t T = 1u << (pg.logL + pg.logC);
  uint32_t* f = F + ((m * 3 + prime) * 2 + op) * N;
  // Tiles of at most 256 columns: element t = t0 + tid + 256 i of the tile
  // (row t >> logC, column t mod C) sits at the thread's byte offset off0 plus
  // a step that is the same for the whole workgroup; the sub-problem offsets
  // stay below N <= 2^27 words.
  const bool lin = pg.logC <= 8;
  const uint32_t RI = NTT_COL_THREADS >> (lin ? pg.logC : 0);   // rows per step of i
  const uint32_t rowB = 4u << logSig;                           // bytes per row
  const uint32_t off0 = ((uint32_t)base + ((threadIdx.x >> pg.logC) << logSig) + j0 + (threadIdx.x & (C - 1))) * 4u;
  // zhi: an operand of at most N/2 limbs leaves the lower half of the rows of
  // the first pass (rows L/2 .. L-1, tile elements T/2 .. T-1) zero, which
  // the first radix pass never reads
  bool zhi = false;
  if (first) {
    const MulDesc d0 = dv.get(m);
    zhi = (uint64_t)(op ? d0.lb : d0.la) <= (N >> 1);
  }
  const uint32_t Tl = zhi ? T >> 1 : T;
  // loads in batches of COL_BATCH per thread, all issued before the first use
  const bool regp = first && lin && zhi && T == (1u << LOGT);
  if (regp) {
    // the whole lower half in registers, the first pass on them
    constexpr int NV = (1 << LOGT) / NTT_COL_THREADS;
    const MulDesc d = dv.get(m);
    const __amdgpu_buffer_rsrc_t rs = words_rsrc(op ? bin + d.b_off : ain + d.a_off, op ? d.lb : d.la);
    uint32_t v[NV / 2];
#pragma unroll
    for (int i = 0; i < NV / 2; i++) v[i] = buf_ld(rs, off0 + i * RI * rowB);
#pragma unroll
    for (int i = 0; i < NV / 2; i++) v[i] = in_limb<AS>(v[i], p);
    const int lr = pass_logr(pg.logL);
    const uint2* tws = tb.tws + (size_t)prime * TWS_ENTRIES;
    const uint2* tw1 = tws + tws_off(pg.logL);
    switch (lr) {
      case 1: col_first_fwd<1, AS, NV>(lds, v, pg.logL, pg.logC, tw1, pc); break;
      case 2: col_first_fwd<2, AS, NV>(lds, v, pg.logL, pg.logC, tw1, pc); break;
      case 3: col_first_fwd<3, AS, NV>(lds, v, pg.logL, pg.logC, tw1, pc); break;
      default: col_first_fwd<4, AS, NV>(lds, v, pg.logL, pg.logC, tw1, pc); break;
    }
    __syncthreads();
    const int rest = pg.logL - lr;
    if (rest >= 4) {
      // the passes between the first and the last through LDS, the last on
      // registers straight to F
      if (rest > 4)
        ntt_fwd_tile<false, AS>(lds, rest, T, (uint32_t)pg.logC, tws, pc, threadIdx.x, blockDim.x, false, 4);
      col_last_fwd_store<AS, NV>(lds, words_rsrc(f, N), (uint32_t)base + j0, rowB, (uint32_t)pg.logC, tw, j0,
                                 pg.logL, tw_logn<AS>() - pg.logS, tb.tw2lo + (size_t)prime * TW2_LO,
                                 tb.tw2hi + (size_t)prime * TW2_HI, pc);
      return;
    }
    ntt_fwd_tile<false, AS>(lds, rest, T, (uint32_t)pg.logC, tws, pc, threadIdx.x, blockDim.x, false);
  } else if (first && lin) {
    const MulDesc d = dv.get(m);
    const __amdgpu_buffer_rsrc_t rs = words_rsrc(op ? bin + d.b_off : ain + d.a_off, op ? d.lb : d.la);
    for (uint32_t t0 = 0; t0 < Tl; t0 += COL_BATCH * NTT_COL_THREADS) {
      const uint32_t ob = off0 + (t0 >> pg.logC) * rowB;
      uint32_t v[COL_BATCH];
#pragma unroll
      for (int i = 0; i < COL_BATCH; i++) v[i] = buf_ld(rs, ob + i * RI * rowB);
#pragma unroll
      for (int i = 0; i < COL_BATCH; i++) {
        const uint32_t t = t0 + threadIdx.x + i * NTT_COL_THREADS;
        if (t < Tl) lds[t] = in_limb<AS>(v[i], p);
      }
    }
  } else if (first) {
    const MulDesc d = dv.get(m);
    const uint32_t* src = op ? bin + d.b_off : ain + d.a_off;
    const uint64_t len = op ? d.lb : d.la;
    for (uint32_t t0 = 0; t0 < T; t0 += COL_BATCH * NTT_COL_THREADS) {
      uint32_t v[COL_BATCH];
#pragma unroll
      for (int i = 0; i < COL_BATCH; i++) {
        const uint32_t t = t0 + threadIdx.x + i * NTT_COL_THREADS;
        const uint32_t tc = t < T ? t : T - 1;
        const uint64_t idx = base + ((uint64_t)(tc >> pg.logC) << logSig) + j0 + (tc & (C - 1));
        const uint32_t k = idx < len ? 0xFFFFFFFFu : 0u;
        v[i] = src[idx < len ? idx : 0] & k;
      }
#pragma unroll
      for (int i = 0; i < COL_BATCH; i++) {
        const uint32_t t = t0 + threadIdx.x + i * NTT_COL_THREADS;
        if (t < T) lds[t] = in_limb<AS>(v[i], p);
      }
    }
  } else {
    // pre: this sub-problem is row q' of the previous pass's sub-problem, which
    // left its twiddles omega_{S'}^(j f(q')) to this load; with C <= 256 a
    // thread's positions j advance by a constant step, so the twiddle does too
    uint2 w = make_uint2(0, 0), R = make_uint2(0, 0);
    if (pre) {
      const uint32_t fr = out_freq((uint32_t)(base >> pg.logS) & ((1u << plogL) - 1), plogL);
      const uint32_t ysh = tw_logn<AS>() - plogS, ymask = (1u << tw_logn<AS>()) - 1;
      const uint2* plo = tb.tw2lo + (size_t)prime * TW2_LO;
      const uint32_t* phi = tb.tw2hi + (size_t)prime * TW2_HI;
      const uint32_t jt = ((threadIdx.x >> pg.logC) << logSig) + j0 + (threadIdx.x & (C - 1));
      w = tw2(plo, phi, ((jt * fr) << ysh) & ymask, pc);
      R = tw2(plo, phi, ((((NTT_COL_THREADS >> pg.logC) << logSig) * fr) << ysh) & ymask, pc);
    }
    const __amdgpu_buffer_rsrc_t rs = words_rsrc(f, N);
    for (uint32_t t0 = 0; t0 < T; t0 += COL_BATCH * NTT_COL_THREADS) {
      uint32_t v[COL_BATCH];
      if (lin) {
        const uint32_t ob = off0 + (t0 >> pg.logC) * rowB;
#pragma unroll
        for (int i = 0; i < COL_BATCH; i++) v[i] = buf_ld(rs, ob + i * RI * rowB);
      } else {
#pragma unroll
        for (int i = 0; i < COL_BATCH; i++) {
          const uint32_t t = t0 + threadIdx.x + i * NTT_COL_THREADS;
          const uint32_t tc = t < T ? t : T - 1;
          v[i] = f[base + ((uint64_t)(tc >> pg.logC) << logSig) + j0 + (tc & (C - 1))];
        }
      }
#pragma unroll
      for (int i = 0; i < COL_BATCH; i++) {
        const uint32_t t = t0 + threadIdx.x + i * NTT_COL_THREADS;
        if (pre) {
          v[i] = data_tw<AS>(v[i], w, p);
          w.x = mul_tw(w.x, R.x, R.y, p);
          w.y = w.x * pc.pinv;
        }
        if (t < T) lds[t] = v[i];
      }
    }
  }
  if (!regp) {
    __syncthreads();
    ntt_fwd_tile<false, AS>(lds, pg.logL, T, (uint32_t)pg.logC, tb.tws + (size_t)prime * TWS_ENTRIES, pc,
                            threadIdx.x, blockDim.x, zhi);
  }
  __syncthreads();
  if (!tw) {
    // the pass next to the rows: k_row applies this pass's twiddles
    if (lin) {
      const __amdgpu_buffer_rsrc_t rs = words_rsrc(f, N);
      for (uint32_t k = 0; (k << 8) < T; k++) {
        const uint32_t t = threadIdx.x + (k << 8);
        if (t < T) buf_st(rs, off0 + k * RI * rowB, lds[t]);
      }
    } else {
      for (uint32_t t = threadIdx.x; t < T; t += NTT_COL_THREADS)
        f[base + ((uint64_t)(t >> pg.logC) << logSig) + j0 + (t & (C - 1))] = lds[t];
    }
    return;
  }
  const uint2* lo = tb.tw2lo + (size_t)prime * TW2_LO;
  const uint32_t* hi = tb.tw2hi + (size_t)prime * TW2_HI;
  const uint32_t ysh = tw_logn<AS>() - pg.logS;
  for (uint32_t t0 = 0; t0 < T; t0 += COL_BATCH * NTT_COL_THREADS) {
    uint2 l[COL_BATCH];
    uint32_t h[COL_BATCH];
#pragma unroll
    for (int i = 0; i < COL_BATCH; i++) {
      const uint32_t t = t0 + threadIdx.x + i * NTT_COL_THREADS;
      const uint32_t tc = t < T ? t : T - 1;
      const uint32_t q = tc >> pg.logC, j = j0 + (tc & (C - 1));
      // omega_S^(j f(q)) = omega_{2^27}^y, y = (j f(q) 2^(27 - logS)) mod 2^27:
      // the bits of j f(q) above 2^32 do not reach y
      const uint32_t y = ((j * out_freq(q, pg.logL)) << ysh) & ((1u << tw_logn<AS>()) - 1);
      l[i] = lo[y & (TW2_LO - 1)];
      h[i] = hi[y >> TW2_LO_BITS];
    }
#pragma unroll
    for (int i = 0; i < COL_BATCH; i++) {
      const uint32_t t = t0 + threadIdx.x + i * NTT_COL_THREADS;
      if (t < T) {
        const uint32_t q = t >> pg.logC, j = j0 + (t & (C - 1));
        const uint32_t w = mul_tw(h[i], l[i].x, l[i].y, p);
        f[base + ((uint64_t)q << logSig) + j] = data_tw<AS>(lds[t], make_uint2(w, w * pc.pinv), p);
      }
    }
  }
}

// The last (outermost) inverse column pass on registers, stored as exact
// residues: in a tile of NV * 256 words and at most 256 columns, group
// threadIdx.x + 256 u of that pass (radix 2^LR) holds the elements
// threadIdx.x + 256 (u + j1 NV / 2^LR), all of them stored by this thread, so
// its outputs go to memory without a round trip through LDS.  Same arithmetic
// as groups_inv.
template <int LR, int AS, int NV>
__device__ __forceinline__ void col_last_inv(const uint32_t* lds, uint32_t logL, uint32_t logC,
                                             const uint2* __restrict__ itw, const PrimeC& pc,
                                             __amdgpu_buffer_rsrc_t rs, uint32_t off0, uint32_t stepB) {
  constexpr int R = 1 << LR;
  constexpr int U = NV >> LR;
  const uint32_t logSR = logL - LR;
  const uint32_t stride = 1u << (logSR + logC);
#pragma unroll
  for (int u = 0; u < U; u++) {
    uint32_t jj;
    const uint32_t b = group_base<LR, false>(threadIdx.x + 256u * u, logSR, logC, &jj);
    uint32_t x[R];
#pragma unroll
    for (int k1 = 0; k1 < R; k1++) x[brev_c(k1, LR)] = lds[b + k1 * stride];
    if (logSR > 0) {
      const uint32_t jo = jj * (uint32_t)sizeof(uint2);
      const __amdgpu_buffer_rsrc_t rt = tw_rsrc(itw, (uint32_t)R << logSR);
#pragma unroll
      for (int k1 = 1; k1 < R; k1++) {
        const uint2 t = tw_at(rt, (uint32_t)k1, logSR, jo);
        const int r = brev_c(k1, LR);
        x[r] = tw_mul<AS>(x[r], t.x, t.y, pc.p);
      }
      dft_inv<LR, AS, true>(x, pc);
    } else {
      dft_inv<LR, AS, false>(x, pc);
    }
#pragma unroll
    for (int j1 = 0; j1 < R; j1++) buf_st(rs, off0 + (uint32_t)(u + j1 * U) * stepB, out_residue<AS>(x[j1], pc.p));
  }
}

template <int LOGT, int AS>
__global__ void __launch_bounds__(NTT_COL_THREADS)
k_pass_inv(DescView dv, PassGeom pg, int last, int tw, int post, int plogS, int plogL, uint32_t* __restrict__ F,
           uint32_t* __restrict__ res, uint64_t res_stride, NttTables tb) {
  __shared__ uint32_t lds[1u << LOGT];
  __shared__ uint32_t fq[1u << NTT_COL_MAXL];    // frequency at each output row
  const uint32_t T = 1u << (pg.logL + pg.logC);
  const uint32_t prime = blockIdx.y;
  const PrimeC& pc = primec<AS>(prime);
  const uint32_t p = pc.p;
  uint64_t m, base;
  uint32_t j0;
  pg.locate(xcd_remap(blockIdx.x, gridDim.x), &m, &base, &j0);
  const int logSig = pg.logS - pg.logL;
  const uint32_t C = 1u << pg.logC;
  const uint64_t N = 1ull << pg.logN;
  uint32_t* f = F + ((m * 3 + prime) * 2 + 0) * N;
  const uint2* lo = tb.itw2lo + (size_t)prime * TW2_LO;
  const uint32_t* hi = tb.itw2hi + (size_t)prime * TW2_HI;
  const uint32_t ysh = tw_logn<AS>() - pg.logS;
  // element addressing of tiles of at most 256 columns, as in k_pass_fwd
  const bool lin = pg.logC <= 8;
  const uint32_t RI = NTT_COL_THREADS >> (lin ? pg.logC : 0);
  const uint32_t rowB = 4u << logSig;
  const uint32_t off0 = ((uint32_t)base + ((threadIdx.x >> pg.logC) << logSig) + j0 + (threadIdx.x & (C - 1))) * 4u;
  // the first inverse pass (sub-problems of 16 rows) on the loaded words
  constexpr int NVT = (1 << LOGT) / NTT_COL_THREADS;
  const bool regf = !tw && lin && T == (1u << LOGT) && pg.logL > 4;
  if (regf) {
    col_first_inv_load<AS, NVT>(lds, words_rsrc(f, N), (uint32_t)base + j0, rowB, (uint32_t)pg.logC, pc);
  } else if (!tw) {
    // the pass next to the rows: k_row applied this pass's twiddles
    const __amdgpu_buffer_rsrc_t rs = words_rsrc(f, N);
    for (uint32_t t0 = 0; t0 < T; t0 += COL_BATCH * NTT_COL_THREADS) {
      uint32_t v[COL_BATCH];
      if (lin) {
        const uint32_t ob = off0 + (t0 >> pg.logC) * rowB;
#pragma unroll
        for (int i = 0; i < COL_BATCH; i++) v[i] = buf_ld(rs, ob + i * RI * rowB);
      } else {
#pragma unroll
        for (int i = 0; i < COL_BATCH; i++) {
          const uint32_t t = t0 + threadIdx.x + i * NTT_COL_THREADS;
          const uint32_t tc = t < T ? t : T - 1;
          v[i] = f[base + ((uint64_t)(tc >> pg.logC) << logSig) + j0 + (tc & (C - 1))];
        }
      }
#pragma unroll
      for (int i = 0; i < COL_BATCH; i++) {
        const uint32_t t = t0 + threadIdx.x + i * NTT_COL_THREADS;
        if (t < T) lds[t] = v[i];
      }
    }
  } else {
  for (uint32_t q = threadIdx.x; q < (1u << pg.logL); q += blockDim.x) fq[q] = out_freq(q, pg.logL);
  __syncthreads();
  for (uint32_t t0 = 0; t0 < T; t0 += COL_BATCH * NTT_COL_THREADS) {
    uint2 l[COL_BATCH];
    uint32_t h[COL_BATCH], v[COL_BATCH];
#pragma unroll
    for (int i = 0; i < COL_BATCH; i++) {
      const uint32_t t = t0 + threadIdx.x + i * NTT_COL_THREADS;
      const uint32_t tc = t < T ? t : T - 1;
      const uint32_t q = tc >> pg.logC, j = j0 + (tc & (C - 1));
      const uint32_t y = ((j * fq[q]) << ysh) & ((1u << tw_logn<AS>()) - 1);
      l[i] = lo[y & (TW2_LO - 1)];
      h[i] = hi[y >> TW2_LO_BITS];
      v[i] = f[base + ((uint64_t)q << logSig) + j];
    }
#pragma unroll
    for (int i = 0; i < COL_BATCH; i++) {
      const uint32_t t = t0 + threadIdx.x + i * NTT_COL_THREADS;
      if (t < T) {
        const uint32_t w = mul_tw(h[i], l[i].x, l[i].y, p);
        lds[t] = data_tw<AS>(v[i], make_uint2(w, w * pc.pinv), p);
      }
    }
  }
  }
  __syncthreads();
  const uint2* itws = tb.itws + (size_t)prime * TWS_ENTRIES;
  if (last && lin && T == (1u << LOGT)) {
    // the outermost pass: every pass but the last (and but the first when it
    // ran on registers) through LDS, the last on registers straight to the
    // residues (positions at or past L fall outside the buffer's range: not
    // written)
    const int lr0 = pass_logr(pg.logL);
    if (!regf || pg.logL - lr0 > 4)
      ntt_inv_tile<false, AS>(lds, pg.logL - lr0, T, (uint32_t)pg.logC, itws, pc, threadIdx.x, blockDim.x,
                              regf ? 8 : 4);
    const MulDesc d = dv.get(m);
    const uint64_t L = (uint64_t)d.la + d.lb;
    uint32_t* out = res + (size_t)prime * res_stride + d.r_off;
    const __amdgpu_buffer_rsrc_t rs = words_rsrc(out, L);
    constexpr int NV = (1 << LOGT) / NTT_COL_THREADS;
    const uint2* itw = itws + tws_off(pg.logL);
    const uint32_t stepB = RI * rowB;
    switch (lr0) {
      case 1: col_last_inv<1, AS, NV>(lds, pg.logL, pg.logC, itw, pc, rs, off0, stepB); break;
      case 2: col_last_inv<2, AS, NV>(lds, pg.logL, pg.logC, itw, pc, rs, off0, stepB); break;
      case 3: col_last_inv<3, AS, NV>(lds, pg.logL, pg.logC, itw, pc, rs, off0, stepB); break;
      default: col_last_inv<4, AS, NV>(lds, pg.logL, pg.logC, itw, pc, rs, off0, stepB); break;
    }
    if (base == 0 && j0 == 0)
      for (uint64_t j = N + threadIdx.x; j < L; j += blockDim.x) out[j] = 0u;
    return;
  }
  ntt_inv_tile<false, AS>(lds, pg.logL, T, (uint32_t)pg.logC, itws, pc, threadIdx.x, blockDim.x, regf ? 8 : 4);
  if (!last) {
    if (!post) {
      if (lin) {
        const __amdgpu_buffer_rsrc_t rs = words_rsrc(f, N);
        for (uint32_t k = 0; (k << 8) < T; k++) {
          const uint32_t t = threadIdx.x + (k << 8);
          if (t < T) buf_st(rs, off0 + k * RI * rowB, lds[t]);
        }
      } else {
        for (uint32_t t = threadIdx.x; t < T; t += blockDim.x)
          f[base + ((uint64_t)(t >> pg.logC) << logSig) + j0 + (t & (C - 1))] = lds[t];
      }
      return;
    }
    // post: the inverse twiddles of the previous (outer) pass, at the same
    // positions the forward load of this pass took them, by the same steps
    const uint32_t fr = out_freq((uint32_t)(base >> pg.logS) & ((1u << plogL) - 1), plogL);
    const uint32_t ysh2 = tw_logn<AS>() - plogS, ymask = (1u << tw_logn<AS>()) - 1;
    const uint2* plo = tb.itw2lo + (size_t)prime * TW2_LO;
    const uint32_t* phi = tb.itw2hi + (size_t)prime * TW2_HI;
    const uint32_t jt = ((threadIdx.x >> pg.logC) << logSig) + j0 + (threadIdx.x & (C - 1));
    uint2 w = tw2(plo, phi, ((jt * fr) << ysh2) & ymask, pc);
    const uint2 R = tw2(plo, phi, ((((NTT_COL_THREADS >> pg.logC) << logSig) * fr) << ysh2) & ymask, pc);
    for (uint32_t t = threadIdx.x; t < T; t += NTT_COL_THREADS) {
      f[base + ((uint64_t)(t >> pg.logC) << logSig) + j0 + (t & (C - 1))] = data_tw<AS>(lds[t], w, p);
      w.x = mul_tw(w.x, R.x, R.y, p);
      w.y = w.x * pc.pinv;
    }
    return;
  }
  // the outermost pass: positions are coefficient indices; write exact residues
  const MulDesc d = dv.get(m);
  uint32_t* out = res + (size_t)prime * res_stride + d.r_off;
  const uint64_t L = (uint64_t)d.la + d.lb;
  if (lin) {
    // positions at or past L fall outside the buffer's range: not written
    const __amdgpu_buffer_rsrc_t rs = words_rsrc(out, L);
    for (uint32_t k = 0; (k << 8) < T; k++) {
      const uint32_t t = threadIdx.x + (k << 8);
      if (t < T) buf_st(rs, off0 + k * RI * rowB, out_residue<AS>(lds[t], p));
    }
  } else {
    for (uint32_t t = threadIdx.x; t < T; t += blockDim.x) {
      const uint64_t j = base + ((uint64_t)(t >> pg.logC) << logSig) + j0 + (t & (C - 1));
      if (j < L) out[j] = out_residue<AS>(lds[t], p);
    }
  }
  // coefficient positions in [N, L) (only when L = N + 1) are zero
  if (base == 0 && j0 == 0)
    for (uint64_t j = N + threadIdx.x; j < L; j += blockDim.x) out[j] = 0u;
}

// The outermost pass of a full row tile of 2^LOGT points on registers (radix
// 2^LR = 2^pass_logr(LOGT), groups of elements j + 2^(LOGT-LR) k): thread t
// of the 2^LOGT / 16 loads and stores the elements t + (2^LOGT / 16) i, which
// are exactly its D = 2^(4-LR) groups j = t + (2^LOGT / 16) d of that pass
// (element i = d + D k of group d), so the first forward pass can start from
// the loaded values and the last inverse pass can end in the stored ones.
// Same arithmetic as groups_fwd / groups_inv.
template <int LR, int AS>
__device__ __forceinline__ void row_pass_fwd(uint32_t* v, uint32_t j, uint32_t logSR, const uint2* __restrict__ tw,
                                             const PrimeC& pc) {
  constexpr int R = 1 << LR;
  dft_fwd<LR, AS, true, false>(v, pc);
  const uint32_t jo = j * (uint32_t)sizeof(uint2);
  const __amdgpu_buffer_rsrc_t rs = tw_rsrc(tw, (uint32_t)R << logSR);
#pragma unroll
  for (int k1 = 1; k1 < R; k1++) {
    const uint2 t = tw_at(rs, (uint32_t)k1, logSR, jo);
    const int r = brev_c(k1, LR);
    v[r] = tw_mul<AS>(v[r], t.x, t.y, pc.p);
  }
}
template <int LR, int AS>
__device__ __forceinline__ void row_pass_inv(uint32_t* v, uint32_t j, uint32_t logSR, const uint2* __restrict__ itw,
                                             const PrimeC& pc) {
  constexpr int R = 1 << LR;
  const uint32_t jo = j * (uint32_t)sizeof(uint2);
  const __amdgpu_buffer_rsrc_t rs = tw_rsrc(itw, (uint32_t)R << logSR);
#pragma unroll
  for (int k1 = 1; k1 < R; k1++) {
    const uint2 t = tw_at(rs, (uint32_t)k1, logSR, jo);
    const int r = brev_c(k1, LR);
    v[r] = tw_mul<AS>(v[r], t.x, t.y, pc.p);
  }
  dft_inv<LR, AS, true>(v, pc);
}
// The first forward pass of both operands of a full row (A at [0, 2^LOGT),
// B at [2^LOGT, 2^(LOGT+1)) of the padded tile) from the loaded values.
template <int LOGT, int AS>
__device__ __forceinline__ void row_first_fwd(uint32_t* lds, const uint32_t* va, const uint32_t* vb,
                                              const uint2* __restrict__ tws, const PrimeC& pc) {
  constexpr int LR = pass_logr(LOGT), R = 1 << LR, D = 1 << (4 - LR);
  constexpr uint32_t NT = (1u << LOGT) / 16, SR = 1u << (LOGT - LR), STRIDE = SR + SR / 16;
  const uint2* tw = tws + tws_off(LOGT);
#pragma unroll
  for (int d = 0; d < D; d++) {
    uint32_t xa[R], xb[R];
#pragma unroll
    for (int k = 0; k < R; k++) {
      xa[k] = va[d + D * k];
      xb[k] = vb[d + D * k];
    }
    const uint32_t j = threadIdx.x + NT * d;
    row_pass_fwd<LR, AS>(xa, j, LOGT - LR, tw, pc);
    row_pass_fwd<LR, AS>(xb, j, LOGT - LR, tw, pc);
#pragma unroll
    for (int k1 = 0; k1 < R; k1++) {
      lds[lds_pad(j) + k1 * STRIDE] = xa[brev_c(k1, LR)];
      lds[lds_pad((1u << LOGT) + j) + k1 * STRIDE] = xb[brev_c(k1, LR)];
    }
  }
}
// The last inverse pass of operand A of a full row into vo[i], the value of
// element t + (2^LOGT / 16) i.
template <int LOGT, int AS>
__device__ __forceinline__ void row_last_inv(const uint32_t* lds, uint32_t* vo, const uint2* __restrict__ itws,
                                             const PrimeC& pc) {
  constexpr int LR = pass_logr(LOGT), R = 1 << LR, D = 1 << (4 - LR);
  constexpr uint32_t NT = (1u << LOGT) / 16, SR = 1u << (LOGT - LR), STRIDE = SR + SR / 16;
  const uint2* itw = itws + tws_off(LOGT);
#pragma unroll
  for (int d = 0; d < D; d++) {
    const uint32_t j = threadIdx.x + NT * d;
    uint32_t x[R];
#pragma unroll
    for (int k1 = 0; k1 < R; k1++) x[brev_c(k1, LR)] = lds[lds_pad(j) + k1 * STRIDE];
    row_pass_inv<LR, AS>(x, j, LOGT - LR, itw, pc);
#pragma unroll
    for (int k = 0; k < R; k++) vo[d + D * k] = x[k];
  }
}

// Rows of M = 2^logM <= 2^LOGT elements; 2^LOGT/16 threads.
template <int LOGT, int AS>
__global__ void __launch_bounds__((1 << LOGT) / 16)
// bmode 0: both operands per product.  A stage whose second operand is the
// same for every product computes that operand's row transforms once:
// bmode 1 (rows of product 0 only) transforms them and stores the tile as it
// stands in LDS; bmode 2 then loads it into the second half for every
// product and transforms only the first operand.
k_row(int logN, int logM, int logSl, int logLl, int bmode, uint32_t* __restrict__ F, NttTables tb, uint2 scale0,
      uint2 scale1, uint2 scale2) {
  constexpr uint32_t TT = 1u << LOGT;
  __shared__ uint32_t lds[lds_pad(2 * TT)];
  const uint32_t prime = blockIdx.y;
  const PrimeC& pc = primec<AS>(prime);
  const uint32_t p = pc.p;
  const int logR1 = logN - logM;
  const uint32_t M = 1u << logM;
  const uint64_t N = 1ull << logN;
  const uint64_t m = blockIdx.x >> logR1;
  const uint32_t q = blockIdx.x & ((1u << logR1) - 1);
  uint32_t* fa = F + ((m * 3 + prime) * 2 + 0) * N + ((uint64_t)q << logM);
  uint32_t* fb = F + (((bmode ? 0 : m) * 3 + prime) * 2 + 1) * N + ((uint64_t)q << logM);
  constexpr uint32_t NT = TT / 16;                 // blockDim.x
  // The twiddles of the column pass next to the rows (sub-problems of
  // S = 2^logSl, rows of L = 2^logLl): position j of row q takes
  // omega_S^(j f) with f the frequency of q within its sub-problem, and the
  // inverse on the way back.  A thread's positions j = tid + i NT form a
  // geometric sequence: w_i = w_0 R^i, R = omega_S^(NT f).
  const uint32_t fr = out_freq(q & ((1u << logLl) - 1), logLl);
  const uint32_t ysh = tw_logn<AS>() - logSl, ymask = (1u << tw_logn<AS>()) - 1;
  const uint2* flo = tb.tw2lo + (size_t)prime * TW2_LO;
  const uint32_t* fhi = tb.tw2hi + (size_t)prime * TW2_HI;
  uint2 w = tw2(flo, fhi, ((threadIdx.x * fr) << ysh) & ymask, pc);
  const uint2 R = tw2(flo, fhi, ((NT * fr) << ysh) & ymask, pc);
  const uint2* tws = tb.tws + (size_t)prime * TWS_ENTRIES;
  if (bmode == 1) {
    for (uint32_t t = threadIdx.x; t < M; t += NT) {
      lds[lds_pad(t)] = data_tw<AS>(fb[t], w, p);
      w.x = mul_tw(w.x, R.x, R.y, p);
      w.y = w.x * pc.pinv;
    }
    __syncthreads();
    ntt_fwd_tile<true, AS>(lds, logM, M, 0, tws, pc);
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < M; t += NT) fb[t] = lds[lds_pad(t)];
    return;
  }
  if (bmode == 2) {
    for (uint32_t t = threadIdx.x; t < M; t += NT) {
      lds[lds_pad(t)] = data_tw<AS>(fa[t], w, p);
      lds[lds_pad(M + t)] = fb[t];
      w.x = mul_tw(w.x, R.x, R.y, p);
      w.y = w.x * pc.pinv;
    }
  } else if (M == TT) {
    // full rows: all 32 loads of the thread in flight before the first use
    uint32_t va[16], vb[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
      va[i] = fa[threadIdx.x + i * NT];
      vb[i] = fb[threadIdx.x + i * NT];
    }
#pragma unroll
    for (int i = 0; i < 16; i++) {
      va[i] = data_tw<AS>(va[i], w, p);
      vb[i] = data_tw<AS>(vb[i], w, p);
      w.x = mul_tw(w.x, R.x, R.y, p);
      w.y = w.x * pc.pinv;
    }
    row_first_fwd<LOGT, AS>(lds, va, vb, tws, pc);
  } else {
    for (uint32_t t = threadIdx.x; t < M; t += NT) {
      lds[lds_pad(t)] = data_tw<AS>(fa[t], w, p);
      lds[lds_pad(M + t)] = data_tw<AS>(fb[t], w, p);
      w.x = mul_tw(w.x, R.x, R.y, p);
      w.y = w.x * pc.pinv;
    }
  }
  __syncthreads();
  const uint2 sc = prime == 0 ? scale0 : (prime == 1 ? scale1 : scale2);
  // full rows: the first forward pass ran on registers at the load; the last
  // forward pass, the pointwise product and the first inverse pass run on
  // registers too (mid), except in rows of 2^13, where the extra registers
  // would cost that tile its second workgroup per CU
  const bool full = M == TT && bmode == 0;
  const bool mid = full && LOGT != 13;
  if (mid) {
    ntt_fwd_tile<true, AS>(lds, LOGT - pass_logr(LOGT), 2 * M, 0, tws, pc, threadIdx.x, blockDim.x, false, 4);
    mid_passes<AS, false>(lds, lds_pad(16 * threadIdx.x), lds_pad(TT + 16 * threadIdx.x), sc, pc);
    pass_sync(4, 0);
  } else if (full) {
    ntt_fwd_tile<true, AS>(lds, LOGT - pass_logr(LOGT), 2 * M, 0, tws, pc);   // the passes after the first
  } else {
    ntt_fwd_tile<true, AS>(lds, logM, bmode == 2 ? M : 2 * M, 0, tws, pc);
  }
  if (mid) {
  } else if (M == TT) {
    // thread g wrote A and B at [16 g, 16 g + 16): pointwise in place, and the
    // first inverse pass reads the same positions in the same thread
#pragma unroll
    for (int k = 0; k < 16; k++) {
      const uint32_t t = 16 * threadIdx.x + k;
      const uint32_t x = lds[lds_pad(t)], y = lds[lds_pad(M + t)];
      lds[lds_pad(t)] = pointwise_raw<AS>(x, y, pc);
    }
  } else {
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < M; t += blockDim.x) {
      uint32_t x = lds[lds_pad(t)], y = lds[lds_pad(M + t)];
      lds[lds_pad(t)] = pointwise_raw<AS>(x, y, pc);
    }
    __syncthreads();
  }
  const uint2* itws = tb.itws + (size_t)prime * TWS_ENTRIES;
  // full rows: the last inverse pass (the thread's groups) on registers,
  // vo[i] the value for position threadIdx.x + i NT
  const bool rp = M == TT;
  uint32_t vo[16];
  if (rp) {
    // every pass but the last (and but the first when it ran on registers)
    ntt_inv_tile<true, AS>(lds, LOGT - pass_logr(LOGT), M, 0, itws, pc, threadIdx.x, blockDim.x, mid ? 8 : 4);
    row_last_inv<LOGT, AS>(lds, vo, itws, pc);
  } else {
    ntt_inv_tile<true, AS>(lds, logM, M, 0, itws, pc);
  }
  const uint2* ilo = tb.itw2lo + (size_t)prime * TW2_LO;
  const uint32_t* ihi = tb.itw2hi + (size_t)prime * TW2_HI;
  // the pointwise scale (2^32 / N) rides on the inverse twiddles: every step
  // after the pointwise product is linear mod p
  uint2 wi = tw2(ilo, ihi, ((threadIdx.x * fr) << ysh) & ymask, pc);
  wi.x = mul_tw(wi.x, sc.x, sc.y, p);
  wi.y = wi.x * pc.pinv;
  const uint2 Ri = tw2(ilo, ihi, ((NT * fr) << ysh) & ymask, pc);
  if (rp) {
#pragma unroll
    for (int i = 0; i < 16; i++) {
      fa[threadIdx.x + i * NT] = data_tw<AS>(vo[i], wi, p);
      wi.x = mul_tw(wi.x, Ri.x, Ri.y, p);
      wi.y = wi.x * pc.pinv;
    }
    return;
  }
  for (uint32_t t = threadIdx.x; t < M; t += NT) {
    fa[t] = data_tw<AS>(lds[lds_pad(t)], wi, p);
    wi.x = mul_tw(wi.x, Ri.x, Ri.y, p);
    wi.y = wi.x * pc.pinv;
  }
}

// ---------------------------------------------------------------------------
// Garner CRT of the three residues into V = x0 + p0*x1 + p0*p1*x2 < 2^96.
// x2 = (r2 - x0) (p0 p1)^-1 - x1 p1^-1 mod p2 (both products independent of
// each other), and V in Horner form x0 + p0 (x1 + p1 x2): three 32x32+32-bit
// multiply-adds, none of which can overflow 64 bits.
template <int AS = 0>
__device__ __forceinline__ void garner3(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t& v0, uint32_t& v1,
                                        uint32_t& v2) {
  const CrtC& c_crt = crtc<AS>();
  const uint32_t P1 = primec<AS>(1).p, P2 = primec<AS>(2).p;
  const uint32_t x0 = r0;
  const uint32_t x1 = mul_tw(sub_mod(r1, x0, P1), c_crt.c01, c_crt.c01q, P1);
  const uint32_t e = mul_tw(sub_mod(r2, x0, P2), c_crt.c012, c_crt.c012q, P2);
  const uint32_t x2 = sub_mod(e, mul_tw(x1, c_crt.c12, c_crt.c12q, P2), P2);
  const uint64_t t = (uint64_t)c_crt.p1 * x2 + x1;                        // < p1 p2
  const uint64_t m1 = (uint64_t)c_crt.p0 * (uint32_t)t + x0;
  const uint64_t m2 = (uint64_t)c_crt.p0 * (uint32_t)(t >> 32) + (uint32_t)(m1 >> 32);
  v0 = (uint32_t)m1;
  v1 = (uint32_t)m2;
  v2 = (uint32_t)(m2 >> 32);
}

// Carry resolution.  Given 96-bit column values V(k) = v0 + v1 2^32 + v2 2^64,
// limb_k = (v0(k) + v1(k-1) + v2(k-2) + carries) mod 2^32.  With
// s_k = v0(k)+v1(k-1)+v2(k-2) < 3*2^32, x_k = s_k mod 2^32, y_k = s_k >> 32,
// u_k = x_k + y_{k-1} <= 2^32 + 1 and the remaining carries are binary:
// generate g_k = (u_k >= 2^32), propagate p_k = (u_k == 2^32 - 1).

// Wave-level: carry into each lane for (g, p) with wave carry-in `cin`;
// returns lane's carry in, and the wave carry out in *cout.
__device__ __forceinline__ uint32_t wave_carry(bool g, bool pr, uint32_t cin, uint32_t* cout, bool* allprop) {
  const uint64_t gm = __ballot(g), pm = __ballot(pr);
  const uint64_t a = gm, b = gm | pm;
  const uint64_t s1 = a + b;
  const uint64_t c1 = s1 < a;
  const uint64_t s2 = s1 + cin;
  const uint64_t c2 = s2 < s1;
  *cout = (uint32_t)(c1 | c2);
  *allprop = (pm == ~0ull);
  const uint64_t cm = s2 ^ pm;   // carry into each bit position
  return (uint32_t)((cm >> (threadIdx.x & 63)) & 1ull);
}

// Segments of a CRT launch: device tables (many segments) or up to
// CAT_INLINE_SEG segments carried in the kernel arguments.
#define CAT_INLINE_SEG 32
struct SegView {
  const CrtSeg* segs;        // nullptr => inline tables
  const uint32_t* pref;      // pref[s] = first block of segment s (nseg+1 entries)
  const uint32_t* b2s;       // with segs: the segment of every block (one load, no search)
  uint32_t nseg;
  uint32_t ubl;              // > 0: uniform segments of ubl blocks each (below)
  CrtSeg iseg[CAT_INLINE_SEG];
  uint32_t ipref[CAT_INLINE_SEG + 1];
  // uniform: segment s is iseg[0] with out_pos, res_pos and add_pos advanced
  // by s * ustep[0], s * iseg[0].len and s * ustep[1]
  uint64_t ustep[2];
  __device__ __forceinline__ void find(uint32_t b, CrtSeg* sg, uint32_t* first, uint32_t* end,
                                       uint32_t* segi = nullptr) const {
    if (ubl) {
      const uint32_t q = b / ubl;
      *sg = iseg[0];
      sg->out_pos += q * ustep[0];
      sg->res_pos += q * iseg[0].len;
      sg->add_pos += q * ustep[1];
      *first = q * ubl;
      *end = *first + ubl;
      if (segi) *segi = q;
      return;
    }
    const uint32_t* pr = segs ? pref : ipref;
    uint32_t lo = 0, hi = nseg;   // pr[lo] <= b < pr[lo+1]
    if (segs && b2s) {
      lo = b2s[b];
    } else {
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pr[mid] <= b) lo = mid; else hi = mid;
      }
    }
    *sg = segs ? segs[lo] : iseg[lo];
    *first = pr[lo];
    *end = pr[lo + 1];
    if (segi) *segi = lo;
  }
};

// CRT + carry.  Workgroup b < nblk covers CAT_CRT_BLOCK limbs of one segment;
// workgroups from nblk on copy tail ranges.  The carry into a block follows
// from the generate / all-propagate pair (G, P) of the blocks before it in the
// segment (with carry-in 0).  Each block publishes its pair as
// flags[b] = epoch << 3 | P << 2 | G << 1 | 1 (epoch: this launch's number in
// the call; the flags are cleared when the call starts) and reads its
// predecessor's; a pair that has not appeared after a few polls is recomputed
// from that block's residues instead, so no block ever waits on another
// (nothing is assumed about which workgroups run at the same time).  Most
// blocks need none of this: the u of the few positions below the block, which
// they compute anyway for their left context, decide the carry in unless all
// of them propagate.
#define CAT_SCAN_POLLS 16   // default number of polls of a predecessor's flag

// A thread's CAT_CRT_E consecutive words: one vector access in a block that
// lies inside its segment
struct CrtWords {
  uint32_t w[CAT_CRT_E];
};

// V of one position: Garner's recombination of its three residues, or (RAW)
// the three words themselves when they already hold V = v0 + v1 2^32 + v2 2^64
// (exact column sums of a schoolbook product).  Zero residues give V = 0.
template <bool RAW, int AS>
__device__ __forceinline__ void crt_value(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t& a0, uint32_t& a1,
                                          uint32_t& a2) {
  if constexpr (RAW) {
    a0 = x0;
    a1 = x1;
    a2 = x2;
  } else {
    garner3<AS>(x0, x1, x2, a0, a1, a2);
  }
}

// s = a + b + c as s mod 2^32 and the carry h = s >> 32 (h <= 2)
__device__ __forceinline__ uint32_t col_sum(uint32_t a, uint32_t b, uint32_t c, uint32_t* h) {
  unsigned c1, c2;
  const uint32_t t = __builtin_addc(a, b, 0u, &c1);
  const uint32_t s = __builtin_addc(t, c, 0u, &c2);
  *h = c1 + c2;
  return s;
}

// The thread's CAT_CRT_E positions k0 .. k0+E-1 of the block starting at kb:
// u_k mod 2^32 in ul, the generate bits in gk, the thread's (G, P); wave pairs
// go to tmp[wave].  Column k needs V0(k), V1(k-1), V2(k-2) and the carry
// y_{k-1} of column k-1; from its left neighbour a thread takes V1(k0-1),
// V2(k0-1), V2(k0-2) and y_{k0-1} (which the neighbour has for its own last
// column), through xv[tid] = {V1, V2, V2', y}.  For thread 0 the first
// CRT_CTX lanes of the first wave recompute positions kb-CRT_CTX .. kb-1 from
// their residues.  Their u (positions kb-CRT_CTX+3 .. kb-1) also decide the
// carry into the block unless every one of them propagates: the carry out of
// position kb-1 is the generate bit of the highest position below kb that
// does not propagate.  *spec gets that carry (0 or 1), or 2 when undecided.
#define CRT_CTX 16
template <bool RAW, int AS>
__device__ __forceinline__ void crt_local(const CrtSeg& sg, const uint32_t* __restrict__ r0,
                                          const uint32_t* __restrict__ r1, const uint32_t* __restrict__ r2,
                                          uint64_t kb, uint4* xv, uint32_t* tmp, uint32_t* ul, bool* gk, bool* Gt,
                                          bool* Pt, uint32_t* spec) {
  static_assert(CAT_CRT_E >= 3, "a thread's last column must lie inside the thread");
  const uint32_t tid = threadIdx.x;
  const uint64_t k0 = kb + (uint64_t)tid * CAT_CRT_E;
  const bool lctx = tid < CRT_CTX && kb + tid >= CRT_CTX;
  uint32_t x0[CAT_CRT_E], x1[CAT_CRT_E], x2[CAT_CRT_E];
  uint32_t y0 = 0, y1 = 0, y2 = 0;
  // the thread's 3*E residue loads, and its left-context position, in flight
  // together; positions past the segment read as zero residues (V = 0).
  // The residues are read once, so those loads are non-temporal.
  if (kb + CAT_CRT_BLOCK <= sg.len) {
#pragma unroll
    for (int i = 0; i < CAT_CRT_E; i++) {
      x0[i] = __builtin_nontemporal_load(r0 + k0 + i);
      x1[i] = __builtin_nontemporal_load(r1 + k0 + i);
      x2[i] = __builtin_nontemporal_load(r2 + k0 + i);
    }
  } else {
#pragma unroll
    for (int i = 0; i < CAT_CRT_E; i++) {
      const uint64_t k = k0 + i;
      const bool in = k < sg.len;
      const uint64_t kc = in ? k : 0;
      const uint32_t msk = in ? 0xFFFFFFFFu : 0u;
      x0[i] = r0[kc] & msk;
      x1[i] = r1[kc] & msk;
      x2[i] = r2[kc] & msk;
    }
  }
  if (tid < CRT_CTX) {
    const uint64_t kl = lctx ? kb + tid - CRT_CTX : 0;
    const uint32_t msk = lctx ? 0xFFFFFFFFu : 0u;
    y0 = r0[kl] & msk;
    y1 = r1[kl] & msk;
    y2 = r2[kl] & msk;
  }
  uint32_t a0[CAT_CRT_E], a1[CAT_CRT_E], a2[CAT_CRT_E];
#pragma unroll
  for (int i = 0; i < CAT_CRT_E; i++) crt_value<RAW, AS>(x0[i], x1[i], x2[i], a0[i], a1[i], a2[i]);
  uint32_t lo[CAT_CRT_E], h[CAT_CRT_E];
#pragma unroll
  for (int i = 2; i < CAT_CRT_E; i++) lo[i] = col_sum(a0[i], a1[i - 1], a2[i - 2], &h[i]);
  // the block's context: lane l of the first wave holds V(kb-CRT_CTX+l) for
  // l < CRT_CTX (zero outside the segment)
  uint4 bctx = make_uint4(0, 0, 0, 0);
  uint32_t sp = 2;
  if (tid < 64) {
    uint32_t c0, c1, c2;
    crt_value<RAW, AS>(y0, y1, y2, c0, c1, c2);
    const uint32_t b1 = __shfl_up(c1, 1, 64), b2 = __shfl_up(c2, 1, 64), d2 = __shfl_up(c2, 2, 64);
    uint32_t hh;
    const uint32_t cl = col_sum(c0, b1, d2, &hh);   // column kb-CRT_CTX+l (lanes >= 2)
    const uint32_t hq = __shfl_up(hh, 1, 64);
    unsigned g;
    const uint32_t cu = __builtin_addc(cl, hq, 0u, &g);   // u of that position (lanes >= 3)
    const bool valid = tid >= 3 && tid < CRT_CTX;
    const uint64_t gm = __ballot(valid && g != 0);
    const uint64_t dm = gm | __ballot(valid && g == 0 && cu != 0xFFFFFFFFu);
    if (dm) sp = (uint32_t)((gm >> (63 - __builtin_clzll(dm))) & 1ull);
    bctx = make_uint4(c1, c2, b2, hh);
  }
  __syncthreads();   // xv may still be read by a previous call
  xv[tid + 1] = make_uint4(a1[CAT_CRT_E - 1], a2[CAT_CRT_E - 1], a2[CAT_CRT_E - 2], h[CAT_CRT_E - 1]);
  if (tid == CRT_CTX - 1) xv[0] = bctx;
  if (tid == 0) *spec = sp;
  __syncthreads();
  const uint4 z = xv[tid];
  lo[0] = col_sum(a0[0], z.x, z.z, &h[0]);
  lo[1] = col_sum(a0[1], a1[0], z.y, &h[1]);
  bool G = false, P = true;
  uint32_t hp = z.w;
#pragma unroll
  for (int i = 0; i < CAT_CRT_E; i++) {
    unsigned g;
    ul[i] = __builtin_addc(lo[i], hp, 0u, &g);
    hp = h[i];
    gk[i] = g != 0;
    const bool pr = ul[i] == 0xFFFFFFFFu;
    G = gk[i] || (pr && G);
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

// block pair from the wave pairs: bit 0 = G, bit 1 = P
__device__ __forceinline__ uint32_t crt_block_pair(const uint32_t* tmp) {
  uint32_t bG = 0, bP = 1;
  for (uint32_t w = 0; w < (blockDim.x >> 6); w++) {
    const uint32_t x = tmp[w];
    bG = (x & 1u) | ((x >> 1) & bG);
    bP = bP & (x >> 1);
  }
  return bG | (bP << 1);
}

template <bool RAW, int AS>
__global__ void __launch_bounds__(CAT_CRT_THREADS)
k_crt(SegView sv, const uint32_t* __restrict__ res, uint64_t res_stride, uint32_t* __restrict__ out, uint32_t nblk,
      uint32_t* __restrict__ flags, uint32_t epoch, uint32_t polls, CopyList tails, const uint32_t* __restrict__ tin,
      uint32_t* __restrict__ tout, uint32_t* __restrict__ err) {
  __shared__ uint32_t tmp[16], tmp2[16];
  __shared__ uint4 xv[CAT_CRT_THREADS + 1];   // each thread's context for its right neighbour
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
  const uint64_t kb = (uint64_t)(b - first) * CAT_CRT_BLOCK;
  uint32_t ul[CAT_CRT_E];
  bool gk[CAT_CRT_E];
  bool G, P;
  crt_local<RAW, AS>(sg, r0, r1, r2, kb, xv, tmp, ul, gk, &G, &P, &s_spec);
  const uint32_t own = crt_block_pair(tmp);
  if (tid == 0)
    __hip_atomic_store(flags + b, (epoch << 3) | (own << 1) | 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // the carry in from the positions just below the block when they decide
  // it, else a look-back over the predecessors k = b-1, b-2, ... >= first
  // (block-uniform)
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
      // not published yet: recompute block k's pair from its residues
      uint32_t ul2[CAT_CRT_E];
      bool gk2[CAT_CRT_E];
      bool G2, P2;
      crt_local<RAW, AS>(sg, r0, r1, r2, (uint64_t)(k - first) * CAT_CRT_BLOCK, xv, tmp2, ul2, gk2, &G2, &P2,
                         &s_spec2);
      pair = crt_block_pair(tmp2);
    }
    if (pair & 1u) { cin = 1; done = true; }           // block k generates a carry
    else if (!(pair & 2u)) done = true;                 // block k absorbs any carry-in
    else if (k == first) done = true;                   // all-propagate back to the start
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
  const uint64_t k0 = kb + (uint64_t)tid * CAT_CRT_E;
  CrtWords r;
#pragma unroll
  for (int i = 0; i < CAT_CRT_E; i++) {
    unsigned co;
    r.w[i] = __builtin_addc(ul[i], 0u, c, &co);
    c = (co | (gk[i] ? 1u : 0u));
  }
  if (kb + CAT_CRT_BLOCK <= sg.len) {
    *(CrtWords*)(o + k0) = r;
  } else {
#pragma unroll
    for (int i = 0; i < CAT_CRT_E; i++)
      if (k0 + i < sg.len) o[k0 + i] = r.w[i];
  }
}
