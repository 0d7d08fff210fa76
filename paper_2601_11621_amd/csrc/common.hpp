// Shared definitions of the gfx950 Catalan library: modular arithmetic for the
// three NTT primes, descriptor structs, launch constants.
//
// Every multiplication of the reconstruction phase (Sec. 3.2, Alg. 2 of
// arXiv 2601.11621) is an exact product of little-endian uint32 limb vectors.
// Large products go through a cyclic convolution modulo three primes
//   p0 = 3*2^30+1, p1 = 13*2^28+1, p2 = 29*2^27+1   (all in (2^31, 2^32),
// 2-adicity >= 27, product ~2^95.1), one 32-bit limb per coefficient, and are
// recombined with Garner's CRT.  Exactness: a coefficient of a la x lb limb
// product is < min(la,lb) * 2^64 <= 2^90 for operands up to 2^26 limbs, below
// p0*p1*p2; the transform length N = 2^k <= 2^27 needs 2-adicity >= k.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define CAT_NPRIMES 3
#define CAT_MAX_LOGN 27
#define CAT_MAX_GROUPS 32       // e_p <= log2(2n) < 32
#define CAT_LDS_LOGT 12         // row length of the LDS-resident transforms
#define CAT_LEAF_LF 6         // tree levels folded into the leaf kernel (nodes of 2^LF leaves)
#define CAT_CRT_E 3             // limbs per thread in the CRT/carry kernel (>= 3)
#define CAT_CRT_THREADS 256
#define CAT_CRT_BLOCK (CAT_CRT_E * CAT_CRT_THREADS)

// ----------------------------------------------------------------------------
// Per-prime constants (host computes, device reads from __constant__).
// Montgomery radix R = 2^32.  A "twiddle pair" (w, wq) holds w = W*R mod p
// (Montgomery form of W) and wq = w * p^-1 mod 2^32; mul_tw(a, w, wq) = a*W
// mod p for every 32-bit a.
// ----------------------------------------------------------------------------
struct PrimeC {
  uint32_t p;
  uint32_t pinv;          // p^-1 mod 2^32
  uint32_t w16[8], w16q[8];    // omega_16^i (forward), Montgomery pairs
  uint32_t iw16[8], iw16q[8];  // omega_16^-i (inverse)
};

struct CrtC {
  // Garner: x0 = r0; x1 = (r1 - x0) * c01 mod p1; x2 = (r2 - x0) * c012 - x1 * c12 mod p2
  uint32_t c01, c01q;       // p0^-1 mod p1 (Montgomery pair for p1)
  uint32_t c12, c12q;       // p1^-1 mod p2 (Montgomery pair for p2)
  uint32_t c012, c012q;     // (p0*p1)^-1 mod p2 (Montgomery pair for p2)
  uint32_t p0, p1;
};

// ----------------------------------------------------------------------------
// Modular arithmetic, p odd, 2^31 < p < 2^32.  Inputs of add/sub reduced.
// ----------------------------------------------------------------------------
__device__ __forceinline__ uint32_t sub_mod(uint32_t a, uint32_t b, uint32_t p) {
  uint32_t d;
  const bool borrow = __builtin_usub_overflow(a, b, &d);   // one v_sub_co_u32
  return borrow ? d + p : d;
}
__device__ __forceinline__ uint32_t add_mod(uint32_t a, uint32_t b, uint32_t p) {
  return sub_mod(a, p - b, p);   // p - b in (0, p]
}

// Montgomery multiplication with a precomputed companion (Montgomery 1985,
// with the quotient digit precomputed as in Shoup's method): returns a*w/R
// mod p in [0,p) for any 32-bit a and w < p.
__device__ __forceinline__ uint32_t mul_tw(uint32_t a, uint32_t w, uint32_t wq, uint32_t p) {
  const uint32_t m = a * wq;
  const uint32_t hi = __umulhi(a, w);
  const uint32_t mh = __umulhi(m, p);
  return sub_mod(hi, mh, p);   // hi, mh < p
}
// General Montgomery product a*b/R mod p, a,b < p.
__device__ __forceinline__ uint32_t mont_mul(uint32_t a, uint32_t b, uint32_t p, uint32_t pinv) {
  uint32_t lo = a * b;
  uint32_t hi = __umulhi(a, b);
  const uint32_t m = lo * pinv;
  const uint32_t mh = __umulhi(m, p);
  return sub_mod(hi, mh, p);   // hi, mh < p
}
// limb (any 32-bit value) reduced mod p: 2^32 < 2p, so one subtraction suffices
__device__ __forceinline__ uint32_t reduce_limb(uint32_t x, uint32_t p) { return x >= p ? x - p : x; }

// ----------------------------------------------------------------------------
// The second prime set: q0 = 105*2^23+1, q1 = 107*2^23+1, q2 = 119*2^23+1, all
// below 2^30 (product ~2^89.35, 2-adicity 23).  A coefficient of a product
// with min(la, lb) <= 2^22 limbs is below 2^22 (2^32-1)^2 < 2^86, so
// transforms of up to 2^23 points can use it.  With 4q < 2^32, residues may
// stay unreduced between butterflies (Harvey 2014, "Faster arithmetic for
// number-theoretic transforms"): forward passes keep values in [0, 2q),
// inverse passes in [0, 4q), and only the outputs that leave the transform
// are reduced to [0, q).  Twiddles from tables are Shoup pairs (w in normal
// form, w' = floor(w 2^32 / q)); twiddles computed on the fly stay Montgomery
// pairs as in the first set.
// ----------------------------------------------------------------------------
#define CAT_LAZY_MAX_LOGN 23

// x < 2m -> x mod m (one subtraction, m = q or 2q)
__device__ __forceinline__ uint32_t red2(uint32_t x, uint32_t m) {
  uint32_t d;
  return __builtin_usub_overflow(x, m, &d) ? x : d;
}
// a*w mod q in [0, 2q) for every 32-bit a (Shoup): w < q, ws = floor(w 2^32 / q)
__device__ __forceinline__ uint32_t shoup(uint32_t a, uint32_t w, uint32_t ws, uint32_t q) {
  return a * w - __umulhi(a, ws) * q;
}
// a*w/2^32 mod q in (0, 2q) for every 32-bit a, w < q Montgomery form,
// wq = w * q^-1 mod 2^32: hi(a w) - hi(m q) lies in (-q, q)
__device__ __forceinline__ uint32_t mont_lazy(uint32_t a, uint32_t w, uint32_t wq, uint32_t q) {
  return __umulhi(a, w) - __umulhi(a * wq, q) + q;
}
// x*y/2^32 mod q in (0, 2q) for x, y < 2q (x y < 4q^2, so hi(x y) < q)
__device__ __forceinline__ uint32_t mont_mul_lazy(uint32_t x, uint32_t y, uint32_t q, uint32_t qinv) {
  const uint32_t lo = x * y;
  return __umulhi(x, y) - __umulhi(lo * qinv, q) + q;
}
// limb (any 32-bit value, < 8q) into [0, 2q)
__device__ __forceinline__ uint32_t limb_lazy(uint32_t x, uint32_t q) { return red2(red2(x, 4 * q), 2 * q); }
// [0, 4q) -> [0, q)
__device__ __forceinline__ uint32_t red4(uint32_t x, uint32_t q) { return red2(red2(x, 2 * q), q); }

// ----------------------------------------------------------------------------
// Descriptors of a batch of products c = a * b.
// Explicit: a table in device memory.  Tree: computed from the level of a
// forest of balanced product trees (one tree per exponent group): node i of
// group g at level j covers leaves [i*2^j, min((i+1)*2^j, K_g)) and has exactly
// that many limbs; its parent's output sits at the left child's offset.
// ----------------------------------------------------------------------------
struct MulDesc {
  uint64_t a_off, b_off, c_off, r_off;  // r_off: position in the residue arrays
  uint32_t la, lb;
};

struct TreeLevel {
  uint32_t ngroups;
  uint32_t j;                           // input node size 2^j limbs
  uint64_t base[CAT_MAX_GROUPS];        // arena offset of group g
  uint64_t K[CAT_MAX_GROUPS];           // leaves (limbs) of group g
  uint64_t mpref[CAT_MAX_GROUPS + 1];   // prefix count of products per group
};

#define CAT_INLINE_DESC 16

// Uniform batch: product i reads a at a0 + i*sa and b at b0 + i*sb (la, lb
// limbs each) and writes c at c0 + i*sc; residues at i*(la+lb).
struct UniDesc {
  uint64_t a0, sa, b0, sb, c0, sc;
  uint32_t la, lb;
};

struct DescView {
  const MulDesc* table;  // device table (large explicit batches), or
  uint32_t ninl;         // > 0: explicit descriptors carried in the kernel arguments, or
  uint32_t uni;          // > 0: uniform batch, or
  MulDesc inl[CAT_INLINE_DESC];
  UniDesc u;
  TreeLevel tree;        // tree mode
  __device__ __forceinline__ MulDesc get(uint64_t i) const {
    if (table) return table[i];
    if (ninl) return inl[i];
    if (uni) {
      MulDesc d;
      d.a_off = u.a0 + i * u.sa;
      d.b_off = u.b0 + i * u.sb;
      d.c_off = u.c0 + i * u.sc;
      d.r_off = i * ((uint64_t)u.la + u.lb);
      d.la = u.la;
      d.lb = u.lb;
      return d;
    }
    uint32_t g = 0;
    while (g + 1 < tree.ngroups && i >= tree.mpref[g + 1]) g++;
    uint64_t il = i - tree.mpref[g];
    uint64_t sz = 1ull << tree.j;
    MulDesc d;
    d.a_off = tree.base[g] + 2 * il * sz;
    d.b_off = d.a_off + sz;
    d.c_off = d.a_off;
    d.r_off = d.a_off;
    d.la = (uint32_t)sz;
    uint64_t rem = tree.K[g] - (2 * il + 1) * sz;
    d.lb = (uint32_t)(rem < sz ? rem : sz);
    return d;
  }
};

// CRT/carry segments: out[out_pos + k] for k < len from residues at res_pos + k
// (radix-10^9 products also add the digits add[add_pos + k] for k < add_len).
struct CrtSeg {
  uint64_t out_pos, res_pos, len;
  uint64_t add_pos, add_len;
};

// Bits of the device error word
#define CAT_DEVERR_CARRY_OUT 1u     // a product overflowed its la+lb limbs
#define CAT_DEVERR_NEG_EXP 2u       // negative exponent (C(n) not integral)
#define CAT_DEVERR_BOUNDS 4u        // a prime count exceeded its buffer
#define CAT_DEVERR_SCAN 8u          // a carry look-back gave up waiting (never expected)
#define CAT_DEVERR_RANGE 16u        // an exponent reached 2^32

// Ranges copied unchanged from one arena to the other (the last node of a
// group with an odd node count is carried up a level).  Kernels that take a
// CopyList run extra workgroups for it: workgroup cb (counted from the first
// copy workgroup) copies chunk cb of TAIL_CHUNK words, ranges in order.
#define TAIL_CHUNK 4096u
struct CopyList {
  uint32_t n;
  uint64_t off[CAT_MAX_GROUPS];
  uint64_t len[CAT_MAX_GROUPS];
};
inline uint32_t tail_blocks(const CopyList& cl) {
  uint64_t b = 0;
  for (uint32_t r = 0; r < cl.n; r++) b += (cl.len[r] + TAIL_CHUNK - 1) / TAIL_CHUNK;
  return (uint32_t)b;
}
__device__ __forceinline__ void copy_tail_block(const CopyList& cl, const uint32_t* __restrict__ in,
                                                uint32_t* __restrict__ out, uint32_t cb) {
  for (uint32_t r = 0; r < cl.n; r++) {
    const uint64_t nb = (cl.len[r] + TAIL_CHUNK - 1) / TAIL_CHUNK;
    if (cb < nb) {
      const uint64_t k0 = (uint64_t)cb * TAIL_CHUNK, k1 = min(k0 + (uint64_t)TAIL_CHUNK, cl.len[r]);
      for (uint64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x) out[cl.off[r] + k] = in[cl.off[r] + k];
      return;
    }
    cb -= (uint32_t)nb;
  }
}
