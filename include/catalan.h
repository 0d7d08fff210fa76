/*
 * catalan.h — C ABI of the gfx950 (MI355X) library for exact Catalan numbers,
 * after "Exact Computation of the Catalan Number C(2,050,572,903)"
 * (arXiv 2601.11621).
 *
 * The library computes C(n) = (2n)! / (n! (n+1)!) (Sec. 1) by the paper's two
 * phases: Phase 1 lists every prime p <= 2n with its exponent
 * e_p = v_p((2n)!) - 2 v_p(n!) - v_p(n+1) (Sec. 2, Legendre's formula) and
 * groups the primes by exponent (Sec. 3.1, Alg. 1); Phase 2 forms
 * Q_e = prod_{p in G_e} p and P_e = Q_e^e with balanced product trees and
 * returns prod_e P_e (Sec. 3.2, Alg. 2).  Every multiplication is an exact
 * big-integer product on the GPU.
 *
 * Conventions (all entry points):
 *  - Big integers are little-endian arrays of uint32 limbs.
 *  - Pointers named d_* are device memory of the current HIP device, owned by
 *    the caller; h_* are host memory owned by the caller.  The library owns only
 *    its process-global tables (twiddle factors, plans and graphs it caches).
 *  - `stream` is a hipStream_t (NULL = the default stream).
 *  - d_work is caller-provided device scratch of at least the size the matching
 *    size query returns, 256-byte aligned; its contents are not preserved.
 *  - Return value: CAT_OK (0) or a negative cat_status.  On error, output
 *    contents are undefined and work already queued on `stream` may still run.
 *  - Thread safety: calls are serialised by an internal lock; results do not
 *    depend on the stream, the batch composition or the execution mode.
 */
#ifndef CATALAN_H
#define CATALAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cat_status;
enum {
  CAT_OK = 0,
  CAT_EINVAL = -1,     /* bad argument: n > CAT_N_MAX, NULL required pointer, length too large */
  CAT_ERANGE = -2,     /* a caller capacity is too small; the *needed output is set */
  CAT_ENOMEM = -3,     /* workspace too small, or a library allocation failed */
  CAT_EDEVICE = -4,    /* HIP runtime error; see cat_last_device_error() */
  CAT_EINTERNAL = -5,  /* a device-side invariant failed (negative exponent, carry out of a product) */
  CAT_EAGAIN = -6      /* cat_ticket_query: the queued work has not finished yet */
};

#define CAT_N_MAX 2147483647ull   /* 2n < 2^32, so primes fit in uint32 */
#define CAT_MAX_GROUPS 32         /* e_p <= log2(2n) < 32 */

/* Execution modes (flags of the *_ex entry points). */
#define CAT_MODE_BATCHED 0u  /* every product of one tree level in one launch per kernel stage */
#define CAT_MODE_PLAIN 1u    /* one product per launch (the unbatched reference form) */
#define CAT_MODE_GRAPH 2u    /* with BATCHED: capture the launches in a HIP graph, cached and replayed */

/* Initialise the library on `device` (the current device when < 0): computes
 * the NTT prime constants and uploads the twiddle tables.  Idempotent.  The
 * other entry points call it on first use. */
cat_status cat_init(int device);

/* Static description of a status code. */
const char* cat_strerror(cat_status s);

/* hipError_t of the last failing HIP call (0 if none). */
int cat_last_device_error(void);

/* Host-only size query for n (no device work).
 *  max_primes:      upper bound on the number of primes <= 2n (Dusart's bound).
 *  max_limbs:       upper bound on the limb count of C(n) (C(n) < 4^n).
 *  workspace_bytes: d_work size needed by catalan_factor and catalan_exact.
 * Any pointer may be NULL.  CAT_EINVAL if n > CAT_N_MAX. */
cat_status catalan_sizes(uint64_t n, size_t* max_primes, size_t* max_limbs, size_t* workspace_bytes);

/* Phase 1 (Sec. 3.1, Alg. 1; Sec. 2 for the exponents).
 * Writes the primes with e_p > 0 to d_primes grouped by exponent: group g holds
 * exponent h_exps[g] (ascending over g) and occupies d_primes[h_off[g] ..
 * h_off[g+1]) with its primes ascending.  h_exps needs CAT_MAX_GROUPS entries,
 * h_off CAT_MAX_GROUPS + 1.  Synchronises `stream`.
 * CAT_ERANGE if primes_cap < *n_primes (then *n_primes holds the count). */
cat_status catalan_factor(uint64_t n, uint32_t* d_primes, size_t primes_cap, uint32_t* h_exps,
                          uint64_t* h_off, uint32_t* n_groups, size_t* n_primes, void* d_work,
                          size_t work_bytes, void* stream);

/* Scratch needed by bigint_mul_batched for this batch (host-only). */
cat_status bigint_mul_workspace(uint32_t batch, const uint64_t* h_a_off, const uint64_t* h_b_off,
                                size_t* workspace_bytes);

/* Exact products c_i = a_i * b_i, i < batch (the multiplication inside every
 * BalancedProductTree step, Sec. 3.2).  Operand i is d_a[h_a_off[i] ..
 * h_a_off[i+1]) and d_b[h_b_off[i] .. h_b_off[i+1]); the product is written to
 * d_c[h_c_off[i] .. h_c_off[i] + la_i + lb_i), not normalised (leading zero
 * limbs kept).  Offsets are host arrays of batch+1 entries (h_c_off: batch).
 * Requirements: 1 <= la_i, lb_i and la_i + lb_i - 1 <= 2^27; the c ranges must
 * not overlap each other nor any operand.  flags: CAT_MODE_BATCHED or
 * CAT_MODE_PLAIN.
 * Asynchronous on `stream`: the call returns once the products are queued
 * (CAT_EINVAL / CAT_ENOMEM / CAT_EDEVICE for what the host can see); d_a, d_b,
 * d_c and d_work must stay untouched until that work has finished.  The
 * device-side check (a product needing more than la_i + lb_i limbs, which
 * exact arithmetic rules out) is read by bigint_mul_check.  The library
 * keeps the plans of the last 16 batch shapes (lengths and output offsets),
 * so a repeated shape costs no planning and no table upload; a new shape's
 * descriptor tables are uploaded on `stream`.
 * bigint_mul_check: synchronises `stream` and returns CAT_EINTERNAL if the
 * last product batch run in d_work failed its device check, else CAT_OK. */
cat_status bigint_mul_batched(uint32_t batch, const uint32_t* d_a, const uint64_t* h_a_off,
                              const uint32_t* d_b, const uint64_t* h_b_off, uint32_t* d_c,
                              const uint64_t* h_c_off, void* d_work, size_t work_bytes, void* stream);
cat_status bigint_mul_batched_ex(uint32_t batch, const uint32_t* d_a, const uint64_t* h_a_off,
                                 const uint32_t* d_b, const uint64_t* h_b_off, uint32_t* d_c,
                                 const uint64_t* h_c_off, void* d_work, size_t work_bytes, void* stream,
                                 uint32_t flags);
cat_status bigint_mul_check(void* d_work, void* stream);

/* C(n) (Sec. 1) by Phase 1 + Phase 2 (Alg. 1, Alg. 2) as normalised limbs:
 * d_limbs[0 .. *n_limbs), top limb nonzero, C(0) = C(1) = {1}.
 * d_limbs == NULL is a size query (sets *n_limbs to max_limbs, no device work).
 * CAT_ERANGE if cap < *n_limbs.  Synchronises `stream`.
 * catalan_exact uses CAT_MODE_BATCHED | CAT_MODE_GRAPH. */
cat_status catalan_exact(uint64_t n, uint32_t* d_limbs, size_t cap, size_t* n_limbs, void* d_work,
                         size_t work_bytes, void* stream);
cat_status catalan_exact_ex(uint64_t n, uint32_t* d_limbs, size_t cap, size_t* n_limbs, void* d_work,
                            size_t work_bytes, void* stream, uint32_t flags);

/* Allocation-free C(n), for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same result as catalan_exact, bit for bit, computed with
 * batched launches (no graph) in a static device scratch array of the
 * library instead of a caller workspace; the call allocates nothing on the
 * device and synchronises `stream` before returning.
 *  n:       as catalan_exact; CAT_ENOMEM when the workspace of n (see
 *           catalan_sizes) exceeds the scratch (every n <= 10^7 fits);
 *  d_limbs: device output of cap limbs, caller-owned, not NULL; C(n) as
 *           normalised limbs d_limbs[0 .. *n_limbs); CAT_ERANGE if
 *           cap < *n_limbs (then *n_limbs holds the length).
 * The scratch is one per GPU, shared by every call on that GPU, and keeps the
 * last call's contents (each call clears what it needs).  Calls in one
 * process are serialised by the library lock and end with a stream
 * synchronisation, so they never overlap; overlapping calls would race.
 * catalan_noalloc_max_bytes: the scratch size in bytes (host only). */
cat_status catalan_exact_noalloc(uint64_t n, uint32_t* d_limbs, size_t cap, size_t* n_limbs, void* stream);
cat_status catalan_noalloc_max_bytes(size_t* bytes);

/* sign(floor(x / 2^shift_bits) - y) in *sign (-1, 0, 1) for little-endian limb
 * vectors x[0..lx), y[0..ly) (leading zero limbs allowed).  d_work: at least
 * 16 bytes of device scratch.  Synchronises `stream`.  With x = C(n) and
 * y = 5^k this checks x >= 10^k as floor(x / 2^k) >= 5^k, which settles a
 * decimal digit count exactly (Table 1). */
cat_status bigint_compare(const uint32_t* d_x, size_t lx, uint64_t shift_bits, const uint32_t* d_y, size_t ly,
                          int32_t* sign, void* d_work, size_t work_bytes, void* stream);

/* Exact decimal digit count D of the limb vector d_x[0 .. n_limbs) (device,
 * leading zero limbs allowed; 0 counts as one digit), the count Table 1
 * reports for C(2,050,572,903).  D is settled on the device: 10^(D-1) <= x <
 * 10^D is checked as floor(x / 2^(D-1)) >= 5^(D-1) and floor(x / 2^D) < 5^D,
 * with the powers of five from the Phase-2 engine; the first guess comes from
 * the top limbs.  bigint_decimal_digits_workspace: host only, the d_work bytes
 * for n_limbs.  d_work: device, caller-owned, at least that size (CAT_ENOMEM
 * otherwise), must not overlap d_x.  Synchronises `stream`; CAT_EINVAL for
 * n_limbs > 2^27. */
cat_status bigint_decimal_digits_workspace(size_t n_limbs, size_t* workspace_bytes);
cat_status bigint_decimal_digits(const uint32_t* d_x, size_t n_limbs, uint64_t* digits, void* d_work,
                                 size_t work_bytes, void* stream);

/* Decimal text of x (the optional decimal output of Sec. 3.2): the digits of
 * the little-endian limb vector d_x[0 .. n_limbs) (device; leading zero limbs
 * allowed; n_limbs = 0 means 0), most significant first, no leading zeros
 * ("0" for zero), no terminator, as ASCII into d_out (device, cap bytes).
 * *n_chars is set to the digit count D whenever the conversion ran; CAT_ERANGE
 * if d_out is NULL or cap < D (nothing written), or if n_limbs > 2^27.
 * decimal_sizes: host only; an upper bound on D and the workspace bytes.
 * bigint_to_decimal: d_work of at least that many bytes (device, caller-owned,
 * contents undefined afterwards; CAT_ENOMEM if smaller); d_x, d_out and d_work
 * must not overlap; synchronises `stream`; CAT_EINTERNAL if a device check
 * failed.  The first call for a given (n_limbs, d_x, d_out, cap, d_work)
 * captures the conversion as a HIP graph that later calls with the same
 * arguments replay (the library keeps up to 32 such graphs). */
cat_status decimal_sizes(size_t n_limbs, size_t* max_chars, size_t* workspace_bytes);
cat_status bigint_to_decimal(const uint32_t* d_x, size_t n_limbs, char* d_out, size_t cap, size_t* n_chars,
                             void* d_work, size_t work_bytes, void* stream);

/* Phase 2 on a caller's factorisation (Alg. 2, the reconstruction engine):
 * N = prod_g (prod of the entries of group g)^(h_exps[g]).  Group g is
 * d_entries[h_off[g] .. h_off[g+1]) (device, uint32, nonzero, e.g. the primes of
 * one exponent read from a factorisation file); h_exps strictly ascending, at
 * most CAT_MAX_GROUPS nonempty groups (empty ones are skipped), h_off[0] = 0.
 * max_entry_bits (1..32) bounds the bit length of every entry and sizes the
 * workspace (CAT_EINVAL if an entry is longer).
 * prime_power_product_sizes: host only, bounds on the result limbs and the
 *   workspace bytes.
 * prime_power_product: N as normalised limbs into d_limbs (cap limbs);
 *   flags CAT_MODE_BATCHED or CAT_MODE_PLAIN; synchronises `stream`.
 *   CAT_ERANGE if N could exceed the 2^27-coefficient transform or cap. */
cat_status prime_power_product_sizes(const uint32_t* h_exps, const uint64_t* h_off, uint32_t ngroups,
                                     uint32_t max_entry_bits, size_t* max_limbs, size_t* workspace_bytes);
cat_status prime_power_product(const uint32_t* d_entries, const uint32_t* h_exps, const uint64_t* h_off,
                               uint32_t ngroups, uint32_t max_entry_bits, uint32_t* d_limbs, size_t cap,
                               size_t* n_limbs, void* d_work, size_t work_bytes, void* stream, uint32_t flags);

/* Factorial ratios N = a_1! ... a_k! / (b_1! ... b_m!) (Sec. 6.3: the exponent
 * of p is sum_i v_p(a_i!) - sum_j v_p(b_j!), and the reconstruction is the
 * Phase 2 of C(n) unchanged): binomial and multinomial coefficients,
 * factorials, super-factorials of up to 32 terms.  a[0..k), b[0..m) are host
 * arrays, k, m <= CAT_RATIO_MAX_TERMS, every argument < 2^32.
 *
 * factorial_ratio_sizes: host only; upper bounds on the grouped prime entries,
 *   on the limbs of N, and the workspace bytes.
 * factorial_ratio_factor: Phase 1.  The primes with v_p(N) > 0 are grouped by
 *   the bits of their exponents: group g holds, ascending, the primes whose
 *   exponent has bit b set, and h_exps[g] = 2^b (bits ascending, at most 32
 *   groups), so that N = prod_g (prod of group g)^(h_exps[g]).  Otherwise as
 *   catalan_factor.
 * factorial_ratio_exact: N as normalised limbs (N = 1 gives {1}); flags
 *   CAT_MODE_BATCHED or CAT_MODE_PLAIN; d_limbs == NULL is a size query.
 *   Synchronises `stream`.
 * Errors: CAT_EINVAL for bad arguments and for a ratio that is not an integer
 * (some exponent negative, found by Phase 1); CAT_ERANGE when an exponent
 * reaches 2^32, a product would exceed the 2^27-coefficient transform, or a
 * capacity is too small. */
#define CAT_RATIO_MAX_TERMS 32
cat_status factorial_ratio_sizes(const uint64_t* a, uint32_t k, const uint64_t* b, uint32_t m, size_t* max_primes,
                                 size_t* max_limbs, size_t* workspace_bytes);
cat_status factorial_ratio_factor(const uint64_t* a, uint32_t k, const uint64_t* b, uint32_t m, uint32_t* d_primes,
                                  size_t primes_cap, uint32_t* h_exps, uint64_t* h_off, uint32_t* n_groups,
                                  size_t* n_primes, void* d_work, size_t work_bytes, void* stream);
cat_status factorial_ratio_exact(const uint64_t* a, uint32_t k, const uint64_t* b, uint32_t m, uint32_t* d_limbs,
                                 size_t cap, size_t* n_limbs, void* d_work, size_t work_bytes, void* stream,
                                 uint32_t flags);

/* Asynchronous C(n), for request loops that keep many computations in
 * flight on several streams (every call returns without waiting for the GPU):
 *  catalan_begin    queues Phase 1 of n on `stream` in d_work (sized by
 *                   catalan_sizes) and returns a ticket;
 *  cat_ticket_query CAT_OK once the ticket's queued work has finished,
 *                   CAT_EAGAIN before;
 *  catalan_continue after Phase 1 finished: plans Phase 2 from the group
 *                   counts (host only, no device allocation) and queues it with
 *                   the normalisation and the copy of up to `cap` limbs of C(n)
 *                   into d_limbs (limbs past *n_limbs are zero);
 *  catalan_end      after Phase 2 was queued: waits for it, returns the limb
 *                   count and checks the device error word (CAT_ERANGE if
 *                   cap was too small).  It releases the ticket on every
 *                   path, errors included (CAT_EINVAL when called before
 *                   catalan_continue succeeded: then it first waits for the
 *                   ticket's stream); the ticket must not be used again;
 *  cat_ticket_release drops a ticket that catalan_end has not released, at
 *                   any point: it waits until everything queued on the
 *                   ticket's stream has finished (also the part of Phase 2 a
 *                   failed catalan_continue may have queued), so d_work and
 *                   d_limbs are free to reuse when it returns.
 * d_work and d_limbs must stay untouched until catalan_end.  The same results
 * as catalan_exact, bit for bit. */
typedef struct cat_ticket_s* cat_ticket;
cat_status catalan_begin(uint64_t n, void* d_work, size_t work_bytes, void* stream, cat_ticket* ticket);
cat_status cat_ticket_query(cat_ticket ticket);
cat_status catalan_continue(cat_ticket ticket, uint32_t* d_limbs, size_t cap);
cat_status catalan_end(cat_ticket ticket, size_t* n_limbs);
cat_status cat_ticket_release(cat_ticket ticket);

/* Batches of C(n) requests (continuous batching in a request loop): the
 * requests' Phase 1 runs request by request, then Phase 2 of all of them is
 * planned together, so that each tree level of every request, and each step
 * of their powers and outer products, is one launch per kernel stage (at most
 * CAT_MAX_GROUPS exponent groups per plan; a batch with more runs as several
 * plans one after another on the stream).  Results are bit-identical to
 * catalan_exact for every n.
 *  catalan_batch_sizes:    host only; d_work bytes for the k <= CAT_BATCH_MAX
 *                          values ns[0..k);
 *  catalan_batch_begin:    queues Phase 1 of every request on `stream` in
 *                          d_work and returns a ticket (cat_ticket_query and
 *                          cat_ticket_release work on it);
 *  catalan_batch_continue: after Phase 1 finished: plans and queues Phase 2
 *                          and the copy of up to caps[r] limbs of C(ns[r]) to
 *                          d_limbs[r] (device, k pointers in a host array);
 *  catalan_batch_end:      after Phase 2 was queued: waits for it and sets
 *                          n_limbs[r] and, if req_status is not NULL, the
 *                          status of each request (CAT_ERANGE if caps[r] was
 *                          too small, CAT_EINTERNAL if a device check failed);
 *                          returns the first request's error or CAT_OK, and
 *                          releases the ticket on every path.
 * d_work and the outputs must stay untouched until catalan_batch_end. */
#define CAT_BATCH_MAX 32
cat_status catalan_batch_sizes(uint32_t k, const uint64_t* ns, size_t* workspace_bytes);
cat_status catalan_batch_begin(uint32_t k, const uint64_t* ns, void* d_work, size_t work_bytes, void* stream,
                               cat_ticket* ticket);
cat_status catalan_batch_continue(cat_ticket ticket, uint32_t* const* d_limbs, const size_t* caps);
cat_status catalan_batch_end(cat_ticket ticket, size_t* n_limbs, cat_status* req_status);

/* Reusable plans for repeated batches of the same shape (the batched form
 * of a tree level).  cat_mul_plan_create buckets the products by transform
 * length (schoolbook for la, lb <= 128; LDS-resident NTT up to 2^12
 * coefficients; four-step NTT above) and uploads the descriptor tables;
 * cat_mul_plan_exec queues the products on `stream` (with CAT_MODE_GRAPH the
 * launch sequence is captured on first use and replayed as one HIP graph per
 * set of pointers); cat_mul_plan_check synchronises `stream` and reports a
 * device-side overflow (CAT_EINTERNAL).  flags as in bigint_mul_batched_ex
 * plus CAT_MODE_GRAPH.  A plan is used by one thread at a time. */
typedef struct cat_mul_plan_s* cat_mul_plan;
cat_status cat_mul_plan_create(uint32_t batch, const uint64_t* h_a_off, const uint64_t* h_b_off,
                               const uint64_t* h_c_off, uint32_t flags, cat_mul_plan* plan,
                               size_t* workspace_bytes);
cat_status cat_mul_plan_exec(cat_mul_plan plan, const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_c,
                             void* d_work, size_t work_bytes, void* stream);
cat_status cat_mul_plan_check(cat_mul_plan plan, void* d_work, void* stream);
cat_status cat_mul_plan_destroy(cat_mul_plan plan);

/* Fingerprints of a limb vector (verification, Sec. 6 "modular checks"):
 * h_res[0] = x mod (2^32 - 5), h_res[1] = x mod (2^32 + 1), h_res[2] = x mod (2^32 - 1).
 * d_work needs 24 * ceil(n / 4096) + 256 bytes.  Synchronises `stream`. */
cat_status bigint_residues(const uint32_t* d_x, size_t n, uint64_t* h_res, void* d_work,
                           size_t work_bytes, void* stream);

/* Statistics of the last catalan_exact / bigint_mul_batched call on this
 * process (host side): number of products, kernel launches (graph nodes count
 * once per kernel), and the sum of la+lb over all products; outer_level is
 * the level of Q_1's product tree at which R = prod_{e>=2} P_e entered as a
 * node (-1: C was formed as Q_1 R after the tree; 0 for calls without a
 * product tree, such as bigint_mul_batched). */
typedef struct {
  uint64_t products;
  uint64_t launches;
  uint64_t product_limbs;
  uint64_t n_primes;
  uint32_t levels;
  uint32_t graph_replayed;
  int32_t outer_level;
  uint32_t reserved;
} cat_stats;
cat_status cat_get_stats(cat_stats* out);

/* Product schedule per transform-length bucket (the autotuner's output).
 * Products with la, lb <= school_max use the schoolbook kernel; otherwise
 * bucket k = ceil(log2(la + lb - 1)) (at least 6) selects cls[k]:
 * 1 = one workgroup holds the whole transform (k <= 14) in a tile of
 * 2^max(k, log_row[k]) slots per operand (log_row 12..14: 2^(log_row - k)
 * products and 2^log_row / 16 threads per workgroup), 2 = four-step
 * transform with rows of 2^log_row[k] words (8..14, < k) and column passes of
 * at most 2^log_pass[k] points (4..10).  Every schedule gives the same bits.
 * cat_tune_set(NULL) restores the defaults; CAT_EINVAL for an invalid table.
 * Setting a table drops the cached C(n) plans. */
typedef struct {
  uint32_t school_max;
  uint8_t cls[28];
  uint8_t log_row[28];
  uint8_t log_pass[28];
} cat_tuning;
cat_status cat_tune_set(const cat_tuning* t);
cat_status cat_tune_get(cat_tuning* t);

/* Fused launches of one-workgroup transforms.  Tree levels (the batched form
 * of C(n) and of the other Phase-2 entry points): the consecutive levels
 * above the schoolbook levels whose products are one-workgroup transforms of
 * at most 2^max_logn coefficients run in one kernel that keeps each
 * 4,096-leaf tile of a group in LDS from the first of them to the last
 * (three-prime transforms, Garner recombination and carries inside the
 * workgroup), in trees of at most 2^22 leaves.  Generic batches
 * (bigint_mul_batched, batched form): the buckets of at most 2^max_logn
 * coefficients in one launch over a tile table.
 * max_logn = 0 turns both off (every level or bucket is then a transform
 * launch and a carry launch); 4..12 turns both on up to 2^max_logn;
 * CAT_FUSED_DEFAULT restores the defaults: generic batches fused up to 2^12,
 * tree levels not fused (the separate launches are at least as fast).  The
 * result is the same bit for bit either way.  Cached C(n) plans are dropped. */
#define CAT_FUSED_DEFAULT 0xFFFFFFFFu
cat_status cat_fused_levels_set(uint32_t max_logn);

/* Order of the outer product (Alg. 2: C is the product of the P_e).  With
 * on = 1 (the default) R = prod_{e>=2} P_e, which is short, enters the
 * product tree of Q_1 as one more node of 2^j limbs (R, then zero limbs) at
 * a level j two above the completion of the last group with e >= 2, so that
 * the top product of that tree is C itself; the powers and R run beside the
 * tree's levels below j.  It is used when Q_1's tree has at least 2^(j+2)
 * leaves and the arenas hold 2^j more (otherwise, and with on = 0, C is the
 * product Q_1 R after the tree).  The result is the same bit for bit either
 * way.  Cached C(n) plans are dropped.  Returns CAT_EINVAL above 1. */
cat_status cat_outer_node_set(uint32_t on);

/* Prime set of the transform products (Sec. 3.2: every multiplication of
 * the reconstruction phase).  Products whose transform has at most
 * 2^max_logn points use three primes below 2^30 (105 2^23 + 1,
 * 107 2^23 + 1, 119 2^23 + 1), whose 4q < 2^32 lets the butterflies leave
 * their values unreduced between operations; larger ones use the three
 * primes in (2^31, 2^32).  Both cover every coefficient in their range
 * (products of min(la, lb) <= 2^22 limbs for the first, <= 2^26 for the
 * second), so the result is the same bit for bit either way.
 * max_logn = 0 uses the second set everywhere; otherwise at most 23
 * (default 23).  Cached C(n) and batched-multiply plans are dropped.
 * Returns CAT_EINVAL above 23. */
cat_status cat_lazy_primes_set(uint32_t max_logn);

/* Carry look-back between CRT blocks (diagnostics and tests).  A block reads
 * the generate / propagate pair of the block before it from a flag that block
 * publishes, polling it at most `polls` times (at most 2^20), and otherwise
 * recomputes the pair from that block's residues; the result is the same
 * either way, and polls = 0 always recomputes.  CAT_POLLS_AUTO (the default)
 * recomputes at once in launches of at most 2^15 blocks and polls up to 16
 * times in larger ones.  Cached C(n) plans are dropped; existing product
 * plans keep the value they were recorded with. */
#define CAT_POLLS_AUTO 0xFFFFFFFFu
cat_status cat_lookback_polls_set(uint32_t polls);

/* Kernel timer (measurement only).  cat_timer_set(name) brackets every later
 * launch of the named kernel ("k_ntt_lds", "k_row", "k_pass_fwd", "k_pass_inv",
 * "k_tree_fused", "k_crt", "k_school", "k_leaf", "k_residues") with HIP
 * events on the stream it is launched on, outside graph capture; NULL or ""
 * stops it.  Each call resets the
 * counters.  cat_timer_get waits for the recorded events and returns the summed
 * kernel time, the launch count and the algorithmic work of those launches
 * (radix-2 butterflies for NTT kernels, limbs for k_crt, k_school and
 * k_residues, nodes for k_leaf).  Calls of catalan_exact_noalloc are not
 * timed. */
cat_status cat_timer_set(const char* kernel);
cat_status cat_timer_get(double* ms, uint64_t* launches, double* work);

/* VALU issue-rate probe (measurement only).  Times one launch of a kernel in
 * which every lane runs iters x 32 dependent-chain copies of one instruction
 * form, 8 independent chains per lane and 8 waves per SIMD on every compute
 * unit, on the default stream after one untimed launch, and returns the lane
 * operations per second (and the launch time in ms when `ms` is not NULL).
 * The integer forms are the ones the transform butterflies are built from, so
 * the figures state the cost of a butterfly in cycles.  op: CAT_VALU_* below;
 * iters in 1 .. 2^20.  Allocates and frees a small device buffer.
 * CAT_EINVAL for a bad op, iters or a NULL rate pointer. */
enum {
  CAT_VALU_ADD_U32 = 0,     /* v_add_u32 */
  CAT_VALU_MIN_U32 = 1,     /* v_min_u32 */
  CAT_VALU_MUL_LO_U32 = 2,  /* v_mul_lo_u32 */
  CAT_VALU_MUL_HI_U32 = 3,  /* v_mul_hi_u32 */
  CAT_VALU_MAD_U64_U32 = 4, /* v_mad_u64_u32 */
  CAT_VALU_FMA_F32 = 5,     /* v_fma_f32, for reference (2 flops per lane-op; the published fp32 vector peak assumes packed FMAs) */
  CAT_VALU_NOPS = 6
};
cat_status cat_valu_rate(int op, uint32_t iters, double* lane_ops_per_s, double* ms);

#ifdef __cplusplus
}
#endif
#endif /* CATALAN_H */
