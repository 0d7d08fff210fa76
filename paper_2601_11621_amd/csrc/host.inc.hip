// Host side of the library: constants, workspace layout, the reconstruction
// planner (Sec. 3.2, Alg. 2) and the executor (batched, plain or graph).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/catalan.h"

// ----------------------------------------------------------------------------
// library state
// ----------------------------------------------------------------------------
namespace {

static const uint32_t kP[CAT_NPRIMES] = {3221225473u, 3489660929u, 3892314113u};
static const uint32_t kGen[CAT_NPRIMES] = {5u, 3u, 3u};   // primitive roots
// the second (lazy) set, ascending as Garner's method needs: 105 2^23 + 1,
// 107 2^23 + 1, 119 2^23 + 1
static const uint32_t kQ[CAT_NPRIMES] = {880803841u, 897581057u, 998244353u};
static const uint32_t kQGen[CAT_NPRIMES] = {26u, 3u, 3u};

struct Stage;
struct Plan;
struct MulPlanImpl;

// Constants and twiddle tables of one prime set.
struct PrimeSet {
  PrimeC prc[CAT_NPRIMES];
  CrtC crt;
  RootsC roots;
  uint2* tws = nullptr;
  uint2* itws = nullptr;
  uint2* tw2lo = nullptr;
  uint32_t* tw2hi = nullptr;
  uint2* itw2lo = nullptr;
  uint32_t* itw2hi = nullptr;
};

struct Lib {
  bool inited = false;
  int device = -1;
  PrimeSet set[2];   // 0: primes in (2^31, 2^32); 1: the lazy set below 2^30
  void* pin = nullptr;          // pinned host staging for small D2H
  int last_err = 0;
  std::recursive_mutex mu;
  cat_stats stats{};
  std::map<uint64_t, Plan*> plans;
  std::vector<uint64_t> plan_order;
  std::map<uint64_t, Plan*> noalloc_plans;      // plans of catalan_exact_noalloc
  std::vector<uint64_t> noalloc_order;
  void* scratch_ptr = nullptr;                  // device address of `scratch` on g.device
  bool in_noalloc = false;                      // a catalan_exact_noalloc call is running
  hipStream_t cap_stream = nullptr;
  hipStream_t side_stream = nullptr;            // second branch of captured calls
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::vector<hipEvent_t> dec_ev;               // decimal conversion: P_j ready
  // kernel timer: events around every launch of one named kernel
  std::string timer_name;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> timer_ev;
  size_t timer_used = 0;
  double timer_work = 0;
};
Lib g;

// Device scratch of the allocation-free entry point catalan_exact_noalloc,
// for callers that cannot allocate device memory.  It holds the workspace
// layout of one C(n) call (primes, tree arenas, residues, transform scratch,
// control block) for every n whose workspace fits (n <= 10^7 does).  Each GPU
// that loads the library holds its own copy until the process ends.  In host
// code `scratch` only stands in for the symbol: its device address comes from
// hipGetSymbolAddress at initialisation (g.scratch_ptr), and that address is
// what the kernels receive.
#define CAT_NOALLOC_BYTES ((size_t)144 << 20)
static __device__ __align__(256) unsigned char scratch[CAT_NOALLOC_BYTES];

// Brackets a launch of kernel `name` with events when the timer watches it.
struct KTime {
  bool on = false;
  hipStream_t st;
  size_t idx = 0;
  KTime(const char* name, hipStream_t s, double work) : st(s) {
    if (g.in_noalloc || g.timer_name.empty() || g.timer_name != name) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    if (g.timer_used == g.timer_ev.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
      g.timer_ev.push_back({a, b});
    }
    idx = g.timer_used++;
    g.timer_work += work;
    on = hipEventRecord(g.timer_ev[idx].first, s) == hipSuccess;
  }
  ~KTime() {
    if (on) (void)hipEventRecord(g.timer_ev[idx].second, st);
  }
};
// radix-2 butterflies of `t` length-2^logN transforms
double bfly(double t, int logN) { return t * (double)(1ull << logN) / 2.0 * logN; }

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) {                         \
      g.last_err = (int)e_;                         \
      return CAT_EDEVICE;                           \
    }                                               \
  } while (0)
#define STCHK(x)                  \
  do {                            \
    cat_status s_ = (x);          \
    if (s_ != CAT_OK) return s_;  \
  } while (0)
#define LAUNCHCHK() HIPCHK(hipGetLastError())

// ---------------------------------------------------------------- host modular arithmetic
uint32_t h_mulmod(uint32_t a, uint32_t b, uint32_t p) { return (uint32_t)((uint64_t)a * b % p); }
uint32_t h_powmod(uint32_t b, uint64_t e, uint32_t p) {
  uint32_t r = 1 % p;
  b %= p;
  while (e) {
    if (e & 1) r = h_mulmod(r, b, p);
    b = h_mulmod(b, b, p);
    e >>= 1;
  }
  return r;
}
uint32_t h_inv(uint32_t a, uint32_t p) { return h_powmod(a, p - 2, p); }
uint32_t h_inv32(uint32_t p) {  // p^-1 mod 2^32 (Newton)
  uint32_t x = p;
  for (int i = 0; i < 5; i++) x *= 2u - p * x;
  return x;
}
uint32_t h_mont(uint32_t W, uint32_t p) { return (uint32_t)(((uint64_t)(W % p) << 32) % p); }
void h_pair(uint32_t W, const PrimeC& pc, uint32_t* w, uint32_t* wq) {
  *w = h_mont(W, pc.p);
  *wq = *w * pc.pinv;
}
uint2 h_pair2(uint32_t W, const PrimeC& pc) {
  uint2 r;
  h_pair(W, pc, &r.x, &r.y);
  return r;
}

// Workgroups of the result length scan (k_top_nonzero, 256 threads, one
// atomic each): 512 up to 2^24 limbs, then one per 2^15 limbs up to 4,096, so
// that a long result is read by enough waves to reach HBM bandwidth.
uint32_t top_scan_blocks(uint64_t cap) {
  const uint64_t want = std::min<uint64_t>(std::max<uint64_t>(cap >> 15, 512), 4096);
  return (uint32_t)std::max<uint64_t>(std::min<uint64_t>((cap + 255) / 256, want), 1);
}

uint64_t isqrt64(uint64_t x) {
  uint64_t r = (uint64_t)std::sqrt((double)x);
  while (r * r > x) r--;
  while ((r + 1) * (r + 1) <= x) r++;
  return r;
}
int ceil_log2(uint64_t x) {
  int k = 0;
  while ((1ull << k) < x) k++;
  return k;
}

// Upper bound on pi(x): Dusart (2010) for x >= 355991, Rosser-Schoenfeld below.
uint64_t pi_bound(uint64_t x) {
  if (x < 17) return 8;
  const double lx = std::log((double)x);
  double b;
  if (x >= 355991) b = (double)x / lx * (1.0 + 1.0 / lx + 2.51 / (lx * lx));
  else b = 1.25506 * (double)x / lx;
  return (uint64_t)b + 16;
}

cat_status set_device() {
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != g.device) HIPCHK(hipSetDevice(g.device));
  return CAT_OK;
}

// Constants and tables of prime set `as` (primes P ascending, primitive
// roots G, transforms up to 2^maxlog).  Set 0 keeps Montgomery pairs
// everywhere; set 1 takes Shoup pairs for the in-pass constants and tables.
cat_status init_prime_set(int as, const uint32_t* P, const uint32_t* G, int maxlog) {
  PrimeSet& S = g.set[as];
  memset(&S.roots, 0, sizeof(S.roots));
  for (int i = 0; i < CAT_NPRIMES; i++) {
    PrimeC& pc = S.prc[i];
    memset(&pc, 0, sizeof(pc));
    pc.p = P[i];
    pc.pinv = h_inv32(P[i]);
    const uint32_t p = pc.p;
    const uint32_t wmax = h_powmod(G[i], (uint64_t)(p - 1) >> maxlog, p);
    // a primitive 2^maxlog-th root: its 2^(maxlog-1)-th power is -1
    if (h_powmod(wmax, 1ull << (maxlog - 1), p) != p - 1) return CAT_EINTERNAL;
    const uint32_t iwmax = h_inv(wmax, p);
    for (int s = 0; s <= maxlog; s++) {
      const uint64_t ex = 1ull << (maxlog - s);
      S.roots.r[i][s] = h_mont(h_powmod(wmax, ex, p), p);
      S.roots.ir[i][s] = h_mont(h_powmod(iwmax, ex, p), p);
    }
    S.roots.one[i] = h_mont(1, p);
    const uint32_t w16 = h_powmod(wmax, 1ull << (maxlog - 4), p);
    const uint32_t iw16 = h_inv(w16, p);
    for (int k = 0; k < 8; k++) {
      if (as == 0) {
        h_pair(h_powmod(w16, k, p), pc, &pc.w16[k], &pc.w16q[k]);
        h_pair(h_powmod(iw16, k, p), pc, &pc.iw16[k], &pc.iw16q[k]);
      } else {
        pc.w16[k] = h_powmod(w16, k, p);
        pc.w16q[k] = (uint32_t)(((uint64_t)pc.w16[k] << 32) / p);
        pc.iw16[k] = h_powmod(iw16, k, p);
        pc.iw16q[k] = (uint32_t)(((uint64_t)pc.iw16[k] << 32) / p);
      }
    }
  }
  {
    CrtC& c = S.crt;
    const uint32_t p0 = P[0], p1 = P[1], p2 = P[2];
    h_pair(h_inv(p0 % p1, p1), S.prc[1], &c.c01, &c.c01q);
    h_pair(h_inv(p1 % p2, p2), S.prc[2], &c.c12, &c.c12q);
    const uint32_t p01m2 = h_mulmod(p0 % p2, p1 % p2, p2);
    h_pair(h_inv(p01m2, p2), S.prc[2], &c.c012, &c.c012q);
    c.p0 = p0;
    c.p1 = p1;
  }
  if (as == 0) {
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_primes), S.prc, sizeof(S.prc)));
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_crt), &S.crt, sizeof(S.crt)));
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_roots), &S.roots, sizeof(S.roots)));
  } else {
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_primes1), S.prc, sizeof(S.prc)));
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_crt1), &S.crt, sizeof(S.crt)));
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_roots1), &S.roots, sizeof(S.roots)));
  }
  HIPCHK(hipMalloc(&S.tws, sizeof(uint2) * TWS_ENTRIES * CAT_NPRIMES));
  HIPCHK(hipMalloc(&S.itws, sizeof(uint2) * TWS_ENTRIES * CAT_NPRIMES));
  HIPCHK(hipMalloc(&S.tw2lo, sizeof(uint2) * TW2_LO * CAT_NPRIMES));
  HIPCHK(hipMalloc(&S.itw2lo, sizeof(uint2) * TW2_LO * CAT_NPRIMES));
  HIPCHK(hipMalloc(&S.tw2hi, sizeof(uint32_t) * TW2_HI * CAT_NPRIMES));
  HIPCHK(hipMalloc(&S.itw2hi, sizeof(uint32_t) * TW2_HI * CAT_NPRIMES));
  HIPCHK(hipMemset(S.tw2hi, 0, sizeof(uint32_t) * TW2_HI * CAT_NPRIMES));
  HIPCHK(hipMemset(S.itw2hi, 0, sizeof(uint32_t) * TW2_HI * CAT_NPRIMES));
  if (as == 0) {
    hipLaunchKernelGGL(k_build_tws<0>, dim3(32, CAT_NPRIMES), dim3(256), 0, 0, S.tws, S.itws);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_build_tw2<0>, dim3(64, CAT_NPRIMES), dim3(256), 0, 0, S.tw2lo, S.tw2hi, S.itw2lo, S.itw2hi);
  } else {
    hipLaunchKernelGGL(k_build_tws<1>, dim3(32, CAT_NPRIMES), dim3(256), 0, 0, S.tws, S.itws);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_build_tw2<1>, dim3(64, CAT_NPRIMES), dim3(256), 0, 0, S.tw2lo, S.tw2hi, S.itw2lo, S.itw2hi);
  }
  LAUNCHCHK();
  return CAT_OK;
}

cat_status init_locked(int device) {
  if (g.inited) return CAT_OK;
  if (device < 0) HIPCHK(hipGetDevice(&device));
  g.device = device;
  HIPCHK(hipSetDevice(device));
  STCHK(init_prime_set(0, kP, kGen, CAT_MAX_LOGN));
  STCHK(init_prime_set(1, kQ, kQGen, CAT_LAZY_MAX_LOGN));
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipHostMalloc(&g.pin, 1 << 16, hipHostMallocDefault));
  // the device's own copy of the static scratch (the device is current here)
  HIPCHK(hipGetSymbolAddress(&g.scratch_ptr, HIP_SYMBOL(scratch)));
  if (!g.scratch_ptr) return CAT_EDEVICE;
  HIPCHK(hipStreamCreateWithFlags(&g.cap_stream, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&g.side_stream, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&g.ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&g.ev_join, hipEventDisableTiming));
  g.inited = true;
  return CAT_OK;
}

NttTables tables_for(int as) {
  const PrimeSet& S = g.set[as];
  NttTables tb;
  tb.tws = S.tws;
  tb.itws = S.itws;
  tb.tw2lo = S.tw2lo;
  tb.tw2hi = S.tw2hi;
  tb.itw2lo = S.itw2lo;
  tb.itw2hi = S.itw2hi;
  return tb;
}

// Pass decomposition of a large transform: N = L_0 ... L_{P-1} * M with
// every L_p <= 2^maxL (maxL <= 10, so a tile of L_p x C words with C >= 4
// fits 32 KB) and rows of M = 2^logM.
struct PassPlan {
  int P = 0;
  int logL[8] = {}, logS[8] = {}, logC[8] = {};
};
PassPlan pass_plan(int logN, int logM, int maxL, int logT = NTT_COL_LOGT) {
  PassPlan pp;
  const int rest = logN - logM;
  pp.P = (rest + maxL - 1) / maxL;
  int ls = logN;
  for (int k = 0; k < pp.P; k++) {
    pp.logL[k] = rest / pp.P + (k < rest % pp.P ? 1 : 0);
    pp.logS[k] = ls;
    pp.logC[k] = std::min(logT - pp.logL[k], ls - pp.logL[k]);   // tile L x C <= 2^logT words
    ls -= pp.logL[k];
  }
  return pp;
}

// scale constant 2^32 * N^-1 (Montgomery pair): the pointwise product
// mont_mul(x, y) = x*y/2^32 times it gives x*y/N, undoing the unscaled inverse.
uint2 scale_pair(int prime, int logN, int as = 0) {
  const PrimeC& pc = g.set[as].prc[prime];
  const uint32_t p = pc.p;
  const uint32_t ninv = h_inv(h_powmod(2, logN, p), p);
  const uint32_t W = h_mulmod(ninv, (uint32_t)((1ull << 32) % p), p);
  return h_pair2(W, pc);
}

// ----------------------------------------------------------------------------
// Stages: one batch of products of one class.
// ----------------------------------------------------------------------------
// CLS_COLSUM: a long operand times a short one by exact column sums (only
// chosen by the planner of the outer products, never by the tuning table).
enum { CLS_SCHOOL = 0, CLS_LDS = 1, CLS_LARGE = 2, CLS_COLSUM = 3, CLS_FUSED = 4 };

// Schedule per transform-length bucket 2^k (set by the autotuner, or defaults).
cat_tuning default_tuning() {
  cat_tuning t;
  memset(&t, 0, sizeof(t));
  t.school_max = SCHOOL_MAX;
  for (int k = 0; k <= CAT_MAX_LOGN; k++) {
    t.cls[k] = (k <= CAT_LDS_LOGT) ? CLS_LDS : CLS_LARGE;
    t.log_row[k] = CAT_LDS_LOGT;
    t.log_pass[k] = 10;
  }
  return t;
}
cat_tuning g_tune = default_tuning();
// polls of a predecessor's carry pair; CAT_POLLS_AUTO chooses per launch:
// launches of at most CRT_RECOMPUTE_BLOCKS blocks (one or a few rounds of
// workgroups, latency-bound) recompute the pair at once, which measured 4-5 %
// faster for k_crt at 10^7 and 10^8; larger ones poll (recomputing costs HBM
// bandwidth there: 3 % slower at 2,050,572,903)
uint32_t g_crt_polls = CAT_POLLS_AUTO;
#define CRT_RECOMPUTE_BLOCKS (1u << 15)
inline uint32_t crt_polls(uint32_t nblk) {
  if (g_crt_polls != CAT_POLLS_AUTO) return g_crt_polls;
  return nblk <= CRT_RECOMPUTE_BLOCKS ? 0u : CAT_SCAN_POLLS;
}

bool tuning_valid(const cat_tuning& t) {
  if (t.school_max < 1 || t.school_max > SCHOOL_MAX) return false;
  for (int k = 6; k <= CAT_MAX_LOGN; k++) {
    if (t.cls[k] == CLS_LDS) {
      // log_row: the tile of 2^log_row slots (12..14; at least the transform)
      if (k > CAT_LDS_MAX_LOGT || t.log_row[k] < CAT_LDS_LOGT || t.log_row[k] > CAT_LDS_MAX_LOGT) return false;
    } else if (t.cls[k] == CLS_LARGE) {
      if (t.log_row[k] < 8 || t.log_row[k] > CAT_LDS_MAX_LOGT || k <= t.log_row[k]) return false;
      if (t.log_pass[k] < 4 || t.log_pass[k] > 10) return false;
    } else {
      return false;
    }
  }
  return true;
}

struct Cls {
  int cls, logN, logM, maxL;
};

Cls classify2(uint64_t la, uint64_t lb) {
  Cls c{CLS_SCHOOL, 0, 0, 0};
  if (la <= g_tune.school_max && lb <= g_tune.school_max) return c;
  int k = ceil_log2(la + lb - 1);
  if (k < 6) k = 6;
  c.logN = k;
  if (k > CAT_MAX_LOGN) {   // beyond the transform length: the plan is rejected
    c.cls = CLS_LARGE;
    return c;
  }
  c.cls = g_tune.cls[k];
  c.logM = g_tune.log_row[k];
  c.maxL = g_tune.log_pass[k];
  return c;
}

void classify(uint64_t la, uint64_t lb, int* cls, int* logN) {
  const Cls c = classify2(la, lb);
  *cls = c.cls;
  *logN = c.logN;
}

struct Stage {
  int cls = CLS_SCHOOL;
  int logN = 0;
  int logM = CAT_LDS_LOGT;   // four-step row length
  int maxL = 10;             // four-step column-pass limit
  DescView dv{};           // dv.table is a device pointer (explicit) or nullptr (tree)
  std::vector<MulDesc> host_desc;   // explicit descriptors (host copy)
  uint64_t nmul = 0;
  uint64_t limbs = 0;      // sum of la+lb
  uint64_t a_base = 0, b_base = 0, c_base = 0;   // uint32 offsets from the workspace base
  // CRT (NTT classes)
  std::vector<CrtSeg> host_segs;
  std::vector<uint32_t> host_pref;
  SegView sv{};            // CRT segments (inline or device tables), set by upload_tables
  uint32_t nseg = 0, nblk = 0;
  // carried-up nodes
  CopyList tails{};
  uint64_t tail_in_base = 0, tail_out_base = 0;
  bool is_leaf = false;    // k_leaf<CAT_LEAF_LF>
  TreeLevel leaf{};
  uint64_t leaf_nodes = 0;
  bool dec = false;        // radix-10^9 products (k_crt10; addends in the segments)
  bool is_fused = false;   // k_tree_fused over the levels fused.j0 .. fused.j1
  FusedTree fused{};
  uint32_t fused_tiles = 0;
  double fused_bfly = 0;   // algorithmic butterflies of the fused levels
  int jfirst = 0;          // first tree level this stage computes (tree stages)
  // CLS_FUSED (generic batches): the one-workgroup buckets of up to 2^12
  // coefficients in one k_mul_fused launch over a tile table
  FusedMul fm{};
  std::vector<uint2> host_tiles;
};

// Tree levels fused into one launch: consecutive one-workgroup levels with
// transforms of up to 2^g_fuse_tree_logn coefficients (0: none, each level
// then is a transform launch plus a carry launch), for trees of at most
// FUSE_MAX_LEAVES leaves in the groups concerned.  A fused workgroup holds
// the tiles of all three primes (121 KB of LDS, one workgroup and 12 waves per
// CU) and pays a barrier per transform pass across them; the separate
// launches run four 4-wave workgroups per CU.  Off by default: since the
// one-workgroup transform runs its outermost and innermost passes on
// registers, the separate launches are as fast at n = 10^7 and faster at
// every other n measured (C(10^5): 0.28 vs 0.32 ms, C(3·10^7): 1.48 vs 1.60
// ms).  Generic batches fuse their one-workgroup buckets of up to
// 2^g_fuse_logn coefficients into one k_mul_fused launch.
uint32_t g_fuse_logn = FT_LOGT;
uint32_t g_fuse_tree_logn = 0;
#define FUSE_MAX_LEAVES (1ull << 22)

// Transforms of up to 2^g_lazy_logn points take the lazy prime set (0: none).
// Its three primes cover every coefficient of a product with
// min(la, lb) <= 2^22 limbs, which holds for N <= 2^23.
uint32_t g_lazy_logn = CAT_LAZY_MAX_LOGN;

// host mirror of DescView::get in tree mode
MulDesc tree_desc(const TreeLevel& t, uint64_t i) {
  uint32_t gi = 0;
  while (gi + 1 < t.ngroups && i >= t.mpref[gi + 1]) gi++;
  const uint64_t il = i - t.mpref[gi];
  const uint64_t sz = 1ull << t.j;
  MulDesc d;
  d.a_off = t.base[gi] + 2 * il * sz;
  d.b_off = d.a_off + sz;
  d.c_off = d.a_off;
  d.r_off = d.a_off;
  d.la = (uint32_t)sz;
  const uint64_t rem = t.K[gi] - (2 * il + 1) * sz;
  d.lb = (uint32_t)(rem < sz ? rem : sz);
  return d;
}

void build_crt_segs(Stage& s) {
  s.host_pref.clear();
  uint32_t b = 0;
  for (const CrtSeg& sg : s.host_segs) {
    s.host_pref.push_back(b);
    const uint64_t nb = (sg.len + CAT_CRT_BLOCK - 1) / CAT_CRT_BLOCK;
    b += (uint32_t)nb;
  }
  s.host_pref.push_back(b);
  s.nseg = (uint32_t)s.host_segs.size();
  s.nblk = b;
}

// ----------------------------------------------------------------------------
// Workspace layout for n (uint32 offsets unless noted)
// ----------------------------------------------------------------------------
struct Layout {
  uint64_t n = 0, s = 0, i0 = 0, i_end = 0, nseg = 0;
  int seg_log = SIEVE_SEG_LOG;   // odd numbers per sieve segment (log2)
  // factorial ratios: all primes with v_p(N) > 0 (capacity np_cap) before grouping
  uint64_t np_cap = 0, nchunks = 0;
  size_t P = 0, E = 0, chunk_cnt = 0, chunk_off = 0;      // in uint32 units
  size_t rcounts = 0;                                      // bytes
  uint64_t Kmax = 0, post_cap = 0, res_len = 0, F_words = 0, nblk_max = 0;
  uint64_t res2_len = 0, F2_words = 0, nblk2_max = 0;   // scratch of the side branch
  size_t primes = 0, arenaA = 0, arenaB = 0, post = 0, res = 0, F = 0;       // in uint32 units
  size_t res2 = 0, F2 = 0;                                                    // in uint32 units
  size_t seeds = 0, seed_e = 0, seg_cnt = 0, seg_off = 0, bitmap = 0;        // in uint32 units
  size_t gtab = 0, top = 0, err = 0, ctl_words = 0;                         // bytes (ctl_words: uint32)
  size_t total = 0;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Sieve segment size of the range of odd indices [i0, i_end): 2^16 odd
// numbers when that still gives 2^10 segments (four per CU), else 2^14.
int sieve_seg_log(uint64_t i0, uint64_t i_end) {
  if (i_end > i0 && i_end - i0 >= (1024ull << SIEVE_SEG_LOG_HUGE)) return SIEVE_SEG_LOG_HUGE;
  return (i_end > i0 && i_end - i0 >= (1024ull << SIEVE_SEG_LOG_BIG)) ? SIEVE_SEG_LOG_BIG : SIEVE_SEG_LOG;
}

// byte offsets inside the control block
#define CTL_TOP 1024
#define CTL_ERR 1032
#define CTL_READ 1040
#define CTL_FLAGS 1040
static_assert(sizeof(GroupTable) <= CTL_TOP, "group table must fit the control block head");

// Offsets of every buffer, given the sizes set in L (sieve range, Kmax,
// post_cap, res2_len, and np_cap / nchunks for ratios).
Layout layout_finish(Layout L) {
  const uint64_t seg = 1ull << L.seg_log;
  L.nseg = L.i_end > L.i0 ? (L.i_end - L.i0 + seg - 1) / seg : 0;
  // residues of one stage: by default bounded by everything the tree and the
  // post area can hold; callers with long power chains set a tighter bound
  if (L.res_len == 0) L.res_len = std::max(L.Kmax, L.post_cap) + 64;
  const uint64_t big = 1ull << ceil_log2(L.res_len);
  L.F_words = (big > (1ull << CAT_LDS_LOGT)) ? 12 * big + (1ull << 20) : (1ull << 20);
  L.nblk_max = L.res_len / CAT_CRT_BLOCK + 4096;
  L.F2_words = 12 * (1ull << ceil_log2(L.res2_len)) + (1ull << 16);
  L.nblk2_max = L.res2_len / CAT_CRT_BLOCK + 64;
  size_t off = 0;  // bytes
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  L.primes = take(L.Kmax * 4) / 4;
  L.arenaA = take(L.Kmax * 4) / 4;
  L.arenaB = take(L.Kmax * 4) / 4;
  L.post = take(L.post_cap * 4) / 4;
  L.res = take(3 * L.res_len * 4) / 4;
  L.F = take(L.F_words * 4) / 4;
  L.res2 = take(3 * L.res2_len * 4) / 4;
  L.F2 = take(L.F2_words * 4) / 4;
  L.seeds = take(SEED_MAX * 4) / 4;
  L.seed_e = take(SEED_MAX * 4) / 4;
  L.seg_cnt = take((L.nseg + 1) * 4) / 4;
  L.seg_off = take((L.nseg + 1) * 4) / 4;
  L.bitmap = take(L.nseg * (seg / 32) * 4) / 4;
  if (L.np_cap) {
    L.P = take(L.np_cap * 4) / 4;
    L.E = take(L.np_cap * 4) / 4;
    L.chunk_cnt = take(L.nchunks * 32 * 4) / 4;
    L.chunk_off = take(L.nchunks * 32 * 4) / 4;
    L.rcounts = take(sizeof(RatioCounts));
  }
  // control block, cleared by Phase 1 (k_seeds / k_rseeds): group table | top
  // | error word | CRT look-back flags of the main and the side branch; the
  // first CTL_READ bytes go back to the host in one copy
  L.gtab = take(CTL_FLAGS + 4 * (L.nblk_max + L.nblk2_max));
  L.top = L.gtab + CTL_TOP;
  L.err = L.gtab + CTL_ERR;
  L.ctl_words = (CTL_FLAGS + 4 * (L.nblk_max + L.nblk2_max)) / 4;
  L.total = off;
  return L;
}

Layout make_layout(uint64_t n) {
  Layout L;
  L.n = n;
  L.s = isqrt64(2 * n);
  L.i0 = (L.s + 1) / 2;
  L.i_end = n;
  L.Kmax = std::max<uint64_t>(pi_bound(2 * n), 16);
  const uint64_t sb = std::min<uint64_t>(pi_bound(L.s + 1), SEED_MAX);
  L.post_cap = L.Kmax + 256 * sb + 4096;
  // The powers P_e (e >= 2) and their product R involve only primes below
  // sqrt(2n), each prime power below 2^32: every step of them fits 64 limbs
  // per seed prime.
  L.res2_len = 64 * sb + 4096;
  L.seg_log = sieve_seg_log(L.i0, L.i_end);
  return layout_finish(L);
}

// ----------------------------------------------------------------------------
// The reconstruction plan for one n (depends only on the group counts).
// ----------------------------------------------------------------------------
struct Plan {
  uint64_t n = 0;
  uint32_t ng = 0;
  uint32_t exps[CAT_MAX_GROUPS] = {};
  uint64_t off[CAT_MAX_GROUPS + 1] = {};
  std::vector<Stage> batched;   // leaf kernel + levels
  std::vector<Stage> plain;     // levels from j = 0
  std::vector<Stage> post;      // powers, outer tree, final product (shared by both modes)
  uint64_t result_pos = 0, result_cap = 0;   // uint32 offset from workspace base
  bool result_is_one = false;
  // several requests in one plan (batched serving): group g belongs to
  // request req[g]; the powers, the outer product and the final product are
  // formed per request, with results rpos / rcap / rone (request 0 also in
  // the fields above)
  uint32_t nreq = 1;
  uint32_t req[CAT_MAX_GROUPS] = {};
  uint64_t rpos[CAT_MAX_GROUPS] = {}, rcap[CAT_MAX_GROUPS] = {};
  bool rone[CAT_MAX_GROUPS] = {};
  uint64_t post_end = 0;        // end of the post-tree arena used
  uint64_t root[CAT_MAX_GROUPS] = {};   // Q_e of group g (uint32 offset), the same in both forms
  uint64_t gbits[CAT_MAX_GROUPS] = {};  // bit-length bound of Q_e (group table)
  // Side branch (captured calls): after fork_count batched stages every group
  // with e >= 2 is complete, and post[0, post_final) (powers and R) may run
  // beside the remaining levels of Q_1; post[post_final..] (C = Q_1 R) waits
  // for both.  fork_count < 0: no side branch.
  int fork_count = -1;
  size_t post_final = 0;
  // R = prod_{e>=2} P_e as a node of Q_1's tree (rins_j >= 0): from level
  // rins_j on, group 0 (exponent 1) starts with one node of 2^rins_j limbs
  // that holds R (zero above its limbs), so the tree's top product is C
  // itself and no long-by-short product follows.  The other nodes of every
  // group sit 2^rins_j limbs further into the arenas than in the primes
  // buffer.  The powers and R run before stage rins_stage[form] (batched,
  // plain); R's product writes into that level's input arena.
  int rins_j = -1;
  int rins_stage[2] = {-1, -1};
  uint64_t rins_fill_pos = 0, rins_fill_len = 0;   // R's zero limbs above its product
  uint64_t r_limbs = 0, r_bits = 0;                // size of R's product output, bit bound of R
  void* dev = nullptr;          // device tables (segments, prefixes, descriptors)
  uint64_t products = 0, product_limbs = 0;
  uint32_t levels = 0;
  // graph caches: workspace base -> exec (Phase 2 only); (workspace, output,
  // capacity) -> exec of the whole call (Phase 1 + Phase 2 + copy)
  std::map<uintptr_t, hipGraphExec_t> graphs;
  std::map<std::vector<uintptr_t>, hipGraphExec_t> full_graphs;
  std::vector<uintptr_t> graphs_order;
  std::vector<std::vector<uintptr_t>> full_graphs_order;
};

// Graph caches keep at most PLAN_GRAPHS_MAX executables each (one per set of
// buffers a caller used); the oldest is destroyed once the device is idle.
#define PLAN_GRAPHS_MAX 8
template <class K>
void cache_graph(std::map<K, hipGraphExec_t>& m, std::vector<K>& order, const K& key, hipGraphExec_t ge) {
  m[key] = ge;
  order.push_back(key);
  while (order.size() > PLAN_GRAPHS_MAX) {
    (void)hipDeviceSynchronize();
    auto it = m.find(order.front());
    if (it != m.end()) {
      (void)hipGraphExecDestroy(it->second);
      m.erase(it);
    }
    order.erase(order.begin());
  }
}

// Shape of the forest of one plan: levels until one node per group (J),
// levels folded into the leaf kernel (0..jleaf-1) and the fused one-workgroup
// levels jf0..jf1 of the batched form (jf0 < 0: none).
struct TreeShape {
  int J = 0, jleaf = 0, jf0 = -1, jf1 = -2;
};
TreeShape tree_shape(const Plan& P) {
  TreeShape sh;
  uint64_t Kmax_g = 0, leaves = 0;
  for (uint32_t gi = 0; gi < P.ng; gi++) {
    Kmax_g = std::max(Kmax_g, P.off[gi + 1] - P.off[gi]);
    leaves += P.off[gi + 1] - P.off[gi];
  }
  const int LF = CAT_LEAF_LF;
  sh.J = ceil_log2(std::max<uint64_t>(Kmax_g, 1));
  sh.jleaf = Kmax_g > 1 ? std::min(sh.J, LF) : 0;
  // the consecutive levels above the leaf and schoolbook levels whose
  // products are one-workgroup transforms of at most 2^g_fuse_logn coefficients
  for (int j = std::max(sh.jleaf, 3); j < sh.J && j + 1 <= (int)g_fuse_tree_logn && leaves <= FUSE_MAX_LEAVES; j++) {
    if (classify2(1ull << j, 1ull << j).cls == CLS_LDS) {
      if (sh.jf0 < 0) sh.jf0 = j;
      sh.jf1 = j;
    } else if (sh.jf0 >= 0) {
      break;
    }
  }
  return sh;
}

// Forest levels of the product trees over the groups (one tree per group).
// out(j) = A for even j, B for odd j; in(0) = primes.  Node positions: group
// g's leaf k sits at off[g] + k in the primes buffer and at D + off[g] + k in
// the arenas, D = 2^rins_j when R is a node of Q_1's tree (else 0); from
// level rins_j on group 0 covers [off[0], off[0] + D + K_0): R's node first.
void plan_tree(const Layout& Ly, Plan& P, bool batched) {
  std::vector<Stage>& st = batched ? P.batched : P.plain;
  const uint32_t ng = P.ng;
  auto out_of = [&](int j) -> uint64_t { return (j % 2 == 0) ? Ly.arenaA : Ly.arenaB; };
  auto in_of = [&](int j) -> uint64_t { return j == 0 ? Ly.primes : out_of(j - 1); };
  const int jR = P.rins_j;
  const uint64_t D = jR >= 0 ? (1ull << jR) : 0;
  // first leaf and leaf count of group g at level j (input side)
  auto gpos = [&](uint32_t gi, int j) -> uint64_t {
    if (j == 0) return P.off[gi];
    if (jR >= 0 && gi == 0 && j >= jR) return P.off[0];   // R's node, then the shifted leaves
    return D + P.off[gi];
  };
  auto gK = [&](uint32_t gi, int j) -> uint64_t {
    const uint64_t K = P.off[gi + 1] - P.off[gi];
    return (jR >= 0 && gi == 0 && j >= jR) ? K + D : K;
  };
  const TreeShape sh = tree_shape(P);
  const int LF = CAT_LEAF_LF;
  const int jleaf = sh.jleaf, jf0 = sh.jf0, jf1 = sh.jf1;
  int J = sh.J;
  if (jR >= 0) J = std::max(J, ceil_log2(gK(0, jR)));
  // Q_e is complete after level jdone - 1 (at least the leaf levels), in
  // in_of(jdone); the plain form carries early roots up to the same place.
  // A root completed inside the fused levels is where the fused launch
  // leaves it, in in_of(jf1 + 1), in both forms.
  int jdone[CAT_MAX_GROUPS];
  for (uint32_t gi = 0; gi < ng; gi++) {
    jdone[gi] = std::max(ceil_log2(gK(gi, jR >= 0 ? J : 0)), jleaf);
    if (jf0 >= 0 && jdone[gi] > jf0 && jdone[gi] <= jf1 + 1) jdone[gi] = jf1 + 1;
    P.root[gi] = in_of(jdone[gi]) + gpos(gi, jdone[gi]);
  }
  P.rins_stage[batched ? 0 : 1] = -1;
  int jstart = 0;
  if (batched && sh.J > 0) {
    // leaf packing covers levels 0..LF-1 (reads the primes, writes the arena)
    Stage s;
    s.is_leaf = true;
    s.leaf.ngroups = ng;
    s.leaf.j = LF;
    uint64_t nodes = 0;
    for (uint32_t gi = 0; gi < ng; gi++) {
      s.leaf.base[gi] = P.off[gi];
      s.leaf.K[gi] = P.off[gi + 1] - P.off[gi];
      s.leaf.mpref[gi] = nodes;
      nodes += (s.leaf.K[gi] + (1ull << LF) - 1) >> LF;
    }
    s.leaf.mpref[ng] = nodes;
    s.leaf_nodes = nodes;
    s.a_base = Ly.primes;
    // the buffer the pairwise levels would have written last
    s.c_base = out_of(jleaf - 1) + D;
    for (uint32_t gi = 0; gi < ng; gi++) {
      const uint64_t K = P.off[gi + 1] - P.off[gi];
      // products inside the packed levels: K - nodes
      P.products += K - ((K + (1ull << LF) - 1) >> LF);
    }
    st.push_back(s);
    jstart = jleaf;
  }
  int j = jstart;
  for (; j < J; j++) {
    if (jR >= 0 && j == jR) P.rins_stage[batched ? 0 : 1] = (int)st.size();
    if (batched && j == jf0) {
      // the fused levels: one workgroup per 2^FT_LOGT leaves of every group
      // that still has products there (below rins_j: positions D + off)
      Stage s;
      s.is_fused = true;
      s.jfirst = jf0;
      FusedTree& f = s.fused;
      f.j0 = (uint32_t)jf0;
      f.j1 = (uint32_t)jf1;
      uint32_t tiles = 0;
      for (uint32_t gi = 0; gi < ng; gi++) {
        if (jdone[gi] <= jf0) continue;
        const uint64_t K = gK(gi, jf0);
        f.base[f.ngroups] = gpos(gi, jf0);
        f.K[f.ngroups] = K;
        f.tpref[f.ngroups] = tiles;
        tiles += (uint32_t)((K + FT_SLOTS - 1) / FT_SLOTS);
        f.ngroups++;
      }
      f.tpref[f.ngroups] = tiles;
      s.fused_tiles = tiles;
      for (int jj = jf0; jj <= jf1; jj++) {
        for (int q = 0; q < CAT_NPRIMES; q++) f.scale[jj - jf0][q] = scale_pair(q, jj + 1);
        s.fused_bfly += bfly(9.0 * tiles * (FT_SLOTS >> (jj + 1)), jj + 1);
      }
      s.a_base = in_of(jf0);
      s.c_base = out_of(jf1);
      st.push_back(s);
      j = jf1;
      continue;
    }
    // a stage reading the primes (level 0) writes its nodes D further on
    const uint64_t dout = j == 0 ? D : 0;
    Stage s;
    s.jfirst = j;
    s.dv.table = nullptr;
    TreeLevel& t = s.dv.tree;
    t.ngroups = ng;
    t.j = (uint32_t)j;
    uint64_t m = 0;
    s.tails.n = 0;
    for (uint32_t gi = 0; gi < ng; gi++) {
      const uint64_t K = gK(gi, j), b = gpos(gi, j);
      const uint64_t nodes = (K + (1ull << j) - 1) >> j;
      t.base[gi] = b;
      t.K[gi] = K;
      t.mpref[gi] = m;
      m += nodes / 2;
      // the odd last node moves up; a finished root moves until jdone
      if ((nodes & 1) && (nodes > 1 || j < jdone[gi])) {
        const uint64_t o = b + (nodes - 1) * (1ull << j);
        s.tails.off[s.tails.n] = o;
        s.tails.len[s.tails.n] = b + K - o;
        s.tails.n++;
      }
      // CRT segment: this group's products, contiguous from its base
      const uint64_t seglen = std::min<uint64_t>(K, (nodes / 2) * (2ull << j));
      if (nodes / 2 > 0) s.host_segs.push_back(CrtSeg{b, b, seglen});
    }
    t.mpref[ng] = m;
    s.nmul = m;
    s.limbs = 0;
    for (const CrtSeg& sg : s.host_segs) s.limbs += sg.len;
    {
      const Cls c = classify2(1ull << j, 1ull << j);
      s.cls = c.cls;
      s.logN = c.logN;
      s.logM = c.logM;
      s.maxL = c.maxL;
    }
    s.a_base = s.b_base = in_of(j);
    s.c_base = out_of(j) + dout;
    s.tail_in_base = in_of(j);
    s.tail_out_base = out_of(j) + dout;
    build_crt_segs(s);
    P.products += m;
    P.product_limbs += s.limbs;
    st.push_back(s);
  }
  P.levels = (uint32_t)j;
  if (batched) {
    // stages after which every group with e >= 2 is complete: those that
    // begin at a level below jdone (the leaf stage begins at level 0)
    int jf = -1;
    for (uint32_t gi = 0; gi < ng; gi++)
      if (P.exps[gi] >= 2) jf = std::max(jf, jdone[gi]);
    if (jf < 0) {
      P.fork_count = -1;
    } else {
      int fc = 0;
      for (const Stage& s : st)
        if ((s.is_leaf ? 0 : s.jfirst) <= jf - 1) fc++;
      P.fork_count = fc;
    }
  }
}

// Explicit products after the forest: P_e = Q_e^e (left-to-right binary
// powering), R = prod_{e>=2} P_e (balanced, adjacent pairs), C = Q_1 * R.
struct Item {
  uint64_t pos, cap;   // absolute uint32 offset from the workspace base, limbs read as the operand
  uint64_t bits;       // upper bound on the bit length of the value
};
// the limbs an operand of `bits` bits needs, within the `alloc` limbs written
inline uint64_t cap_of(uint64_t alloc, uint64_t bits) {
  return std::max<uint64_t>(1, std::min<uint64_t>(alloc, (bits + 31) / 32));
}

// A long times a short operand (la >= 8 lb) beyond the schoolbook bound:
// column sums cost la lb 32x32 multiply-adds (two VALU instructions each,
// about 2.5 with the window's shifts and LDS reads) in one pass; the transform
// costs 9 (N/2) log2 N butterflies (about 14 each).  Against the four-step
// path (four launches per product) the column sums are chosen up to 1.25
// times the transform's instruction count: on a batch of 4,096 uneven
// products the time is 4.64, 4.54, 4.55 and 4.56 ms at 0.75, 1.25, 1.9 and
// 2.9; C(10^7) and C(10^8) are flat over that range.  Against the
// one-workgroup transform (one launch, no HBM round trip) they are chosen up
// to its instruction count (the same batch: 4.58, 4.53, 4.48 and 4.46 ms at
// 0, 0.25, 0.5 and 1; in C(10^7) the short products of the side branch,
// about 150 x 6 limbs, leave the transform: 0.325 -> 0.266 ms of k_ntt_lds
// per call, hidden before beside the Q_1 tree).
bool colsum_wins(uint64_t la, uint64_t lb, const Cls& c) {
  if (c.cls == CLS_SCHOOL || c.cls == CLS_COLSUM || lb > COLSUM_MAX_LB || la < 8 * lb) return false;
  const double cs = 2.5 * (double)la * (double)lb;
  const double ntt = 14.0 * 9.0 * 0.5 * (double)(1ull << c.logN) * c.logN;
  return cs <= (c.cls == CLS_LARGE ? 1.25 : 1.0) * ntt;
}

void add_products(Plan& P, std::vector<std::pair<Item, Item>>& pairs, std::vector<Item>& outs) {
  // group the products of one step by class; positions already assigned
  std::map<std::pair<int, int>, Stage> by;
  uint64_t rpos = 0;
  for (size_t k = 0; k < pairs.size(); k++) {
    Item a = pairs[k].first, b = pairs[k].second;
    const Item c = outs[k];
    Cls cc = classify2(a.cap, b.cap);
    if (a.cap < b.cap) std::swap(a, b);   // a: the longer operand
    if (colsum_wins(a.cap, b.cap, cc)) cc = Cls{CLS_COLSUM, 0, 0, 0};
    Stage& s = by[{cc.cls, cc.logN}];
    s.cls = cc.cls;
    s.logN = cc.logN;
    s.logM = cc.logM;
    s.maxL = cc.maxL;
    MulDesc d;
    d.a_off = a.pos;
    d.b_off = b.pos;
    d.c_off = c.pos;
    d.r_off = rpos;
    d.la = (uint32_t)a.cap;
    d.lb = (uint32_t)b.cap;
    rpos += a.cap + b.cap;
    s.host_desc.push_back(d);
    s.host_segs.push_back(CrtSeg{c.pos, d.r_off, a.cap + b.cap});
    s.limbs += a.cap + b.cap;
  }
  for (auto& kv : by) {
    Stage& s = kv.second;
    // split into stages of at most CAT_INLINE_DESC products (kernel-argument tables)
    for (size_t k0 = 0; k0 < s.host_desc.size(); k0 += CAT_INLINE_DESC) {
      Stage t;
      t.cls = s.cls;
      t.logN = s.logN;
      t.logM = s.logM;
      t.maxL = s.maxL;
      const size_t k1 = std::min(s.host_desc.size(), k0 + CAT_INLINE_DESC);
      uint64_t r = 0;
      for (size_t k = k0; k < k1; k++) {
        MulDesc d = s.host_desc[k];
        d.r_off = r;
        r += (uint64_t)d.la + d.lb;
        t.host_desc.push_back(d);
        t.host_segs.push_back(CrtSeg{d.c_off, d.r_off, (uint64_t)d.la + d.lb});
        t.limbs += (uint64_t)d.la + d.lb;
      }
      t.nmul = t.host_desc.size();
      t.a_base = t.b_base = t.c_base = 0;
      build_crt_segs(t);
      P.products += t.nmul;
      P.product_limbs += t.limbs;
      P.post.push_back(t);
    }
  }
}

void plan_post(const Layout& Ly, Plan& P) {
  uint64_t bump = Ly.post;
  // a product's output: la + lb limbs written, read back as cap_of(...) limbs
  auto alloc = [&](uint64_t limbs, uint64_t bits) {
    Item it{bump, cap_of(limbs, bits), bits};
    bump += limbs;
    return it;
  };
  const uint32_t nr = std::max<uint32_t>(P.nreq, 1);
  std::vector<std::vector<Item>> pe(nr);   // P_e for e >= 2 of each request, exponent ascending
  std::vector<Item> q1(nr, Item{0, 0, 0});
  std::vector<bool> has_q1(nr, false);
  // powers: all chains advance one step per stage
  struct Chain {
    Item q, r;
    uint32_t e;
    int bit;
    bool sq_done;
    uint32_t req;
  };
  std::vector<Chain> ch;
  for (uint32_t gi = 0; gi < P.ng; gi++) {
    // Q_e occupies K limbs of its node; its value fits ceil(gbits / 32) of them
    const uint64_t K = P.off[gi + 1] - P.off[gi];
    Item q{P.root[gi], cap_of(K, P.gbits[gi]), std::min<uint64_t>(P.gbits[gi], 32 * K)};
    const uint32_t r = P.nreq > 1 ? P.req[gi] : 0;
    if (P.exps[gi] == 1) {
      q1[r] = q;
      has_q1[r] = true;
      continue;
    }
    int top = 31;
    while (!((P.exps[gi] >> top) & 1)) top--;
    ch.push_back(Chain{q, q, P.exps[gi], top - 1, false, r});
  }
  for (;;) {
    std::vector<std::pair<Item, Item>> pairs;
    std::vector<Item> outs;
    std::vector<size_t> who;
    for (size_t k = 0; k < ch.size(); k++) {
      Chain& c = ch[k];
      if (c.bit < 0) continue;
      if (!c.sq_done) {
        pairs.push_back({c.r, c.r});
        outs.push_back(alloc(2 * c.r.cap, 2 * c.r.bits));
      } else {
        pairs.push_back({c.r, c.q});
        outs.push_back(alloc(c.r.cap + c.q.cap, c.r.bits + c.q.bits));
      }
      who.push_back(k);
    }
    if (pairs.empty()) break;
    add_products(P, pairs, outs);
    for (size_t t = 0; t < who.size(); t++) {
      Chain& c = ch[who[t]];
      c.r = outs[t];
      if (!c.sq_done) {
        if ((c.e >> c.bit) & 1) c.sq_done = true;
        else c.bit--;
      } else {
        c.sq_done = false;
        c.bit--;
      }
    }
  }
  for (auto& c : ch) pe[c.req].push_back(c.r);
  // outer product of the P_e, e >= 2, of each request; one round of pairs
  // of every request per step
  for (;;) {
    std::vector<std::pair<Item, Item>> pairs;
    std::vector<Item> outs;
    std::vector<std::vector<Item>> next(nr);
    for (uint32_t r = 0; r < nr; r++) {
      if (pe[r].size() <= 1) {
        next[r] = pe[r];
        continue;
      }
      for (size_t k = 0; k + 1 < pe[r].size(); k += 2) {
        pairs.push_back({pe[r][k], pe[r][k + 1]});
        outs.push_back(alloc(pe[r][k].cap + pe[r][k + 1].cap, pe[r][k].bits + pe[r][k + 1].bits));
        next[r].push_back(outs.back());
      }
      if (pe[r].size() & 1) next[r].push_back(pe[r].back());
    }
    if (pairs.empty()) break;
    add_products(P, pairs, outs);
    pe = next;
  }
  P.post_final = P.post.size();
  // the product that leaves R (one request): its output size, for the choice
  // of R as a node of Q_1's tree
  Stage* r_stage = nullptr;
  size_t r_k = 0;
  if (nr == 1 && has_q1[0] && !pe[0].empty()) {
    for (Stage& t : P.post)
      for (size_t k = 0; k < t.host_desc.size(); k++)
        if (t.host_desc[k].c_off == pe[0][0].pos) {
          r_stage = &t;
          r_k = k;
        }
    if (r_stage) {
      P.r_limbs = (uint64_t)r_stage->host_desc[r_k].la + r_stage->host_desc[r_k].lb;
      P.r_bits = pe[0][0].bits;
    }
  }
  if (P.rins_j >= 0) {
    // R's product writes its limbs to R's node (position 0 of the arena
    // that level rins_j reads, the limbs above them cleared by a fill), and
    // the root of group 0 is C itself
    const uint64_t npos = (((P.rins_j - 1) % 2 == 0) ? Ly.arenaA : Ly.arenaB) + P.off[0];
    MulDesc& d = r_stage->host_desc[r_k];
    const uint64_t old = d.c_off;
    d.c_off = npos;
    for (CrtSeg& sg : r_stage->host_segs)
      if (sg.out_pos == old) sg.out_pos = npos;
    P.rins_fill_pos = npos + P.r_limbs;
    P.rins_fill_len = (1ull << P.rins_j) - P.r_limbs;
    const uint64_t K0 = P.off[1] - P.off[0] + (1ull << P.rins_j);
    const uint64_t bits = P.gbits[0] + P.r_bits;
    P.rpos[0] = P.root[0];
    P.rcap[0] = cap_of(K0, bits);
    P.rone[0] = false;
    P.result_pos = P.rpos[0];
    P.result_cap = P.rcap[0];
    P.result_is_one = false;
    P.post_end = bump;
    return;
  }
  bool any_final = false;
  for (uint32_t r = 0; r < nr; r++) any_final = any_final || (has_q1[r] && !pe[r].empty());
  // nothing runs beside the Q_1 tree (one request only: batches run in line)
  if (!any_final || nr > 1) P.fork_count = -1;
  std::vector<std::pair<Item, Item>> pairs;
  std::vector<Item> outs;
  std::vector<uint32_t> who;
  for (uint32_t r = 0; r < nr; r++) {
    P.rone[r] = false;
    if (has_q1[r] && !pe[r].empty()) {
      pairs.push_back({q1[r], pe[r][0]});
      outs.push_back(alloc(q1[r].cap + pe[r][0].cap, q1[r].bits + pe[r][0].bits));
      who.push_back(r);
    } else if (has_q1[r]) {
      P.rpos[r] = q1[r].pos;
      P.rcap[r] = q1[r].cap;
    } else if (!pe[r].empty()) {
      P.rpos[r] = pe[r][0].pos;
      P.rcap[r] = pe[r][0].cap;
    } else {
      P.rone[r] = true;
    }
  }
  if (!pairs.empty()) add_products(P, pairs, outs);
  for (size_t t = 0; t < who.size(); t++) {
    P.rpos[who[t]] = outs[t].pos;
    P.rcap[who[t]] = outs[t].cap;
  }
  P.result_pos = P.rpos[0];
  P.result_cap = P.rcap[0];
  P.result_is_one = P.rone[0];
  P.post_end = bump;
}

// Descriptor and segment tables: carried inline in the kernel arguments when
// small (every catalan plan), otherwise uploaded to one device buffer (large
// generic batches).  *dev stays nullptr when nothing needs device memory.
cat_status upload_tables(std::vector<Stage*>& all, void** dev, bool device_tables = true,
                         std::vector<char>* keep = nullptr, hipStream_t st = nullptr) {
  size_t bytes = 0;
  for (Stage* s : all) {
    if (s->cls == CLS_FUSED) {
      bytes = align_up(bytes, 16) + s->host_desc.size() * sizeof(MulDesc);
      bytes = align_up(bytes, 16) + s->host_tiles.size() * sizeof(uint2);
      continue;
    }
    if (s->host_desc.size() > CAT_INLINE_DESC) bytes = align_up(bytes, 16) + s->host_desc.size() * sizeof(MulDesc);
    if (s->host_segs.size() > CAT_INLINE_SEG) {
      bytes = align_up(bytes, 16) + s->host_segs.size() * sizeof(CrtSeg);
      bytes = align_up(bytes, 16) + s->host_pref.size() * sizeof(uint32_t);
      bytes = align_up(bytes, 16) + (size_t)s->nblk * sizeof(uint32_t);
    }
  }
  // callers that must not allocate get CAT_EINTERNAL instead (C(n) plans
  // always fit the kernel arguments)
  if (bytes && !device_tables) return CAT_EINTERNAL;
  char* d = nullptr;
  std::vector<char> h(std::max<size_t>(bytes, 16), 0);
  if (bytes) HIPCHK(hipMalloc(&d, bytes));
  size_t o = 0;
  for (Stage* s : all) {
    if (s->cls == CLS_FUSED) {
      o = align_up(o, 16);
      memcpy(&h[o], s->host_desc.data(), s->host_desc.size() * sizeof(MulDesc));
      s->fm.desc = (const MulDesc*)(d + o);
      o += s->host_desc.size() * sizeof(MulDesc);
      o = align_up(o, 16);
      memcpy(&h[o], s->host_tiles.data(), s->host_tiles.size() * sizeof(uint2));
      s->fm.tiles = (const uint2*)(d + o);
      o += s->host_tiles.size() * sizeof(uint2);
      continue;
    }
    s->dv.ninl = 0;
    if (!s->host_desc.empty()) {
      if (s->host_desc.size() > CAT_INLINE_DESC) {
        o = align_up(o, 16);
        memcpy(&h[o], s->host_desc.data(), s->host_desc.size() * sizeof(MulDesc));
        s->dv.table = (const MulDesc*)(d + o);
        o += s->host_desc.size() * sizeof(MulDesc);
      } else {
        s->dv.table = nullptr;
        s->dv.ninl = (uint32_t)s->host_desc.size();
        for (size_t k = 0; k < s->host_desc.size(); k++) s->dv.inl[k] = s->host_desc[k];
      }
    }
    s->sv = SegView{};
    s->sv.nseg = (uint32_t)s->host_segs.size();
    if (s->host_segs.size() > CAT_INLINE_SEG) {
      o = align_up(o, 16);
      memcpy(&h[o], s->host_segs.data(), s->host_segs.size() * sizeof(CrtSeg));
      s->sv.segs = (const CrtSeg*)(d + o);
      o += s->host_segs.size() * sizeof(CrtSeg);
      o = align_up(o, 16);
      memcpy(&h[o], s->host_pref.data(), s->host_pref.size() * sizeof(uint32_t));
      s->sv.pref = (const uint32_t*)(d + o);
      o += s->host_pref.size() * sizeof(uint32_t);
      // block -> segment, so that a block of a large batch finds its product
      // with one load instead of a binary search over the prefix table
      o = align_up(o, 16);
      uint32_t* b2s = (uint32_t*)&h[o];
      for (size_t k = 0; k + 1 < s->host_pref.size(); k++)
        for (uint32_t b = s->host_pref[k]; b < s->host_pref[k + 1]; b++) b2s[b] = (uint32_t)k;
      s->sv.b2s = (const uint32_t*)(d + o);
      o += (size_t)s->nblk * sizeof(uint32_t);
    } else {
      for (size_t k = 0; k < s->host_segs.size(); k++) s->sv.iseg[k] = s->host_segs[k];
      for (size_t k = 0; k < s->host_pref.size(); k++) s->sv.ipref[k] = s->host_pref[k];
    }
  }
  if (bytes && keep) {
    // stream-ordered upload; the host image lives as long as the plan
    keep->swap(h);
    HIPCHK(hipMemcpyAsync(d, keep->data(), bytes, hipMemcpyHostToDevice, st));
  } else if (bytes) {
    HIPCHK(hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice));
  }
  *dev = d;
  return CAT_OK;
}

void free_plan(Plan* P) {
  for (auto& kv : P->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& kv : P->full_graphs) (void)hipGraphExecDestroy(kv.second);
  if (P->dev) (void)hipFree(P->dev);
  delete P;
}

// R = prod_{e>=2} P_e enters Q_1's tree as a node of level j (returned; -1:
// the final product Q_1 R stays).  j leaves two levels of Q_1 between the
// completion of the last group with e >= 2 and R's level, for the powers and
// R to run beside them; it lies above the leaf and fused levels and holds R's
// product.  Taken when R's node is at most a quarter of Q_1's tree and the
// arenas have room for the extra 2^j leaves.
bool g_rins = true;
int rins_level(const Layout& Ly, const Plan& P) {
  if (!g_rins || P.nreq != 1 || P.ng < 2 || P.exps[0] != 1 || P.r_limbs == 0) return -1;
  const TreeShape sh = tree_shape(P);
  int jdone2 = -1;
  for (uint32_t gi = 1; gi < P.ng; gi++) {
    int jd = std::max(ceil_log2(P.off[gi + 1] - P.off[gi]), sh.jleaf);
    if (sh.jf0 >= 0 && jd > sh.jf0 && jd <= sh.jf1 + 1) jd = sh.jf1 + 1;
    if (P.exps[gi] >= 2) jdone2 = std::max(jdone2, jd);
  }
  const int j = std::max({ceil_log2(P.r_limbs), jdone2 + 2, sh.jleaf + 1, sh.jf1 + 1});
  if (ceil_log2(P.off[1] - P.off[0]) < j + 2) return -1;
  if ((1ull << j) + P.off[P.ng] > Ly.Kmax) return -1;
  return j;
}

cat_status make_plan(const Layout& Ly, const GroupTable& gt, Plan** out, bool device_tables = true,
                     const uint32_t* req = nullptr, uint32_t nreq = 1) {
  Plan* P = new Plan();
  P->n = Ly.n;
  P->ng = gt.ngroups;
  P->nreq = req ? nreq : 1;
  if (req)
    for (uint32_t gi = 0; gi < gt.ngroups; gi++) P->req[gi] = req[gi];
  for (uint32_t gi = 0; gi < gt.ngroups; gi++) {
    P->exps[gi] = gt.exps[gi];
    P->gbits[gi] = gt.gbits[gi];
  }
  for (uint32_t gi = 0; gi <= gt.ngroups; gi++) P->off[gi] = gt.off[gi];
  auto plan_all = [&]() {
    P->batched.clear();
    P->plain.clear();
    P->post.clear();
    P->fork_count = -1;
    P->post_final = 0;
    plan_tree(Ly, *P, true);
    // products and their limbs are counted from the pairwise levels of the
    // plain form (the leaf kernel of the batched form folds the lowest levels)
    P->products = 0;
    P->product_limbs = 0;
    plan_tree(Ly, *P, false);
    plan_post(Ly, *P);
  };
  plan_all();
  const int jR = rins_level(Ly, *P);
  if (jR >= 0) {
    P->rins_j = jR;
    plan_all();
  }
  std::vector<Stage*> all;
  for (auto& s : P->batched) all.push_back(&s);
  for (auto& s : P->plain) all.push_back(&s);
  for (auto& s : P->post) all.push_back(&s);
  // the plan must fit the workspace layout sized from n alone
  for (Stage* s : all) {
    if (s->is_leaf) continue;
    if (s->logN > CAT_MAX_LOGN) {   // a product longer than the longest exact transform
      free_plan(P);
      return CAT_ERANGE;
    }
    uint64_t rmax = 0;
    for (const CrtSeg& sg : s->host_segs) rmax = std::max(rmax, sg.res_pos + sg.len);
    const uint64_t fneed = (s->cls == CLS_LARGE) ? s->nmul * 6ull << s->logN : 0;
    if (rmax > Ly.res_len || fneed > Ly.F_words || s->nblk > Ly.nblk_max) {
      free_plan(P);
      return CAT_EINTERNAL;
    }
  }
  // the side branch runs with its own scratch; without room there the powers
  // run in line
  for (size_t k = 0; k < P->post_final && P->fork_count >= 0; k++) {
    const Stage& s = P->post[k];
    uint64_t rmax = 0;
    for (const CrtSeg& sg : s.host_segs) rmax = std::max(rmax, sg.res_pos + sg.len);
    const uint64_t fneed = (s.cls == CLS_LARGE) ? s.nmul * 6ull << s.logN : 0;
    if (rmax > Ly.res2_len || fneed > Ly.F2_words || s.nblk > Ly.nblk2_max) P->fork_count = -1;
  }
  if (P->post_end > Ly.post + Ly.post_cap) {
    free_plan(P);
    return CAT_EINTERNAL;
  }
  cat_status st = upload_tables(all, &P->dev, device_tables);
  if (st != CAT_OK) {
    free_plan(P);
    return st;
  }
  *out = P;
  return CAT_OK;
}

// ----------------------------------------------------------------------------
// Execution
// ----------------------------------------------------------------------------
struct Exec {
  uint32_t* W = nullptr;   // workspace base
  const uint32_t* A = nullptr;   // caller operand / output bases (generic batches)
  const uint32_t* B = nullptr;
  uint32_t* C = nullptr;
  uint32_t* res = nullptr;
  uint64_t res_stride = 0;
  uint32_t* F = nullptr;
  uint32_t* flags = nullptr;   // CRT look-back flags (cleared when the call starts)
  uint32_t crt_epoch = 0;      // CRT launches so far in this call
  // side branch: stream (nullptr: everything runs in order on st) and its scratch
  hipStream_t side = nullptr;
  uint32_t* res2 = nullptr;
  uint64_t res2_stride = 0;
  uint32_t* F2 = nullptr;
  uint32_t* flags2 = nullptr;
  uint32_t* err = nullptr;
  hipStream_t st = nullptr;
  uint64_t launches = 0;
};

cat_status launch_crt(Exec& X, uint32_t* out, SegView sv, uint32_t nblk, const CopyList* tails = nullptr,
                      const uint32_t* tin = nullptr, uint32_t* tout = nullptr, bool raw = false, int as = 0) {
  static const CopyList none{};
  const CopyList& cl = tails ? *tails : none;
  const uint32_t grid = nblk + tail_blocks(cl);
  if (grid == 0) return CAT_OK;
  {
    KTime kt("k_crt", X.st, (double)nblk * CAT_CRT_BLOCK);
    X.crt_epoch++;
    if (raw)
      hipLaunchKernelGGL((k_crt<true, 0>), dim3(grid), dim3(CAT_CRT_THREADS), 0, X.st, sv, X.res, X.res_stride, out,
                         nblk, X.flags, X.crt_epoch, crt_polls(nblk), cl, tin, tout, X.err);
    else if (as == 0)
      hipLaunchKernelGGL((k_crt<false, 0>), dim3(grid), dim3(CAT_CRT_THREADS), 0, X.st, sv, X.res, X.res_stride, out,
                         nblk, X.flags, X.crt_epoch, crt_polls(nblk), cl, tin, tout, X.err);
    else
      hipLaunchKernelGGL((k_crt<false, 1>), dim3(grid), dim3(CAT_CRT_THREADS), 0, X.st, sv, X.res, X.res_stride, out,
                         nblk, X.flags, X.crt_epoch, crt_polls(nblk), cl, tin, tout, X.err);
  }
  LAUNCHCHK();
  X.launches++;
  return CAT_OK;
}

// Radix-10^9 CRT + carry + addend (addends are read relative to the workspace).
cat_status launch_crt10(Exec& X, uint32_t* out, const SegView& sv, uint32_t nblk, const CopyList* tails,
                        const uint32_t* tin, uint32_t* tout) {
  const uint32_t grid = nblk + tail_blocks(*tails);
  if (grid == 0) return CAT_OK;
  {
    KTime kt("k_crt10", X.st, (double)nblk * DEC_CRT_BLOCK);
    X.crt_epoch++;
    hipLaunchKernelGGL(k_crt10, dim3(grid), dim3(DEC_CRT_THREADS), 0, X.st, sv, X.res, X.res_stride, out, X.W, nblk,
                       X.flags, X.crt_epoch, crt_polls(nblk), *tails, tin, tout, X.err);
  }
  LAUNCHCHK();
  X.launches++;
  return CAT_OK;
}

// Products of a stage given by `dv` (cnt of them): the NTT or schoolbook part.
uint32_t* out_base(Exec& X, const Stage& s) { return X.C ? X.C : X.W + s.c_base; }

// prime set of a transform stage (radix-10^9 products keep the first set,
// whose CRT kernel carries in that radix)
int stage_as(const Stage& s) {
  if (s.dec || (s.cls != CLS_LDS && s.cls != CLS_LARGE)) return 0;
  return (uint32_t)s.logN <= g_lazy_logn ? 1 : 0;
}

cat_status launch_products(Exec& X, const Stage& s, DescView dv, uint64_t cnt, bool with_tails = false) {
  const uint32_t* ain = X.A ? X.A : X.W + s.a_base;
  const uint32_t* bin = X.B ? X.B : X.W + s.b_base;
  uint32_t* out = out_base(X, s);
  if (s.cls == CLS_SCHOOL) {
    static const CopyList none{};
    const CopyList& cl = with_tails ? s.tails : none;
    const uint64_t blocks = (cnt + SCHOOL_WAVES - 1) / SCHOOL_WAVES;
    {
      KTime kt("k_school", X.st, (double)s.limbs);
      hipLaunchKernelGGL(k_school, dim3((uint32_t)blocks + tail_blocks(cl)), dim3(64 * SCHOOL_WAVES), 0, X.st, dv,
                         cnt, ain, bin, out, X.err, (uint32_t)blocks, cl, X.W + s.tail_in_base,
                         X.W + s.tail_out_base);
    }
    LAUNCHCHK();
    X.launches++;
    return CAT_OK;
  }
  if (s.cls == CLS_COLSUM) {
    // every product of the stage in one launch, one workgroup per CRT block
    SegView sv = s.sv;
    uint32_t nblk = s.nblk;
    if (s.nmul != cnt) {
      // one product (plain mode): a single segment of its own
      if (cnt != 1 || dv.ninl != 1) return CAT_EINTERNAL;
      const MulDesc d = dv.inl[0];
      sv = SegView{};
      sv.nseg = 1;
      sv.iseg[0] = CrtSeg{d.c_off, d.r_off, (uint64_t)d.la + d.lb};
      nblk = (uint32_t)((sv.iseg[0].len + CAT_CRT_BLOCK - 1) / CAT_CRT_BLOCK);
      sv.ipref[0] = 0;
      sv.ipref[1] = nblk;
    }
    if (nblk == 0) return CAT_OK;
    KTime kt("k_colsum", X.st, (double)nblk * COLSUM_COLS);
    hipLaunchKernelGGL(k_colsum, dim3(nblk), dim3(COLSUM_T), 0, X.st, dv, sv, ain, bin, X.res, X.res_stride, X.err);
    LAUNCHCHK();
    X.launches++;
    return CAT_OK;
  }
  const int as = stage_as(s);
  const NttTables tb = tables_for(as);
  const uint2 s0 = scale_pair(0, s.logN, as), s1 = scale_pair(1, s.logN, as), s2 = scale_pair(2, s.logN, as);
  if (s.cls == CLS_LDS) {
    // tile 2^lt (2^lt / 16 threads, 2^(lt - logN) products per workgroup): the
    // schedule's tile for the bucket (log_row of a one-workgroup bucket)
    // (at most 64 products per tile: the kernel's descriptor array)
    const int lt = std::max(s.logN, std::min({std::max(s.logM, CAT_LDS_LOGT), CAT_LDS_MAX_LOGT, s.logN + 6}));
    const uint64_t per = (1ull << lt) >> s.logN;
    const uint64_t tiles = (cnt + per - 1) / per;
    const dim3 grid((uint32_t)(tiles * CAT_NPRIMES)), block((1u << lt) / 16);
    // a second operand common to all products (decimal joins): transformed
    // once per prime into the stage scratch, then reused, where the stage is
    // large enough for the saved transforms to outweigh the extra launch
    const bool constb = dv.uni && dv.u.sb == 0 && cnt > 1 && (cnt << s.logN) >= (1ull << 21);
    KTime kt("k_ntt_lds", X.st, constb ? bfly(6.0 * cnt + 3.0, s.logN) : bfly(9.0 * cnt, s.logN));
#define LDS_LAUNCH(LT, BM, G)                                                                                \
  do {                                                                                                         \
    if (as == 0)                                                                                               \
      hipLaunchKernelGGL((k_ntt_lds<LT, BM, 0>), G, block, 0, X.st, dv, cnt, s.logN, ain, bin, X.res,          \
                         X.res_stride, tb, s0, s1, s2, X.F);                                                   \
    else                                                                                                       \
      hipLaunchKernelGGL((k_ntt_lds<LT, BM, 1>), G, block, 0, X.st, dv, cnt, s.logN, ain, bin, X.res,          \
                         X.res_stride, tb, s0, s1, s2, X.F);                                                   \
  } while (0)
    if (constb) {
      if (lt == 12) LDS_LAUNCH(12, 1, dim3(CAT_NPRIMES));
      else if (lt == 13) LDS_LAUNCH(13, 1, dim3(CAT_NPRIMES));
      else LDS_LAUNCH(14, 1, dim3(CAT_NPRIMES));
      LAUNCHCHK();
      X.launches++;
      if (lt == 12) LDS_LAUNCH(12, 2, grid);
      else if (lt == 13) LDS_LAUNCH(13, 2, grid);
      else LDS_LAUNCH(14, 2, grid);
    } else {
      if (lt == 12) LDS_LAUNCH(12, 0, grid);
      else if (lt == 13) LDS_LAUNCH(13, 0, grid);
      else LDS_LAUNCH(14, 0, grid);
    }
#undef LDS_LAUNCH
    LAUNCHCHK();
    X.launches++;
    return CAT_OK;
  }
  // column tiles: the smaller size when the stage cannot fill the GPU
  const int logT = ((double)cnt * (double)(1ull << s.logN) < 4194304.0) ? NTT_COL_LOGT_SMALL : NTT_COL_LOGT;
  const PassPlan pp = pass_plan(s.logN, s.logM, s.maxL, logT);
  const int logM = s.logM, logR1 = s.logN - logM;
  const double N = (double)(1ull << s.logN);
  // The twiddles of pass k are applied by pass k itself (forward: at its
  // store; inverse: at its load), or, when the next pass's tiles have at most
  // 256 columns (a thread's positions then advance by a constant step), by
  // pass k + 1 (forward: at its load; inverse: at its store); those of the
  // last pass by k_row.
  bool defer[8] = {};
  for (int k = 0; k + 1 < pp.P; k++) defer[k] = pp.logC[k + 1] <= 8;
  auto self_tw = [&](int k) { return (k + 1 < pp.P && !defer[k]) ? 1 : 0; };
  auto pre_tw = [&](int k) { return (k >= 1 && defer[k - 1]) ? 1 : 0; };
  // A second operand that is the same for every product (the power P_j of a
  // decimal join) is transformed once: its column passes for product 0 only,
  // its row transforms once (k_row mode 1), reused by every product (mode 2).
  const bool constb = dv.uni && dv.u.sb == 0 && cnt > 1;
  auto pass_fwd = [&](const PassGeom& pg, int k, int plS, int plL, uint64_t gx, uint32_t nop, int op_base) {
    const dim3 grid((uint32_t)(gx * CAT_NPRIMES), 1, nop);
#define PASS_FWD(LT, A)                                                                                            \
  hipLaunchKernelGGL((k_pass_fwd<LT, A>), grid, dim3(NTT_COL_THREADS), 0, X.st, dv, pg, k == 0 ? 1 : 0, self_tw(k), \
                     pre_tw(k), plS, plL, op_base, ain, bin, X.F, tb)
    if (logT == NTT_COL_LOGT_SMALL) {
      if (as == 0) PASS_FWD(NTT_COL_LOGT_SMALL, 0);
      else PASS_FWD(NTT_COL_LOGT_SMALL, 1);
    } else {
      if (as == 0) PASS_FWD(NTT_COL_LOGT, 0);
      else PASS_FWD(NTT_COL_LOGT, 1);
    }
#undef PASS_FWD
  };
  for (int k = 0; k < pp.P; k++) {
    PassGeom pg{s.logN, pp.logS[k], pp.logL[k], pp.logC[k]};
    const int plS = k >= 1 ? pp.logS[k - 1] : 0, plL = k >= 1 ? pp.logL[k - 1] : 0;
    const uint64_t gx1 = 1ull << (s.logN - pp.logL[k] - pp.logC[k]);   // tiles of one product
    const uint64_t gx = cnt * gx1;
    // L-point DFTs of both operands, 3 primes: (N/2) log2 L butterflies each
    KTime kt("k_pass_fwd", X.st, (constb ? 3.0 * (cnt + 1) : 6.0 * cnt) * N / 2 * pp.logL[k]);
    if (constb) {
      pass_fwd(pg, k, plS, plL, gx, 1, 0);
      LAUNCHCHK();
      pass_fwd(pg, k, plS, plL, gx1, 1, 1);
    } else {
      pass_fwd(pg, k, plS, plL, gx, 2, 0);
    }
    LAUNCHCHK();
    if (constb) X.launches++;
  }
  {
    // row DFTs: two forward and one inverse per row, 3 primes
    const double rows = (double)cnt * (1ull << logR1);
    // rows of 2^11 run in their own tile (full rows, 128 threads); shorter
    // rows share the 2^12 tile
    const int lt = logM == 11 ? 11 : std::max(logM, CAT_LDS_LOGT);
    const dim3 block((1u << lt) / 16);
    auto row = [&](uint64_t nprod, int bmode) {
      const dim3 grid((uint32_t)(nprod << logR1), CAT_NPRIMES);
#define ROW(LT, A)                                                                                              \
  hipLaunchKernelGGL((k_row<LT, A>), grid, block, 0, X.st, s.logN, logM, pp.logS[pp.P - 1], pp.logL[pp.P - 1], \
                     bmode, X.F, tb, s0, s1, s2)
      if (lt == 11) {
        if (as == 0) ROW(11, 0);
        else ROW(11, 1);
      } else if (lt == 12) {
        if (as == 0) ROW(12, 0);
        else ROW(12, 1);
      } else if (lt == 13) {
        if (as == 0) ROW(13, 0);
        else ROW(13, 1);
      } else {
        if (as == 0) ROW(14, 0);
        else ROW(14, 1);
      }
#undef ROW
    };
    KTime kt("k_row", X.st, constb ? bfly(6.0 * rows + 3.0 * (1ull << logR1), logM) : bfly(9.0 * rows, logM));
    if (constb) {
      row(1, 1);
      LAUNCHCHK();
      X.launches++;
      row(cnt, 2);
    } else {
      row(cnt, 0);
    }
  }
  LAUNCHCHK();
  for (int k = pp.P - 1; k >= 0; k--) {
    PassGeom pg{s.logN, pp.logS[k], pp.logL[k], pp.logC[k]};
    const int plS = k >= 1 ? pp.logS[k - 1] : 0, plL = k >= 1 ? pp.logL[k - 1] : 0;
    const uint64_t gx = cnt << (s.logN - pp.logL[k] - pp.logC[k]);
    KTime kt("k_pass_inv", X.st, 3.0 * cnt * N / 2 * pp.logL[k]);
#define PASS_INV(LT, A)                                                                                         \
  hipLaunchKernelGGL((k_pass_inv<LT, A>), dim3((uint32_t)gx, CAT_NPRIMES), dim3(NTT_COL_THREADS), 0, X.st, dv, pg, \
                     k == 0 ? 1 : 0, self_tw(k), pre_tw(k), plS, plL, X.F, X.res, X.res_stride, tb)
    if (logT == NTT_COL_LOGT_SMALL) {
      if (as == 0) PASS_INV(NTT_COL_LOGT_SMALL, 0);
      else PASS_INV(NTT_COL_LOGT_SMALL, 1);
    } else {
      if (as == 0) PASS_INV(NTT_COL_LOGT, 0);
      else PASS_INV(NTT_COL_LOGT, 1);
    }
#undef PASS_INV
    LAUNCHCHK();
  }
  X.launches += 2 * pp.P + 1;
  return CAT_OK;
}

cat_status copy_tails(Exec& X, const Stage& s) {
  if (s.tails.n == 0) return CAT_OK;
  uint64_t mx = 0;
  for (uint32_t k = 0; k < s.tails.n; k++) mx = std::max(mx, s.tails.len[k]);
  const uint32_t blocks = (uint32_t)std::min<uint64_t>((mx + 255) / 256, 1024);
  hipLaunchKernelGGL(k_copy_ranges, dim3(blocks, s.tails.n), dim3(256), 0, X.st, s.tails, X.W + s.tail_in_base,
                     X.W + s.tail_out_base);
  LAUNCHCHK();
  X.launches++;
  return CAT_OK;
}

SegView stage_segs(const Stage& s) { return s.sv; }

cat_status run_stage_batched(Exec& X, const Stage& s) {
  if (s.cls == CLS_FUSED) {
    if (s.host_tiles.empty()) return CAT_OK;
    {
      KTime kt("k_mul_fused", X.st, s.fused_bfly);
      hipLaunchKernelGGL(k_mul_fused, dim3((uint32_t)s.host_tiles.size()), dim3(FT_THREADS), 0, X.st, s.fm,
                         X.A ? X.A : X.W + s.a_base, X.B ? X.B : X.W + s.b_base, out_base(X, s), tables_for(0),
                         X.err);
    }
    LAUNCHCHK();
    X.launches++;
    return CAT_OK;
  }
  if (s.is_fused) {
    if (s.fused_tiles == 0) return CAT_OK;
    {
      KTime kt("k_tree_fused", X.st, s.fused_bfly);
      hipLaunchKernelGGL(k_tree_fused, dim3(s.fused_tiles), dim3(FT_THREADS), 0, X.st, s.fused, X.W + s.a_base,
                         X.W + s.c_base, tables_for(0), X.err);
    }
    LAUNCHCHK();
    X.launches++;
    return CAT_OK;
  }
  if (s.is_leaf) {
    const uint32_t blocks = (uint32_t)((s.leaf_nodes + 255) / 256);
    {
      KTime kt("k_leaf", X.st, (double)s.leaf_nodes);
      hipLaunchKernelGGL(k_leaf<CAT_LEAF_LF>, dim3(blocks), dim3(256), 0, X.st, s.leaf, s.leaf_nodes, X.W + s.a_base,
                         X.W + s.c_base);
    }
    LAUNCHCHK();
    X.launches++;
    return CAT_OK;
  }
  if (s.nmul > 0 && s.dec) {
    if (s.cls == CLS_SCHOOL) return CAT_EINTERNAL;
    STCHK(launch_products(X, s, s.dv, s.nmul));
    return launch_crt10(X, out_base(X, s), s.sv, s.nblk, &s.tails, X.W + s.tail_in_base, X.W + s.tail_out_base);
  }
  if (s.nmul > 0) {
    // the tail copies ride along with the last kernel of the level
    STCHK(launch_products(X, s, s.dv, s.nmul, s.cls == CLS_SCHOOL));
    if (s.cls != CLS_SCHOOL)
      STCHK(launch_crt(X, out_base(X, s), stage_segs(s), s.nblk, &s.tails, X.W + s.tail_in_base,
                       X.W + s.tail_out_base, s.cls == CLS_COLSUM, stage_as(s)));
    return CAT_OK;
  }
  return copy_tails(X, s);
}

// One product per launch (per kernel stage of that product).
cat_status run_stage_plain(Exec& X, const Stage& s) {
  if (s.is_leaf) return CAT_EINTERNAL;
  for (uint64_t i = 0; i < s.nmul; i++) {
    const bool expl = !s.host_desc.empty();
    const MulDesc d = expl ? s.host_desc[i] : tree_desc(s.dv.tree, i);
    DescView one{};
    if (expl) {
      one.table = nullptr;
      one.ninl = 1;
      one.inl[0] = d;
    } else {
      // a one-group, two-node tree whose only product is d
      one.table = nullptr;
      one.tree.ngroups = 1;
      one.tree.j = s.dv.tree.j;
      one.tree.base[0] = d.a_off;
      one.tree.K[0] = (uint64_t)d.la + d.lb;
      one.tree.mpref[0] = 0;
      one.tree.mpref[1] = 1;
    }
    STCHK(launch_products(X, s, one, 1));
    if (s.cls != CLS_SCHOOL) {
      SegView sv{};
      sv.segs = nullptr;
      sv.nseg = 1;
      sv.iseg[0] = CrtSeg{d.c_off, d.r_off, (uint64_t)d.la + d.lb};
      const uint32_t nb = (uint32_t)((sv.iseg[0].len + CAT_CRT_BLOCK - 1) / CAT_CRT_BLOCK);
      sv.ipref[0] = 0;
      sv.ipref[1] = nb;
      STCHK(launch_crt(X, out_base(X, s), sv, nb, nullptr, nullptr, nullptr, s.cls == CLS_COLSUM, stage_as(s)));
    }
  }
  return copy_tails(X, s);
}

template <class F>
cat_status capture_graph(F&& rec, hipGraphExec_t* out) {
  HIPCHK(hipStreamBeginCapture(g.cap_stream, hipStreamCaptureModeThreadLocal));
  cat_status s = rec(g.cap_stream);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(g.cap_stream, &graph);
  if (s != CAT_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) {
    g.last_err = (int)e;
    return CAT_EDEVICE;
  }
  e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    g.last_err = (int)e;
    return CAT_EDEVICE;
  }
  return CAT_OK;
}

// R's node: clear the limbs above R's product, then the powers and R
cat_status run_rins_side(Exec& S, Plan& P, bool plain) {
  if (P.rins_fill_len > 0) {
    hipLaunchKernelGGL(k_fill, dim3((uint32_t)std::min<uint64_t>((P.rins_fill_len + 255) / 256, 1024)), dim3(256), 0,
                       S.st, S.W + P.rins_fill_pos, P.rins_fill_len, 0u);
    LAUNCHCHK();
    S.launches++;
  }
  for (size_t k = 0; k < P.post_final; k++) STCHK(plain ? run_stage_plain(S, P.post[k]) : run_stage_batched(S, P.post[k]));
  return CAT_OK;
}

cat_status run_phase2(Exec& X, Plan& P, bool plain) {
  std::vector<Stage>& st = plain ? P.plain : P.batched;
  if (P.rins_j >= 0) {
    // R is a node of Q_1's tree at the level of stage sr: the powers and R
    // run before it (beside the levels that follow the completion of the
    // groups with e >= 2 when the call has a side stream)
    const size_t sr = std::min<size_t>((size_t)P.rins_stage[plain ? 1 : 0], st.size());
    if (!plain && X.side && P.fork_count >= 0) {
      const size_t nf = std::min<size_t>((size_t)P.fork_count, sr);
      for (size_t k = 0; k < nf; k++) STCHK(run_stage_batched(X, st[k]));
      HIPCHK(hipEventRecord(g.ev_fork, X.st));
      HIPCHK(hipStreamWaitEvent(X.side, g.ev_fork, 0));
      for (size_t k = nf; k < sr; k++) STCHK(run_stage_batched(X, st[k]));
      Exec S = X;
      S.st = X.side;
      S.res = X.res2;
      S.res_stride = X.res2_stride;
      S.F = X.F2;
      S.flags = X.flags2;
      S.crt_epoch = 0;
      S.launches = 0;
      STCHK(run_rins_side(S, P, false));
      HIPCHK(hipEventRecord(g.ev_join, S.st));
      HIPCHK(hipStreamWaitEvent(X.st, g.ev_join, 0));
      X.launches += S.launches;
    } else {
      for (size_t k = 0; k < sr; k++) STCHK(plain ? run_stage_plain(X, st[k]) : run_stage_batched(X, st[k]));
      STCHK(run_rins_side(X, P, plain));
    }
    for (size_t k = sr; k < st.size(); k++) STCHK(plain ? run_stage_plain(X, st[k]) : run_stage_batched(X, st[k]));
    return CAT_OK;
  }
  if (!plain && X.side && P.fork_count >= 0) {
    // Q_1's upper levels on st; the powers and R on the side stream with
    // their own scratch; C = Q_1 R once both are done.  Q_1's levels are
    // issued first: a graph submits its nodes in the order they were
    // captured, and the short power steps issued first held the long levels
    // back until the whole chain had run.
    const size_t nf = std::min<size_t>((size_t)P.fork_count, st.size());
    for (size_t k = 0; k < nf; k++) STCHK(run_stage_batched(X, st[k]));
    HIPCHK(hipEventRecord(g.ev_fork, X.st));
    HIPCHK(hipStreamWaitEvent(X.side, g.ev_fork, 0));
    for (size_t k = nf; k < st.size(); k++) STCHK(run_stage_batched(X, st[k]));
    Exec S = X;
    S.st = X.side;
    S.res = X.res2;
    S.res_stride = X.res2_stride;
    S.F = X.F2;
    S.flags = X.flags2;
    S.crt_epoch = 0;
    S.launches = 0;
    for (size_t k = 0; k < P.post_final; k++) STCHK(run_stage_batched(S, P.post[k]));
    HIPCHK(hipEventRecord(g.ev_join, S.st));
    HIPCHK(hipStreamWaitEvent(X.st, g.ev_join, 0));
    for (size_t k = P.post_final; k < P.post.size(); k++) STCHK(run_stage_batched(X, P.post[k]));
    X.launches += S.launches;
    return CAT_OK;
  }
  for (const Stage& s : st) STCHK(plain ? run_stage_plain(X, s) : run_stage_batched(X, s));
  for (const Stage& s : P.post) STCHK(plain ? run_stage_plain(X, s) : run_stage_batched(X, s));
  return CAT_OK;
}

// ----------------------------------------------------------------------------
// Phase 1 launches (into the workspace; primes to `primes` with capacity cap)
// ----------------------------------------------------------------------------
cat_status run_phase1(const Layout& Ly, char* wb, uint32_t* primes, uint64_t cap, hipStream_t st, uint64_t* launches) {
  uint32_t* W = (uint32_t*)wb;
  GroupTable* gt = (GroupTable*)(wb + Ly.gtab);
  hipLaunchKernelGGL(k_seeds, dim3(1), dim3(1024), 0, st, Ly.n, (uint32_t)Ly.s, W + Ly.seeds, (int32_t*)(W + Ly.seed_e),
                     gt, (uint32_t*)gt, (uint64_t)Ly.ctl_words);
  LAUNCHCHK();
  if (Ly.nseg > 0) {
    if (Ly.seg_log == SIEVE_SEG_LOG_HUGE)
      hipLaunchKernelGGL(k_sieve<SIEVE_SEG_LOG_HUGE>, dim3((uint32_t)Ly.nseg), dim3(SIEVE_THREADS), 0, st, Ly.n, Ly.i0,
                         Ly.i_end, (const uint32_t*)(W + Ly.seeds), (const GroupTable*)gt, W + Ly.bitmap,
                         W + Ly.seg_cnt);
    else if (Ly.seg_log == SIEVE_SEG_LOG_BIG)
      hipLaunchKernelGGL(k_sieve<SIEVE_SEG_LOG_BIG>, dim3((uint32_t)Ly.nseg), dim3(SIEVE_THREADS), 0, st, Ly.n, Ly.i0,
                         Ly.i_end, (const uint32_t*)(W + Ly.seeds), (const GroupTable*)gt, W + Ly.bitmap,
                         W + Ly.seg_cnt);
    else
      hipLaunchKernelGGL(k_sieve<SIEVE_SEG_LOG>, dim3((uint32_t)Ly.nseg), dim3(SIEVE_THREADS), 0, st, Ly.n, Ly.i0,
                         Ly.i_end, (const uint32_t*)(W + Ly.seeds), (const GroupTable*)gt, W + Ly.bitmap,
                         W + Ly.seg_cnt);
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_groups, dim3(1), dim3(1024), 0, st, (uint32_t)Ly.nseg, (const uint32_t*)(W + Ly.seg_cnt),
                     W + Ly.seg_off, (const uint32_t*)(W + Ly.seeds), (const int32_t*)(W + Ly.seed_e), primes, cap, gt);
  LAUNCHCHK();
  if (Ly.nseg > 0) {
    if (Ly.seg_log == SIEVE_SEG_LOG_HUGE)
      hipLaunchKernelGGL(k_scatter<SIEVE_SEG_LOG_HUGE>, dim3((uint32_t)Ly.nseg), dim3(SIEVE_THREADS), 0, st, Ly.i0,
                         (const uint32_t*)(W + Ly.bitmap), (const uint32_t*)(W + Ly.seg_off), (const GroupTable*)gt,
                         primes, cap);
    else if (Ly.seg_log == SIEVE_SEG_LOG_BIG)
      hipLaunchKernelGGL(k_scatter<SIEVE_SEG_LOG_BIG>, dim3((uint32_t)Ly.nseg), dim3(SIEVE_THREADS), 0, st, Ly.i0,
                         (const uint32_t*)(W + Ly.bitmap), (const uint32_t*)(W + Ly.seg_off), (const GroupTable*)gt,
                         primes, cap);
    else
      hipLaunchKernelGGL(k_scatter<SIEVE_SEG_LOG>, dim3((uint32_t)Ly.nseg), dim3(SIEVE_THREADS), 0, st, Ly.i0,
                         (const uint32_t*)(W + Ly.bitmap), (const uint32_t*)(W + Ly.seg_off), (const GroupTable*)gt,
                         primes, cap);
    LAUNCHCHK();
  }
  *launches += Ly.nseg > 0 ? 4 : 2;
  return CAT_OK;
}

cat_status read_groups(const Layout& Ly, char* wb, hipStream_t st, GroupTable* out) {
  HIPCHK(hipMemcpyAsync(g.pin, wb + Ly.gtab, sizeof(GroupTable), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  memcpy(out, g.pin, sizeof(GroupTable));
  if (out->err & CAT_DEVERR_NEG_EXP) return CAT_EINTERNAL;
  if (out->ngroups > CAT_MAX_GROUPS) return CAT_EINTERNAL;
  return CAT_OK;
}

Plan* find_plan_in(std::map<uint64_t, Plan*>& plans, uint64_t n, const GroupTable& gt) {
  auto it = plans.find(n);
  if (it == plans.end()) return nullptr;
  Plan* P = it->second;
  if (P->ng != gt.ngroups) return nullptr;
  for (uint32_t k = 0; k < gt.ngroups; k++)
    if (P->exps[k] != gt.exps[k] || P->off[k + 1] != gt.off[k + 1] || P->gbits[k] != gt.gbits[k]) return nullptr;
  return P;
}

Plan* find_plan(uint64_t n, const GroupTable& gt) { return find_plan_in(g.plans, n, gt); }

// Plans of the allocation-free entry point: kept apart from the main cache
// (whose eviction destroys graphs); they hold no device memory, so dropping
// one frees host memory only.
#define NOALLOC_PLANS_MAX 64
void remember_noalloc_plan(Plan* P) {
  auto it = g.noalloc_plans.find(P->n);
  if (it != g.noalloc_plans.end()) {
    free_plan(it->second);
    g.noalloc_plans.erase(it);
    g.noalloc_order.erase(std::find(g.noalloc_order.begin(), g.noalloc_order.end(), P->n));
  }
  g.noalloc_plans[P->n] = P;
  g.noalloc_order.push_back(P->n);
  while (g.noalloc_order.size() > NOALLOC_PLANS_MAX) {
    const uint64_t old = g.noalloc_order.front();
    g.noalloc_order.erase(g.noalloc_order.begin());
    free_plan(g.noalloc_plans[old]);
    g.noalloc_plans.erase(old);
  }
}

void remember_plan(Plan* P) {
  auto it = g.plans.find(P->n);
  if (it != g.plans.end()) {
    free_plan(it->second);
    g.plans.erase(it);
    g.plan_order.erase(std::find(g.plan_order.begin(), g.plan_order.end(), P->n));
  }
  g.plans[P->n] = P;
  g.plan_order.push_back(P->n);
  while (g.plan_order.size() > 256) {
    const uint64_t old = g.plan_order.front();
    g.plan_order.erase(g.plan_order.begin());
    free_plan(g.plans[old]);
    g.plans.erase(old);
  }
}

Exec make_exec(const Layout& Ly, char* wb, hipStream_t st) {
  Exec X;
  X.W = (uint32_t*)wb;
  X.res = X.W + Ly.res;
  X.res_stride = Ly.res_len;
  X.F = X.W + Ly.F;
  X.err = (uint32_t*)(wb + Ly.err);
  X.flags = (uint32_t*)(wb + Ly.gtab + CTL_FLAGS);
  X.res2 = X.W + Ly.res2;
  X.res2_stride = Ly.res2_len;
  X.F2 = X.W + Ly.F2;
  X.flags2 = X.flags + Ly.nblk_max;
  X.st = st;
  return X;
}

// ----------------------------------------------------------------------------
// Generic batches c_i = a_i * b_i: products bucketed by class and transform
// length, one stage (launch sequence) per bucket.
// ----------------------------------------------------------------------------
// byte offsets inside a product plan's control block
#define MUL_CTL_FLAGS 16
struct MulPlanImpl {
  uint32_t batch = 0;
  uint32_t flags = 0;
  std::vector<Stage> stages;
  CopyList zeros{};                          // unused (zero-length products are rejected)
  void* dev = nullptr;
  uint64_t res_len = 0, F_words = 0, nblk_max = 0;
  size_t off_res = 0, off_F = 0, off_ctl = 0, total = 0;   // control block: error word | look-back flags
  uint64_t products = 0, product_limbs = 0;
  std::map<std::vector<uintptr_t>, hipGraphExec_t> graphs;
  std::vector<std::vector<uintptr_t>> graphs_order;
  std::vector<char> host_tables;             // source of an asynchronous table upload
};

// async_upload: the device tables are copied on `st` (ordered before the
// plan's launches there) instead of by a synchronous copy.
cat_status mul_plan_create(uint32_t batch, const uint64_t* a_off, const uint64_t* b_off, const uint64_t* c_off,
                           uint32_t flags, MulPlanImpl** out, bool async_upload = false, hipStream_t upload_st = nullptr) {
  if (!a_off || !b_off || (!c_off && batch > 0)) return CAT_EINVAL;
  MulPlanImpl* M = new MulPlanImpl();
  M->batch = batch;
  M->flags = flags;
  std::map<std::pair<int, int>, Stage> by;
  for (uint32_t i = 0; i < batch; i++) {
    if (a_off[i + 1] < a_off[i] || b_off[i + 1] < b_off[i]) { delete M; return CAT_EINVAL; }
    const uint64_t la = a_off[i + 1] - a_off[i], lb = b_off[i + 1] - b_off[i];
    if (la == 0 || lb == 0 || la + lb - 1 > (1ull << CAT_MAX_LOGN) || la >= (1ull << 31) || lb >= (1ull << 31)) {
      delete M;
      return CAT_EINVAL;
    }
    Cls cc = classify2(la, lb);
    if (colsum_wins(std::max(la, lb), std::min(la, lb), cc)) cc = Cls{CLS_COLSUM, 0, 0, 0};
    Stage& st = by[{cc.cls, cc.logN}];
    st.cls = cc.cls;
    st.logN = cc.logN;
    st.logM = cc.logM;
    st.maxL = cc.maxL;
    MulDesc d;
    d.a_off = a_off[i];
    d.b_off = b_off[i];
    d.c_off = c_off[i];
    d.r_off = st.limbs;
    d.la = (uint32_t)la;
    d.lb = (uint32_t)lb;
    st.host_desc.push_back(d);
    st.host_segs.push_back(CrtSeg{d.c_off, d.r_off, la + lb});
    st.limbs += la + lb;
  }
  uint64_t nblk = 0;
  for (auto& kv : by) {
    Stage& st = kv.second;
    st.nmul = st.host_desc.size();
    build_crt_segs(st);
    if (st.cls != CLS_SCHOOL) M->res_len = std::max(M->res_len, st.limbs);
    if (st.cls == CLS_LARGE) M->F_words = std::max<uint64_t>(M->F_words, st.nmul * 6ull << st.logN);
    nblk = std::max<uint64_t>(nblk, st.nblk);
    M->products += st.nmul;
    M->product_limbs += st.limbs;
    M->stages.push_back(st);
  }
  M->nblk_max = nblk + 1;
  // the one-workgroup buckets of up to 2^g_fuse_logn coefficients in one
  // fused launch (batched form, while they hold at most FUSE_MAX_LEAVES
  // coefficient slots: beyond that the per-bucket launches run at higher
  // occupancy)
  if (!(flags & CAT_MODE_PLAIN) && g_fuse_logn) {
    uint64_t slots = 0;
    int nf = 0;
    for (const Stage& st : M->stages)
      if (st.cls == CLS_LDS && st.logN <= (int)g_fuse_logn) {
        slots += st.nmul << st.logN;
        nf++;
      }
    if (nf > 0 && slots <= FUSE_MAX_LEAVES) {
      Stage f;
      f.cls = CLS_FUSED;
      std::vector<Stage> kept;
      for (Stage& st : M->stages) {
        if (!(st.cls == CLS_LDS && st.logN <= (int)g_fuse_logn)) {
          kept.push_back(st);
          continue;
        }
        const uint32_t per = FT_SLOTS >> st.logN;
        for (size_t i0 = 0; i0 < st.host_desc.size(); i0 += per) {
          const uint32_t cnt = (uint32_t)std::min<size_t>(per, st.host_desc.size() - i0);
          f.host_tiles.push_back(make_uint2((uint32_t)(f.host_desc.size() + i0), (uint32_t)st.logN | (cnt << 8)));
        }
        f.host_desc.insert(f.host_desc.end(), st.host_desc.begin(), st.host_desc.end());
        f.nmul += st.nmul;
        f.limbs += st.limbs;
        f.fused_bfly += bfly(9.0 * st.nmul, st.logN);
      }
      for (int k = 0; k <= FT_LOGT; k++)
        for (int q = 0; q < CAT_NPRIMES; q++) f.fm.scale[k][q] = k >= 1 ? scale_pair(q, k) : make_uint2(0, 0);
      M->stages = kept;
      M->stages.insert(M->stages.begin(), f);
    }
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  // the control block first: the error word of every product plan is the
  // first word of its workspace (bigint_mul_check reads it there)
  M->off_ctl = take(MUL_CTL_FLAGS + 4 * M->nblk_max);
  M->off_res = take(3 * (M->res_len + 64) * 4);
  M->off_F = take(M->F_words * 4);
  M->total = off;
  std::vector<Stage*> all;
  for (auto& st : M->stages) all.push_back(&st);
  cat_status e = upload_tables(all, &M->dev, true, async_upload ? &M->host_tables : nullptr, upload_st);
  if (e != CAT_OK) { delete M; return e; }
  *out = M;
  return CAT_OK;
}

void mul_plan_free(MulPlanImpl* M) {
  for (auto& kv : M->graphs) (void)hipGraphExecDestroy(kv.second);
  if (M->dev) (void)hipFree(M->dev);
  delete M;
}

// Plans of bigint_mul_batched, cached by shape (batch, mode and the three
// offset arrays), so that a call only queues work.  A plan is destroyed only
// once the event recorded after its last queued use has completed.
struct MulCacheEntry {
  std::vector<uint64_t> key;
  MulPlanImpl* M = nullptr;
  hipEvent_t ev = nullptr;   // after the last queued use
  hipEvent_t up = nullptr;   // after the table upload (a later call may come on another stream)
};
std::vector<MulCacheEntry> g_mul_cache;   // least recently used first
#define MUL_CACHE_MAX 16

void mul_cache_drop(MulCacheEntry& e) {
  if (e.ev) {
    (void)hipEventSynchronize(e.ev);
    (void)hipEventDestroy(e.ev);
  }
  if (e.up) (void)hipEventDestroy(e.up);
  mul_plan_free(e.M);
}

void mul_cache_clear() {
  for (auto& e : g_mul_cache) mul_cache_drop(e);
  g_mul_cache.clear();
}

Exec mul_exec(MulPlanImpl* M, const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_c, char* wb, hipStream_t st) {
  Exec X;
  X.W = (uint32_t*)wb;
  X.A = d_a;
  X.B = d_b;
  X.C = d_c;
  X.res = (uint32_t*)(wb + M->off_res);
  X.res_stride = M->res_len + 64;
  X.F = (uint32_t*)(wb + M->off_F);
  X.err = (uint32_t*)(wb + M->off_ctl);
  X.flags = (uint32_t*)(wb + M->off_ctl + MUL_CTL_FLAGS);
  X.st = st;
  return X;
}

cat_status mul_plan_record(MulPlanImpl* M, Exec& X, bool plain) {
  const uint64_t words = (MUL_CTL_FLAGS + 4 * M->nblk_max) / 4;
  hipLaunchKernelGGL(k_fill, dim3((uint32_t)std::min<uint64_t>((words + 255) / 256, 256)), dim3(256), 0, X.st, X.err,
                     words, 0u);
  LAUNCHCHK();
  X.launches++;
  for (const Stage& s : M->stages) STCHK(plain ? run_stage_plain(X, s) : run_stage_batched(X, s));
  return CAT_OK;
}

cat_status mul_plan_exec(MulPlanImpl* M, const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_c, void* d_work,
                         size_t work_bytes, hipStream_t st, uint64_t* launches) {
  if (work_bytes < M->total || (!d_work && M->total > 0)) return CAT_ENOMEM;
  if (M->batch == 0) return CAT_OK;
  if (!d_a || !d_b || !d_c) return CAT_EINVAL;
  char* wb = (char*)d_work;
  const bool plain = (M->flags & CAT_MODE_PLAIN) != 0;
  const bool use_graph = !plain && (M->flags & CAT_MODE_GRAPH) != 0;
  Exec X = mul_exec(M, d_a, d_b, d_c, wb, st);
  if (!use_graph) {
    STCHK(mul_plan_record(M, X, plain));
    *launches = X.launches;
    return CAT_OK;
  }
  std::vector<uintptr_t> key{(uintptr_t)d_a, (uintptr_t)d_b, (uintptr_t)d_c, (uintptr_t)wb};
  auto it = M->graphs.find(key);
  hipGraphExec_t ge = nullptr;
  if (it != M->graphs.end()) {
    ge = it->second;
    *launches = 1;
  } else {
    Exec C = X;
    C.st = g.cap_stream;
    HIPCHK(hipStreamBeginCapture(g.cap_stream, hipStreamCaptureModeThreadLocal));
    cat_status s = mul_plan_record(M, C, false);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(g.cap_stream, &graph);
    if (s != CAT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) {
      g.last_err = (int)e;
      return CAT_EDEVICE;
    }
    e = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      g.last_err = (int)e;
      return CAT_EDEVICE;
    }
    cache_graph(M->graphs, M->graphs_order, key, ge);
    *launches = C.launches;
  }
  HIPCHK(hipGraphLaunch(ge, st));
  return CAT_OK;
}

// ----------------------------------------------------------------------------
// Asynchronous C(n): tickets.  Each ticket owns a 2 KB slice of pinned host
// memory (group table, top index, error word) and an event; slices and events
// are pooled so the serving loop never allocates.
// ----------------------------------------------------------------------------
struct BatchState;
struct Ticket {
  uint64_t n = 0;
  Layout Ly;
  char* wb = nullptr;
  hipStream_t st = nullptr;
  int state = 0;              // 1: Phase 1 queued, 2: Phase 2 queued
  hipEvent_t ev = nullptr;
  char* pin = nullptr;
  bool one = false;           // C(n) = 1
  uint64_t cap = 0;
  BatchState* batch = nullptr;   // a batch of requests (catalan_batch_*)
};

struct TicketPool {
  char* pinned = nullptr;
  std::vector<char*> free_slices;
  std::vector<hipEvent_t> free_events;
};
TicketPool tp;
#define TICKET_SLICE 2048
#define TICKET_SLICES 4096

cat_status ticket_alloc(Ticket** out) {
  if (!tp.pinned) {
    HIPCHK(hipHostMalloc((void**)&tp.pinned, (size_t)TICKET_SLICE * TICKET_SLICES, hipHostMallocDefault));
    for (int k = TICKET_SLICES - 1; k >= 0; k--) tp.free_slices.push_back(tp.pinned + (size_t)k * TICKET_SLICE);
  }
  if (tp.free_slices.empty()) return CAT_ENOMEM;
  Ticket* t = new Ticket();
  t->pin = tp.free_slices.back();
  tp.free_slices.pop_back();
  if (!tp.free_events.empty()) {
    t->ev = tp.free_events.back();
    tp.free_events.pop_back();
  } else {
    hipError_t e = hipEventCreateWithFlags(&t->ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      tp.free_slices.push_back(t->pin);
      delete t;
      g.last_err = (int)e;
      return CAT_EDEVICE;
    }
  }
  *out = t;
  return CAT_OK;
}

void batch_free(BatchState* b);
void ticket_free(Ticket* t) {
  tp.free_slices.push_back(t->pin);
  tp.free_events.push_back(t->ev);
  if (t->batch) batch_free(t->batch);
  delete t;
}

// ----------------------------------------------------------------------------
// Batches of C(n) requests (continuous batching in a request loop): every
// request's Phase 1 runs in a small region of its own, its primes land in a
// staging array, and the primes of all requests are compacted into one array
// so that their groups sit side by side.  Phase 2 is planned once for all of
// them (at most CAT_MAX_GROUPS groups per plan; a larger batch is cut into
// chunks run one after another): each tree level of every request is one
// launch per kernel stage, and the powers, outer products and final products
// of all requests share the launches of their steps.
// ----------------------------------------------------------------------------
#define CAT_BATCH_MAX 32
#define BATCH_PIN (64 << 10)

// Phase 1 of one request of a batch: the sieve's scratch and a control block
Layout layout_phase1(uint64_t n) {
  Layout L;
  L.n = n;
  L.s = isqrt64(2 * n);
  L.i0 = (L.s + 1) / 2;
  L.i_end = n;
  L.seg_log = sieve_seg_log(L.i0, L.i_end);
  const uint64_t seg = 1ull << L.seg_log;
  L.nseg = L.i_end > L.i0 ? (L.i_end - L.i0 + seg - 1) / seg : 0;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  L.seeds = take(SEED_MAX * 4) / 4;
  L.seed_e = take(SEED_MAX * 4) / 4;
  L.seg_cnt = take((L.nseg + 1) * 4) / 4;
  L.seg_off = take((L.nseg + 1) * 4) / 4;
  L.bitmap = take(L.nseg * (seg / 32) * 4) / 4;
  L.gtab = take(CTL_READ);
  L.top = L.gtab + CTL_TOP;
  L.err = L.gtab + CTL_ERR;
  L.ctl_words = CTL_READ / 4;
  L.total = off;
  return L;
}

struct BatchLayout {
  uint32_t k = 0;
  std::vector<uint64_t> n;
  std::vector<Layout> p1;
  std::vector<size_t> p1_off;      // bytes
  std::vector<uint64_t> kmax;      // prime capacity of each request
  std::vector<uint64_t> stage;     // request's primes in the staging array (uint32 units)
  Layout c;                        // Phase 2 of all requests
  size_t c_off = 0, tops_off = 0, total = 0;
};

BatchLayout make_batch_layout(uint32_t k, const uint64_t* ns) {
  BatchLayout B;
  B.k = k;
  size_t off = 0;
  uint64_t ksum = 0, post = 0;
  for (uint32_t r = 0; r < k; r++) {
    const Layout full = make_layout(ns[r]);
    B.n.push_back(ns[r]);
    B.p1.push_back(layout_phase1(ns[r]));
    B.p1_off.push_back(off);
    off = align_up(off + B.p1.back().total, 256);
    B.kmax.push_back(full.Kmax);
    B.stage.push_back(ksum);
    ksum += full.Kmax;
    post += full.post_cap;
  }
  Layout L;
  L.n = 0;
  L.Kmax = std::max<uint64_t>(ksum, 16);
  L.post_cap = post + 4096;
  L.res2_len = 4096;
  B.c = layout_finish(L);
  B.c_off = off;
  off = align_up(off + B.c.total, 256);
  B.tops_off = off;
  off = align_up(off + 8 * (size_t)k, 256);
  B.total = off;
  return B;
}

struct BatchState {
  BatchLayout B;
  char* pin = nullptr;                     // group tables | tops | error word (pinned)
  std::vector<cat_status> status;          // per request
  std::vector<size_t> cap;
};

struct BigPinPool {
  std::vector<char*> free_bufs;
};
BigPinPool bpp;

void batch_free(BatchState* b) {
  if (b->pin) bpp.free_bufs.push_back(b->pin);
  delete b;
}

// byte offsets inside a batch's pinned buffer
inline size_t bpin_gt(uint32_t r) { return (size_t)r * sizeof(GroupTable); }
inline size_t bpin_tops() { return (size_t)CAT_BATCH_MAX * sizeof(GroupTable); }
inline size_t bpin_err() { return bpin_tops() + 8 * CAT_BATCH_MAX; }
static_assert(CAT_BATCH_MAX * sizeof(GroupTable) + 8 * CAT_BATCH_MAX + 16 <= BATCH_PIN, "batch pinned buffer");

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
// ----------------------------------------------------------------------------
// Products of prime powers from a caller's grouped factorisation (Alg. 2 on
// groups read from a factorisation file, or any other exponent source)
// ----------------------------------------------------------------------------
struct GroupsIn {
  uint32_t ng = 0;
  uint32_t exps[CAT_MAX_GROUPS];
  uint64_t off[CAT_MAX_GROUPS + 1];
  uint64_t total = 0;
  double lbits = 0;   // bound on log2 of the product from max_entry_bits
};

cat_status groups_in(const uint32_t* h_exps, const uint64_t* h_off, uint32_t ngroups, uint32_t max_entry_bits,
                     GroupsIn* out) {
  if (ngroups > CAT_MAX_GROUPS || (ngroups && (!h_exps || !h_off))) return CAT_EINVAL;
  if (max_entry_bits < 1 || max_entry_bits > 32) return CAT_EINVAL;
  if (ngroups && h_off[0] != 0) return CAT_EINVAL;
  GroupsIn G;
  G.off[0] = 0;
  uint32_t last = 0;
  for (uint32_t g = 0; g < ngroups; g++) {
    if (h_off[g + 1] < h_off[g] || h_exps[g] == 0) return CAT_EINVAL;
    if (h_off[g + 1] == h_off[g]) continue;          // empty groups are dropped
    if (h_exps[g] <= last) return CAT_EINVAL;         // one group per exponent, ascending
    last = h_exps[g];
    G.exps[G.ng] = h_exps[g];
    G.off[G.ng + 1] = G.off[G.ng] + (h_off[g + 1] - h_off[g]);
    G.lbits += (double)h_exps[g] * (double)(h_off[g + 1] - h_off[g]) * max_entry_bits;
    G.ng++;
  }
  G.total = G.off[G.ng];
  if (G.total >= (1ull << 32)) return CAT_ERANGE;
  *out = G;
  return CAT_OK;
}

// Arena room for R's node in Q_1's tree (at most a quarter of the longest
// tree, rounded to a power of two): 2^(ceil(log2 K) - 2) leaves beyond K.
uint64_t rins_room(uint64_t K) {
  const int c = ceil_log2(std::max<uint64_t>(K, 1));
  return c >= 2 ? (1ull << (c - 2)) : 0;
}

Layout make_layout_groups(const GroupsIn& G) {
  Layout L;
  L.n = 0;
  L.Kmax = std::max<uint64_t>(G.total + rins_room(G.total), 16);
  // the power chains (about twice their results), the outer tree (one pass
  // over the powers per level) and the final product
  uint32_t nchain = 0;
  for (uint32_t q = 0; q < G.ng; q++) nchain += G.exps[q] >= 2;
  const double levels = nchain > 1 ? std::ceil(std::log2((double)nchain)) : 0.0;
  L.post_cap = (uint64_t)((5.0 + levels) * (G.lbits + 64.0) / 32.0) + L.Kmax + 256ull * G.ng + 8192;
  // one stage's products (a step of every chain, a level of the outer tree,
  // or the final product) add up to at most the result's bound
  L.res_len = std::max<uint64_t>(L.Kmax, (uint64_t)((G.lbits + 64.0) / 32.0) + 64ull * G.ng + 4096) + 64;
  L.res2_len = 4096;
  return layout_finish(L);
}

// ----------------------------------------------------------------------------
// Factorial ratios N = prod_i a_i! / prod_j b_j! (Sec. 6.3)
// ----------------------------------------------------------------------------
struct RatioSpec {
  RatioTerms rt{};
  uint64_t A = 0;        // largest argument
  uint64_t S = 0;        // sum of the numerator arguments
  double log2N = 0;      // log2 of N (from log-gamma), 0 when N = 1
};

cat_status ratio_spec(const uint64_t* a, uint32_t k, const uint64_t* b, uint32_t m, RatioSpec* out) {
  if (k > RATIO_MAX_TERMS || m > RATIO_MAX_TERMS || (k && !a) || (m && !b)) return CAT_EINVAL;
  RatioSpec r;
  r.rt.k = k;
  r.rt.m = m;
  double lg = 0;
  for (uint32_t i = 0; i < k; i++) {
    if (a[i] > 0xFFFFFFFFull) return CAT_EINVAL;
    r.rt.a[i] = (uint32_t)a[i];
    r.A = std::max(r.A, a[i]);
    r.S += a[i];
    lg += std::lgamma((double)a[i] + 1.0);
  }
  for (uint32_t j = 0; j < m; j++) {
    if (b[j] > 0xFFFFFFFFull) return CAT_EINVAL;
    r.rt.b[j] = (uint32_t)b[j];
    r.A = std::max(r.A, b[j]);
    lg -= std::lgamma((double)b[j] + 1.0);
  }
  r.log2N = std::max(0.0, lg / std::log(2.0));
  *out = r;
  // N itself must fit the longest exact product (2^27 coefficients)
  if (r.log2N > 32.0 * (double)((1ull << CAT_MAX_LOGN) - 64)) return CAT_ERANGE;
  return CAT_OK;
}

// upper bound on the limbs of N (a non-integral ratio is rejected later)
uint64_t ratio_limbs_bound(const RatioSpec& r) {
  return (uint64_t)((r.log2N * (1.0 + 1e-12) + 64.0) / 32.0) + 2;
}

Layout make_layout_ratio(const RatioSpec& r) {
  Layout L;
  L.n = 0;
  L.s = isqrt64(r.A);
  L.i0 = (L.s + 1) / 2;
  L.i_end = (r.A + 1) / 2;   // odd m = 2i + 1 <= A
  L.np_cap = pi_bound(r.A) + 64;
  L.nchunks = (L.np_cap + RATIO_CHUNK - 1) / RATIO_CHUNK;
  // grouped entries: p enters once per set bit of v_p(N) <= S / (p - 1), so a
  // bit t needs p <= S / 2^t + 1
  uint64_t ent = 0;
  for (uint64_t x = r.S; x >= 1; x >>= 1) ent += pi_bound(std::min<uint64_t>(r.A, x + 1));
  L.Kmax = std::max<uint64_t>(ent + rins_room(ent), 16);
  // post-tree allocations: the power chains, the outer tree and the final
  // product together stay below 16 log2(N) / 32 limbs plus the operands' slack
  L.post_cap = (uint64_t)(16.0 * (r.log2N + 64.0) / 32.0) + L.Kmax + 8192;
  // one stage's products add up to at most sum_p v_p(N) bitlen(p) <= 2 log2 N
  // bits (plus a few limbs per group)
  L.res_len = std::max<uint64_t>(L.Kmax, (uint64_t)(2.0 * (r.log2N + 64.0) / 32.0) + 4096) + 64;
  L.res2_len = 4096;
  return layout_finish(L);
}

cat_status run_phase1_ratio(const Layout& Ly, const RatioSpec& r, char* wb, uint32_t* primes, uint64_t cap,
                            hipStream_t st, uint64_t* launches) {
  uint32_t* W = (uint32_t*)wb;
  GroupTable* gt = (GroupTable*)(wb + Ly.gtab);
  RatioCounts* rc = (RatioCounts*)(wb + Ly.rcounts);
  hipLaunchKernelGGL(k_rseeds, dim3(1), dim3(1024), 0, st, r.rt, (uint32_t)Ly.s, W + Ly.seeds, W + Ly.seed_e, gt,
                     (uint32_t*)gt, (uint64_t)Ly.ctl_words, rc);
  LAUNCHCHK();
  if (Ly.nseg > 0) {
    hipLaunchKernelGGL(k_rsieve, dim3((uint32_t)Ly.nseg), dim3(SIEVE_THREADS), 0, st, r.rt, Ly.i0, Ly.i_end,
                       (const uint32_t*)(W + Ly.seeds), gt, W + Ly.bitmap, W + Ly.seg_cnt);
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_rscan, dim3(1), dim3(1024), 0, st, (uint32_t)Ly.nseg, (const uint32_t*)(W + Ly.seg_cnt),
                     W + Ly.seg_off, (const uint32_t*)(W + Ly.seeds), (const uint32_t*)(W + Ly.seed_e), gt, W + Ly.P,
                     W + Ly.E, (uint64_t)Ly.np_cap, rc);
  LAUNCHCHK();
  if (Ly.nseg > 0) {
    hipLaunchKernelGGL(k_rscatter, dim3((uint32_t)Ly.nseg), dim3(SIEVE_THREADS), 0, st, r.rt, Ly.i0,
                       (const uint32_t*)(W + Ly.bitmap), (const uint32_t*)(W + Ly.seg_off), (const GroupTable*)gt,
                       W + Ly.P, W + Ly.E, (uint64_t)Ly.np_cap);
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_rbits, dim3((uint32_t)Ly.nchunks), dim3(256), 0, st, (const uint32_t*)(W + Ly.P),
                     (const uint32_t*)(W + Ly.E), (const RatioCounts*)rc, W + Ly.chunk_cnt, rc);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_rbitscan, dim3(32), dim3(1024), 0, st, (uint32_t)Ly.nchunks, (const uint32_t*)(W + Ly.chunk_cnt),
                     W + Ly.chunk_off);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_rtable, dim3(1), dim3(64), 0, st, (const RatioCounts*)rc, gt, cap);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_rbitscatter, dim3((uint32_t)Ly.nchunks), dim3(256), 0, st, (const uint32_t*)(W + Ly.P),
                     (const uint32_t*)(W + Ly.E), (const RatioCounts*)rc, (const uint32_t*)(W + Ly.chunk_off),
                     (const GroupTable*)gt, primes, cap);
  LAUNCHCHK();
  *launches += Ly.nseg > 0 ? 8 : 6;
  return CAT_OK;
}

// the group table of a ratio's Phase 1, with its error word mapped
cat_status read_groups_ratio(const Layout& Ly, char* wb, hipStream_t st, GroupTable* out) {
  HIPCHK(hipMemcpyAsync(g.pin, wb + Ly.gtab, sizeof(GroupTable), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  memcpy(out, g.pin, sizeof(GroupTable));
  if (out->err & CAT_DEVERR_NEG_EXP) return CAT_EINVAL;    // N is not an integer
  if (out->err & CAT_DEVERR_RANGE) return CAT_ERANGE;      // an exponent reaches 2^32
  if (out->err & CAT_DEVERR_BOUNDS) return CAT_EINTERNAL;
  if (out->ngroups > CAT_MAX_GROUPS) return CAT_EINTERNAL;
  return CAT_OK;
}

// The general form of a C(n) call in a given workspace: Phase 1, the group
// table to the host, the plan of n (cached by n), Phase 2 as launches or as
// one captured graph, the normalisation and the copy of the result to
// d_limbs.  With `noalloc` nothing is allocated on the device: the plan comes
// from a cache of its own whose plans carry no device tables and no graphs.
static cat_status exact_in_workspace(uint64_t n, const Layout& Ly, char* wb, uint32_t* d_limbs, size_t cap,
                              size_t* n_limbs, hipStream_t st, bool plain, bool use_graph, bool noalloc,
                              uint64_t launches) {
  cat_stats stats{};
  unsigned long long* top = (unsigned long long*)(wb + Ly.top);
  STCHK(run_phase1(Ly, wb, (uint32_t*)wb + Ly.primes, Ly.Kmax, st, &launches));
  GroupTable gt;
  STCHK(read_groups(Ly, wb, st, &gt));
  if (gt.err & CAT_DEVERR_BOUNDS) return CAT_EINTERNAL;
  Plan* P = noalloc ? find_plan_in(g.noalloc_plans, n, gt) : find_plan(n, gt);
  if (!P) {
    STCHK(make_plan(Ly, gt, &P, !noalloc));
    if (noalloc) remember_noalloc_plan(P);
    else remember_plan(P);
  }
  Exec X = make_exec(Ly, wb, st);
  uint32_t* W = X.W;
  if (P->result_is_one) {
    if (cap < 1) {
      *n_limbs = 1;
      return CAT_ERANGE;
    }
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, d_limbs, (uint64_t)1, 1u);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(st));
    *n_limbs = 1;
    g.stats = stats;
    return CAT_OK;
  }
  auto record = [&](Exec& E) -> cat_status {
    STCHK(run_phase2(E, *P, plain));
    const uint32_t blocks = top_scan_blocks(P->result_cap);
    hipLaunchKernelGGL(k_top_nonzero, dim3(blocks), dim3(256), 0, E.st, W + P->result_pos, P->result_cap, top,
                       (uint32_t*)nullptr, (uint64_t)0);
    LAUNCHCHK();
    E.launches++;
    return CAT_OK;
  };
  bool replayed = false;
  if (use_graph) {
    hipGraphExec_t ge = nullptr;
    auto it = P->graphs.find((uintptr_t)wb);
    if (it != P->graphs.end()) {
      ge = it->second;
      replayed = true;
    } else {
      Exec C = X;
      C.st = g.cap_stream;
      C.side = g.side_stream;
      HIPCHK(hipStreamBeginCapture(g.cap_stream, hipStreamCaptureModeThreadLocal));
      cat_status s = record(C);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(g.cap_stream, &graph);
      if (s != CAT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
      }
      if (e != hipSuccess) {
        g.last_err = (int)e;
        return CAT_EDEVICE;
      }
      e = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) {
        g.last_err = (int)e;
        return CAT_EDEVICE;
      }
      cache_graph(P->graphs, P->graphs_order, (uintptr_t)wb, ge);
      launches += C.launches;
    }
    HIPCHK(hipGraphLaunch(ge, st));
    if (replayed) launches += 1;
  } else {
    STCHK(record(X));
    launches += X.launches;
  }
  // top limb index and error word (adjacent in the control block)
  HIPCHK(hipMemcpyAsync(g.pin, wb + Ly.top, 12, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  uint64_t L = 0;
  uint32_t derr = 0;
  memcpy(&L, g.pin, 8);
  memcpy(&derr, (char*)g.pin + 8, 4);
  if (derr) return CAT_EINTERNAL;
  if (L == 0) return CAT_EINTERNAL;   // C(n) >= 1
  *n_limbs = (size_t)L;
  stats.products = P->products;
  stats.product_limbs = P->product_limbs;
  stats.launches = launches;
  stats.n_primes = gt.off[gt.ngroups];
  stats.levels = P->levels;
  stats.outer_level = P->rins_j;
  stats.graph_replayed = replayed ? 1 : 0;
  g.stats = stats;
  if (cap < L) return CAT_ERANGE;
  HIPCHK(hipMemcpyAsync(d_limbs, W + P->result_pos, L * 4, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return CAT_OK;
}

extern "C" {

cat_status cat_init(int device) {
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  return init_locked(device);
}

const char* cat_strerror(cat_status s) {
  switch (s) {
    case CAT_OK: return "ok";
    case CAT_EINVAL: return "invalid argument";
    case CAT_ERANGE: return "capacity too small";
    case CAT_ENOMEM: return "workspace too small or allocation failed";
    case CAT_EDEVICE: return "HIP runtime error";
    case CAT_EINTERNAL: return "device invariant violated";
    case CAT_EAGAIN: return "not finished yet";
    default: return "unknown status";
  }
}

int cat_last_device_error(void) { return g.last_err; }

cat_status cat_tune_set(const cat_tuning* t) {
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  const cat_tuning v = t ? *t : default_tuning();
  if (!tuning_valid(v)) return CAT_EINVAL;
  g_tune = v;
  // cached plans and graphs were made with the old schedule
  mul_cache_clear();
  if (!g.plans.empty()) HIPCHK(hipDeviceSynchronize());
  for (auto& kv : g.plans) free_plan(kv.second);
  g.plans.clear();
  g.plan_order.clear();
  return CAT_OK;
}

cat_status cat_fused_levels_set(uint32_t max_logn) {
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  if (max_logn == CAT_FUSED_DEFAULT) {
    g_fuse_logn = FT_LOGT;
    g_fuse_tree_logn = 0;
  } else {
    if (max_logn != 0 && (max_logn < 4 || max_logn > FT_LOGT)) return CAT_EINVAL;
    g_fuse_logn = max_logn;
    g_fuse_tree_logn = max_logn;
  }
  // cached plans were made with the old setting
  if (!g.plans.empty() || !g.noalloc_plans.empty()) HIPCHK(hipDeviceSynchronize());
  for (auto& kv : g.plans) free_plan(kv.second);
  g.plans.clear();
  g.plan_order.clear();
  for (auto& kv : g.noalloc_plans) free_plan(kv.second);
  g.noalloc_plans.clear();
  g.noalloc_order.clear();
  return CAT_OK;
}

cat_status cat_outer_node_set(uint32_t on) {
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  if (on > 1) return CAT_EINVAL;
  g_rins = on != 0;
  // cached plans and their graphs were made with the old setting
  if (!g.plans.empty() || !g.noalloc_plans.empty()) HIPCHK(hipDeviceSynchronize());
  for (auto& kv : g.plans) free_plan(kv.second);
  g.plans.clear();
  g.plan_order.clear();
  for (auto& kv : g.noalloc_plans) free_plan(kv.second);
  g.noalloc_plans.clear();
  g.noalloc_order.clear();
  return CAT_OK;
}

cat_status cat_lazy_primes_set(uint32_t max_logn) {
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  if (max_logn > CAT_LAZY_MAX_LOGN) return CAT_EINVAL;
  g_lazy_logn = max_logn;
  // cached plans and their graphs were made with the old setting
  if (!g.plans.empty() || !g.noalloc_plans.empty()) HIPCHK(hipDeviceSynchronize());
  for (auto& kv : g.plans) free_plan(kv.second);
  g.plans.clear();
  g.plan_order.clear();
  for (auto& kv : g.noalloc_plans) free_plan(kv.second);
  g.noalloc_plans.clear();
  g.noalloc_order.clear();
  mul_cache_clear();
  return CAT_OK;
}

cat_status cat_lookback_polls_set(uint32_t polls) {
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  if (polls > (1u << 20) && polls != CAT_POLLS_AUTO) return CAT_EINVAL;
  g_crt_polls = polls;
  // cached graphs of C(n) carry the old value
  if (!g.plans.empty()) HIPCHK(hipDeviceSynchronize());
  for (auto& kv : g.plans) free_plan(kv.second);
  g.plans.clear();
  g.plan_order.clear();
  return CAT_OK;
}

cat_status cat_tune_get(cat_tuning* t) {
  if (!t) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  *t = g_tune;
  return CAT_OK;
}

cat_status cat_timer_set(const char* kernel) {
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  g.timer_name = kernel ? kernel : "";
  g.timer_used = 0;
  g.timer_work = 0;
  return CAT_OK;
}

cat_status cat_timer_get(double* ms, uint64_t* launches, double* work) {
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  double tot = 0;
  for (size_t i = 0; i < g.timer_used; i++) {
    HIPCHK(hipEventSynchronize(g.timer_ev[i].second));
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, g.timer_ev[i].first, g.timer_ev[i].second));
    tot += t;
  }
  if (ms) *ms = tot;
  if (launches) *launches = g.timer_used;
  if (work) *work = g.timer_work;
  return CAT_OK;
}

cat_status cat_get_stats(cat_stats* out) {
  if (!out) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  *out = g.stats;
  return CAT_OK;
}

cat_status catalan_sizes(uint64_t n, size_t* max_primes, size_t* max_limbs, size_t* workspace_bytes) {
  if (n > CAT_N_MAX) return CAT_EINVAL;
  const Layout Ly = make_layout(n);
  if (max_primes) *max_primes = (size_t)Ly.Kmax;
  if (max_limbs) *max_limbs = (size_t)((2 * n + 1) / 32 + 2);
  if (workspace_bytes) *workspace_bytes = Ly.total;
  return CAT_OK;
}

cat_status catalan_factor(uint64_t n, uint32_t* d_primes, size_t primes_cap, uint32_t* h_exps, uint64_t* h_off,
                          uint32_t* n_groups, size_t* n_primes, void* d_work, size_t work_bytes, void* stream) {
  if (n > CAT_N_MAX || !h_exps || !h_off || !n_groups || !n_primes || !d_work) return CAT_EINVAL;
  if (!d_primes && primes_cap > 0) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  const Layout Ly = make_layout(n);
  if (work_bytes < Ly.total) return CAT_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  uint64_t launches = 0;
  uint32_t dummy = 0;
  STCHK(run_phase1(Ly, (char*)d_work, d_primes ? d_primes : &dummy, d_primes ? primes_cap : 0, st, &launches));
  GroupTable gt;
  STCHK(read_groups(Ly, (char*)d_work, st, &gt));
  *n_groups = gt.ngroups;
  for (uint32_t k = 0; k < gt.ngroups; k++) h_exps[k] = gt.exps[k];
  for (uint32_t k = 0; k <= gt.ngroups; k++) h_off[k] = gt.off[k];
  *n_primes = (size_t)gt.off[gt.ngroups];
  g.stats = cat_stats{};
  g.stats.launches = launches;
  g.stats.n_primes = *n_primes;
  if (*n_primes > primes_cap) return CAT_ERANGE;
  return CAT_OK;
}

cat_status catalan_exact_ex(uint64_t n, uint32_t* d_limbs, size_t cap, size_t* n_limbs, void* d_work, size_t work_bytes,
                            void* stream, uint32_t flags) {
  if (n > CAT_N_MAX || !n_limbs) return CAT_EINVAL;
  if (!d_limbs) {
    *n_limbs = (size_t)((2 * n + 1) / 32 + 2);
    return CAT_OK;
  }
  if (!d_work) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  const Layout Ly = make_layout(n);
  if (work_bytes < Ly.total) return CAT_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  char* wb = (char*)d_work;
  const bool plain = (flags & CAT_MODE_PLAIN) != 0;
  const bool use_graph = !plain && (flags & CAT_MODE_GRAPH) != 0;
  cat_stats stats{};
  uint64_t launches = 0;
  unsigned long long* top = (unsigned long long*)(wb + Ly.top);
  // Fast path: the plan of n is known (it depends only on n).  One graph runs
  // Phase 1, Phase 2, the normalisation and the copy out; the group table the
  // device computed is checked against the plan afterwards.
  auto pit = g.plans.find(n);
  if (use_graph && pit != g.plans.end() && !pit->second->result_is_one) {
    Plan* P = pit->second;
    const std::vector<uintptr_t> key{(uintptr_t)wb, (uintptr_t)d_limbs, (uintptr_t)cap};
    hipGraphExec_t ge = nullptr;
    bool replayed = false;
    auto git = P->full_graphs.find(key);
    if (git != P->full_graphs.end()) {
      ge = git->second;
      replayed = true;
    } else {
      uint64_t nl = 0;
      STCHK(capture_graph(
          [&](hipStream_t cs) -> cat_status {
            STCHK(run_phase1(Ly, wb, (uint32_t*)wb + Ly.primes, Ly.Kmax, cs, &nl));
            Exec E = make_exec(Ly, wb, cs);
            E.side = g.side_stream;
            STCHK(run_phase2(E, *P, false));
            const uint32_t blocks = top_scan_blocks(P->result_cap);
            const uint64_t ncopy = std::min<uint64_t>(P->result_cap, cap);
            hipLaunchKernelGGL(k_top_nonzero, dim3(blocks), dim3(256), 0, cs, E.W + P->result_pos, P->result_cap,
                               top, d_limbs, ncopy);
            LAUNCHCHK();
            nl += E.launches + 1;
            return CAT_OK;
          },
          &ge));
      cache_graph(P->full_graphs, P->full_graphs_order, key, ge);
      launches = nl;
    }
    HIPCHK(hipGraphLaunch(ge, st));
    // group table, top and error word in one copy
    char* pin = (char*)g.pin;
    HIPCHK(hipMemcpyAsync(pin, wb + Ly.gtab, CTL_READ, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    GroupTable gt;
    memcpy(&gt, pin, sizeof(GroupTable));
    uint64_t L = 0;
    uint32_t derr = 0;
    memcpy(&L, pin + CTL_TOP, 8);
    memcpy(&derr, pin + CTL_ERR, 4);
    if (gt.err || find_plan(n, gt) != P) return CAT_EINTERNAL;
    if (derr || L == 0) return CAT_EINTERNAL;
    *n_limbs = (size_t)L;
    stats.products = P->products;
    stats.product_limbs = P->product_limbs;
    stats.launches = replayed ? 1 : launches;
    stats.n_primes = gt.off[gt.ngroups];
    stats.levels = P->levels;
  stats.outer_level = P->rins_j;
    stats.graph_replayed = replayed ? 1 : 0;
    g.stats = stats;
    if (cap < L) return CAT_ERANGE;
    return CAT_OK;
  }
  return exact_in_workspace(n, Ly, wb, d_limbs, cap, n_limbs, st, plain, use_graph, false, launches);
}


cat_status cat_mul_plan_create(uint32_t batch, const uint64_t* h_a_off, const uint64_t* h_b_off,
                               const uint64_t* h_c_off, uint32_t flags, cat_mul_plan* plan,
                               size_t* workspace_bytes) {
  if (!plan) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  MulPlanImpl* M = nullptr;
  STCHK(mul_plan_create(batch, h_a_off, h_b_off, h_c_off, flags, &M));
  *plan = (cat_mul_plan)M;
  if (workspace_bytes) *workspace_bytes = M->total;
  return CAT_OK;
}

cat_status cat_mul_plan_exec(cat_mul_plan plan, const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_c,
                             void* d_work, size_t work_bytes, void* stream) {
  if (!plan) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(set_device());
  MulPlanImpl* M = (MulPlanImpl*)plan;
  uint64_t launches = 0;
  STCHK(mul_plan_exec(M, d_a, d_b, d_c, d_work, work_bytes, (hipStream_t)stream, &launches));
  cat_stats st{};
  st.products = M->products;
  st.product_limbs = M->product_limbs;
  st.launches = launches;
  st.graph_replayed = (M->flags & CAT_MODE_GRAPH) && launches == 1 ? 1 : 0;
  g.stats = st;
  return CAT_OK;
}

cat_status cat_mul_plan_check(cat_mul_plan plan, void* d_work, void* stream) {
  if (!plan || !d_work) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  MulPlanImpl* M = (MulPlanImpl*)plan;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipMemcpyAsync(g.pin, (char*)d_work + M->off_ctl, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  uint32_t e = 0;
  memcpy(&e, g.pin, 4);
  return e ? CAT_EINTERNAL : CAT_OK;
}

cat_status cat_mul_plan_destroy(cat_mul_plan plan) {
  if (!plan) return CAT_OK;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  HIPCHK(hipDeviceSynchronize());
  mul_plan_free((MulPlanImpl*)plan);
  return CAT_OK;
}

cat_status bigint_mul_workspace(uint32_t batch, const uint64_t* h_a_off, const uint64_t* h_b_off,
                                size_t* workspace_bytes) {
  if (!workspace_bytes) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  std::vector<uint64_t> c(batch + 1, 0);
  MulPlanImpl* M = nullptr;
  STCHK(mul_plan_create(batch, h_a_off, h_b_off, c.data(), 0, &M));
  *workspace_bytes = M->total;
  mul_plan_free(M);
  return CAT_OK;
}

cat_status bigint_mul_batched_ex(uint32_t batch, const uint32_t* d_a, const uint64_t* h_a_off, const uint32_t* d_b,
                                 const uint64_t* h_b_off, uint32_t* d_c, const uint64_t* h_c_off, void* d_work,
                                 size_t work_bytes, void* stream, uint32_t flags) {
  if (!h_a_off || !h_b_off || (batch > 0 && !h_c_off)) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  hipStream_t st = (hipStream_t)stream;
  const uint32_t mode = flags & CAT_MODE_PLAIN;
  std::vector<uint64_t> key;
  key.reserve(3 * (size_t)batch + 4);
  key.push_back(batch);
  key.push_back(mode);
  key.insert(key.end(), h_a_off, h_a_off + batch + 1);
  key.insert(key.end(), h_b_off, h_b_off + batch + 1);
  if (batch) key.insert(key.end(), h_c_off, h_c_off + batch);
  size_t k = 0;
  while (k < g_mul_cache.size() && g_mul_cache[k].key != key) k++;
  if (k < g_mul_cache.size()) {
    MulCacheEntry e = g_mul_cache[k];
    g_mul_cache.erase(g_mul_cache.begin() + k);
    g_mul_cache.push_back(e);
    HIPCHK(hipStreamWaitEvent(st, e.up, 0));
  } else {
    MulCacheEntry e;
    STCHK(mul_plan_create(batch, h_a_off, h_b_off, h_c_off, mode, &e.M, true, st));
    hipError_t he = hipEventCreateWithFlags(&e.ev, hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&e.up, hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventRecord(e.up, st);
    if (he != hipSuccess) {
      (void)hipStreamSynchronize(st);
      if (e.ev) (void)hipEventDestroy(e.ev);
      if (e.up) (void)hipEventDestroy(e.up);
      mul_plan_free(e.M);
      g.last_err = (int)he;
      return CAT_EDEVICE;
    }
    e.key.swap(key);
    if (g_mul_cache.size() >= MUL_CACHE_MAX) {
      mul_cache_drop(g_mul_cache.front());
      g_mul_cache.erase(g_mul_cache.begin());
    }
    g_mul_cache.push_back(e);
  }
  MulCacheEntry& e = g_mul_cache.back();
  uint64_t launches = 0;
  cat_status s = mul_plan_exec(e.M, d_a, d_b, d_c, d_work, work_bytes, st, &launches);
  const hipError_t he = hipEventRecord(e.ev, st);
  if (s == CAT_OK && he != hipSuccess) {
    g.last_err = (int)he;
    s = CAT_EDEVICE;
  }
  cat_stats stt{};
  stt.products = e.M->products;
  stt.product_limbs = e.M->product_limbs;
  stt.launches = launches;
  g.stats = stt;
  return s;
}

cat_status bigint_mul_check(void* d_work, void* stream) {
  if (!d_work) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(set_device());
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipMemcpyAsync(g.pin, d_work, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  uint32_t e = 0;
  memcpy(&e, g.pin, 4);
  return e ? CAT_EINTERNAL : CAT_OK;
}

cat_status bigint_mul_batched(uint32_t batch, const uint32_t* d_a, const uint64_t* h_a_off, const uint32_t* d_b,
                              const uint64_t* h_b_off, uint32_t* d_c, const uint64_t* h_c_off, void* d_work,
                              size_t work_bytes, void* stream) {
  return bigint_mul_batched_ex(batch, d_a, h_a_off, d_b, h_b_off, d_c, h_c_off, d_work, work_bytes, stream,
                               CAT_MODE_BATCHED);
}

cat_status bigint_residues(const uint32_t* d_x, size_t n, uint64_t* h_res, void* d_work, size_t work_bytes,
                           void* stream) {
  if (!h_res || (!d_x && n > 0)) return CAT_EINVAL;
  const uint64_t chunk = RES_BLOCK;
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (n == 0) {
    h_res[0] = h_res[1] = h_res[2] = 0;
    return CAT_OK;
  }
  if (!d_work || work_bytes < nch * 24 + 256) return CAT_ENOMEM;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  hipStream_t st = (hipStream_t)stream;
  uint64_t* part = (uint64_t*)d_work;
  // 5^256 mod (2^32 - 5): the weight of one step of a thread's Horner pass
  const uint32_t w256 = (uint32_t)h_powmod(5u, RES_T, (uint32_t)RES_Q0);
  {
    KTime kt("k_residues", st, (double)n);
    hipLaunchKernelGGL(k_residues, dim3((uint32_t)nch), dim3(RES_T), 0, st, d_x, (uint64_t)n, w256, part);
  }
  LAUNCHCHK();
  std::vector<uint64_t> h(nch * 3);
  HIPCHK(hipMemcpyAsync(h.data(), part, nch * 24, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const uint64_t mods[3] = {4294967291ull, 4294967297ull, 4294967295ull};
  for (int m = 0; m < 3; m++) {
    const uint64_t q = mods[m];
    // (2^32)^chunk mod q
    unsigned __int128 pw = 1, b = ((unsigned __int128)1 << 32) % q;
    for (uint64_t e = chunk; e; e >>= 1) {
      if (e & 1) pw = pw * b % q;
      b = b * b % q;
    }
    unsigned __int128 acc = 0;
    for (uint64_t c = nch; c > 0; c--) acc = (acc * pw + h[(c - 1) * 3 + m]) % q;
    h_res[m] = (uint64_t)acc;
  }
  return CAT_OK;
}

cat_status catalan_begin(uint64_t n, void* d_work, size_t work_bytes, void* stream, cat_ticket* ticket) {
  if (n > CAT_N_MAX || !d_work || !ticket) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  Ticket* t = nullptr;
  STCHK(ticket_alloc(&t));
  t->n = n;
  t->Ly = make_layout(n);
  if (work_bytes < t->Ly.total) {
    ticket_free(t);
    return CAT_ENOMEM;
  }
  t->wb = (char*)d_work;
  t->st = (hipStream_t)stream;
  uint64_t launches = 0;
  cat_status s = run_phase1(t->Ly, t->wb, (uint32_t*)t->wb + t->Ly.primes, t->Ly.Kmax, t->st, &launches);
  if (s == CAT_OK) {
    hipError_t e = hipMemcpyAsync(t->pin, t->wb + t->Ly.gtab, sizeof(GroupTable), hipMemcpyDeviceToHost, t->st);
    if (e == hipSuccess) e = hipEventRecord(t->ev, t->st);
    if (e != hipSuccess) {
      g.last_err = (int)e;
      s = CAT_EDEVICE;
    }
  }
  if (s != CAT_OK) {
    (void)hipStreamSynchronize(t->st);
    ticket_free(t);
    return s;
  }
  t->state = 1;
  *ticket = (cat_ticket)t;
  return CAT_OK;
}

cat_status cat_ticket_query(cat_ticket ticket) {
  if (!ticket) return CAT_EINVAL;
  Ticket* t = (Ticket*)ticket;
  hipError_t e = hipEventQuery(t->ev);
  if (e == hipSuccess) return CAT_OK;
  if (e == hipErrorNotReady) return CAT_EAGAIN;
  g.last_err = (int)e;
  return CAT_EDEVICE;
}

cat_status catalan_continue(cat_ticket ticket, uint32_t* d_limbs, size_t cap) {
  if (!ticket || !d_limbs) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  Ticket* t = (Ticket*)ticket;
  if (t->state != 1) return CAT_EINVAL;
  HIPCHK(hipEventSynchronize(t->ev));
  GroupTable gt;
  memcpy(&gt, t->pin, sizeof(GroupTable));
  if (gt.err || gt.ngroups > CAT_MAX_GROUPS) return CAT_EINTERNAL;
  Plan* P = find_plan(t->n, gt);
  if (!P) {
    STCHK(make_plan(t->Ly, gt, &P));
    remember_plan(P);
  }
  t->cap = cap;
  Exec X = make_exec(t->Ly, t->wb, t->st);
  unsigned long long* top = (unsigned long long*)(t->wb + t->Ly.top);
  if (P->result_is_one) {
    t->one = true;
    if (cap < 1) return CAT_ERANGE;
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, t->st, d_limbs, (uint64_t)1, 1u);
    LAUNCHCHK();
  } else {
    STCHK(run_phase2(X, *P, false));
    const uint32_t blocks = top_scan_blocks(P->result_cap);
    const uint64_t ncopy = std::min<uint64_t>(P->result_cap, cap);
    hipLaunchKernelGGL(k_top_nonzero, dim3(blocks), dim3(256), 0, t->st, X.W + P->result_pos, P->result_cap, top,
                       d_limbs, ncopy);
    LAUNCHCHK();
    // top and error word, adjacent in the control block
    HIPCHK(hipMemcpyAsync(t->pin + CTL_TOP, t->wb + t->Ly.top, 12, hipMemcpyDeviceToHost, t->st));
  }
  HIPCHK(hipEventRecord(t->ev, t->st));
  t->state = 2;
  return CAT_OK;
}

cat_status catalan_end(cat_ticket ticket, size_t* n_limbs) {
  if (!ticket) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  Ticket* t = (Ticket*)ticket;
  // the ticket is released on every path below: the caller never uses it again
  if (!n_limbs || t->state != 2) {
    (void)hipStreamSynchronize(t->st);
    ticket_free(t);
    return CAT_EINVAL;
  }
  hipError_t e = hipEventSynchronize(t->ev);
  if (e != hipSuccess) {
    g.last_err = (int)e;
    (void)hipStreamSynchronize(t->st);
    ticket_free(t);
    return CAT_EDEVICE;
  }
  cat_status s = CAT_OK;
  if (t->one) {
    *n_limbs = 1;
  } else {
    uint64_t L = 0;
    uint32_t derr = 0;
    memcpy(&L, t->pin + CTL_TOP, 8);
    memcpy(&derr, t->pin + CTL_ERR, 4);
    *n_limbs = (size_t)L;
    if (derr || L == 0) s = CAT_EINTERNAL;
    else if (L > t->cap) s = CAT_ERANGE;
  }
  ticket_free(t);
  return s;
}

cat_status cat_ticket_release(cat_ticket ticket) {
  if (!ticket) return CAT_OK;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  Ticket* t = (Ticket*)ticket;
  // everything the ticket queued (a failed catalan_continue may have queued
  // part of Phase 2 after the last event) has finished before d_work and
  // d_limbs go back to the caller
  (void)hipStreamSynchronize(t->st);
  ticket_free(t);
  return CAT_OK;
}

cat_status catalan_batch_sizes(uint32_t k, const uint64_t* ns, size_t* workspace_bytes) {
  if (!workspace_bytes || !ns || k == 0 || k > CAT_BATCH_MAX) return CAT_EINVAL;
  for (uint32_t r = 0; r < k; r++)
    if (ns[r] > CAT_N_MAX) return CAT_EINVAL;
  *workspace_bytes = make_batch_layout(k, ns).total;
  return CAT_OK;
}

cat_status catalan_batch_begin(uint32_t k, const uint64_t* ns, void* d_work, size_t work_bytes, void* stream,
                               cat_ticket* ticket) {
  if (!ns || !d_work || !ticket || k == 0 || k > CAT_BATCH_MAX) return CAT_EINVAL;
  for (uint32_t r = 0; r < k; r++)
    if (ns[r] > CAT_N_MAX) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  BatchLayout B = make_batch_layout(k, ns);
  if (work_bytes < B.total) return CAT_ENOMEM;
  char* pin = nullptr;
  if (!bpp.free_bufs.empty()) {
    pin = bpp.free_bufs.back();
    bpp.free_bufs.pop_back();
  } else {
    HIPCHK(hipHostMalloc((void**)&pin, BATCH_PIN, hipHostMallocDefault));
  }
  Ticket* t = nullptr;
  const cat_status ta = ticket_alloc(&t);
  if (ta != CAT_OK) {
    bpp.free_bufs.push_back(pin);
    return ta;
  }
  BatchState* b = new BatchState();
  b->B = B;
  b->pin = pin;
  b->status.assign(k, CAT_OK);
  t->batch = b;
  t->wb = (char*)d_work;
  t->st = (hipStream_t)stream;
  char* wb = t->wb;
  uint32_t* stage = (uint32_t*)(wb + B.c_off) + B.c.arenaA;
  uint64_t launches = 0;
  cat_status s = CAT_OK;
  for (uint32_t r = 0; r < k && s == CAT_OK; r++) {
    s = run_phase1(B.p1[r], wb + B.p1_off[r], stage + B.stage[r], B.kmax[r], t->st, &launches);
    if (s == CAT_OK) {
      const hipError_t e = hipMemcpyAsync(pin + bpin_gt(r), wb + B.p1_off[r] + B.p1[r].gtab, sizeof(GroupTable),
                                          hipMemcpyDeviceToHost, t->st);
      if (e != hipSuccess) {
        g.last_err = (int)e;
        s = CAT_EDEVICE;
      }
    }
  }
  if (s == CAT_OK) {
    const hipError_t e = hipEventRecord(t->ev, t->st);
    if (e != hipSuccess) {
      g.last_err = (int)e;
      s = CAT_EDEVICE;
    }
  }
  if (s != CAT_OK) {
    (void)hipStreamSynchronize(t->st);
    ticket_free(t);
    return s;
  }
  t->state = 1;
  *ticket = (cat_ticket)t;
  return CAT_OK;
}

cat_status catalan_batch_continue(cat_ticket ticket, uint32_t* const* d_limbs, const size_t* caps) {
  if (!ticket || !d_limbs || !caps) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  Ticket* t = (Ticket*)ticket;
  BatchState* b = t->batch;
  if (!b || t->state != 1) return CAT_EINVAL;
  const BatchLayout& B = b->B;
  const uint32_t k = B.k;
  for (uint32_t r = 0; r < k; r++)
    if (!d_limbs[r]) return CAT_EINVAL;
  HIPCHK(hipEventSynchronize(t->ev));
  std::vector<GroupTable> gts(k);
  for (uint32_t r = 0; r < k; r++) {
    memcpy(&gts[r], b->pin + bpin_gt(r), sizeof(GroupTable));
    if (gts[r].err || gts[r].ngroups > CAT_MAX_GROUPS) b->status[r] = CAT_EINTERNAL;
  }
  hipStream_t st = t->st;
  char* wb = t->wb;
  char* cw = wb + B.c_off;
  uint32_t* W = (uint32_t*)cw;
  // the primes of all requests side by side (request order)
  std::vector<uint64_t> q(k, 0);
  MoveList ml{};
  uint64_t qn = 0, lmax = 0;
  for (uint32_t r = 0; r < k; r++) {
    if (b->status[r] != CAT_OK) continue;
    const uint64_t np = gts[r].off[gts[r].ngroups];
    q[r] = qn;
    if (np) {
      ml.src[ml.n] = B.stage[r];
      ml.dst[ml.n] = qn;
      ml.len[ml.n] = np;
      ml.n++;
      lmax = std::max(lmax, np);
    }
    qn += np;
  }
  if (ml.n) {
    hipLaunchKernelGGL(k_move_ranges, dim3((uint32_t)std::min<uint64_t>((lmax + 255) / 256, 1024), ml.n), dim3(256),
                       0, st, ml, (const uint32_t*)(W + B.c.arenaA), W + B.c.primes);
    LAUNCHCHK();
  }
  // control block (look-back flags, error word) and the top indices cleared
  unsigned long long* tops = (unsigned long long*)(wb + B.tops_off);
  hipLaunchKernelGGL(k_fill, dim3((uint32_t)std::min<uint64_t>((B.c.ctl_words + 255) / 256, 1024)), dim3(256), 0, st,
                     (uint32_t*)(cw + B.c.gtab), (uint64_t)B.c.ctl_words, 0u);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, (uint32_t*)tops, (uint64_t)(2 * k), 0u);
  LAUNCHCHK();
  // chunks of whole requests with at most CAT_MAX_GROUPS groups each
  uint32_t epoch = 0;
  uint32_t r0 = 0;
  while (r0 < k) {
    uint32_t r1 = r0, ng = 0;
    while (r1 < k && (b->status[r1] != CAT_OK || ng + gts[r1].ngroups <= CAT_MAX_GROUPS)) {
      if (b->status[r1] == CAT_OK) ng += gts[r1].ngroups;
      r1++;
    }
    GroupTable gtc{};
    uint32_t req[CAT_MAX_GROUPS] = {};
    std::vector<uint32_t> members;
    for (uint32_t r = r0; r < r1; r++) {
      if (b->status[r] != CAT_OK) continue;
      const uint32_t i = (uint32_t)members.size();
      members.push_back(r);
      for (uint32_t gg = 0; gg < gts[r].ngroups; gg++) {
        gtc.exps[gtc.ngroups] = gts[r].exps[gg];
        gtc.off[gtc.ngroups] = q[r] + gts[r].off[gg];
        gtc.gbits[gtc.ngroups] = gts[r].gbits[gg];
        req[gtc.ngroups] = i;
        gtc.ngroups++;
      }
      gtc.off[gtc.ngroups] = q[r] + gts[r].off[gts[r].ngroups];
    }
    Plan* P = nullptr;
    if (gtc.ngroups) {
      // no device tables: the plan is freed as soon as its launches are queued
      STCHK(make_plan(B.c, gtc, &P, false, req, (uint32_t)members.size()));
      Exec X = make_exec(B.c, cw, st);
      X.crt_epoch = epoch;
      const cat_status rs = run_phase2(X, *P, false);
      epoch = X.crt_epoch;
      if (rs != CAT_OK) {
        free_plan(P);
        return rs;
      }
    }
    for (uint32_t i = 0; i < (uint32_t)members.size(); i++) {
      const uint32_t r = members[i];
      if (!P || P->rone[i]) {
        // C(n) = 1
        if (caps[r] >= 1) hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, d_limbs[r], (uint64_t)1, 1u);
        hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, (uint32_t*)(tops + r), (uint64_t)1, 1u);
      } else {
        hipLaunchKernelGGL(k_top_nonzero, dim3(top_scan_blocks(P->rcap[i])), dim3(256), 0, st, W + P->rpos[i],
                           P->rcap[i], tops + r, d_limbs[r], std::min<uint64_t>(P->rcap[i], caps[r]));
      }
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) {
        if (P) free_plan(P);
        g.last_err = (int)e;
        return CAT_EDEVICE;
      }
    }
    if (P) free_plan(P);
    r0 = r1;
  }
  HIPCHK(hipMemcpyAsync(b->pin + bpin_tops(), tops, 8 * (size_t)k, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(b->pin + bpin_err(), cw + B.c.err, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipEventRecord(t->ev, st));
  b->cap.assign(caps, caps + k);
  t->state = 2;
  return CAT_OK;
}

cat_status catalan_batch_end(cat_ticket ticket, size_t* n_limbs, cat_status* req_status) {
  if (!ticket) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  Ticket* t = (Ticket*)ticket;
  BatchState* b = t->batch;
  // the ticket is released on every path below
  if (!b || !n_limbs || t->state != 2) {
    (void)hipStreamSynchronize(t->st);
    ticket_free(t);
    return CAT_EINVAL;
  }
  hipError_t e = hipEventSynchronize(t->ev);
  if (e != hipSuccess) {
    g.last_err = (int)e;
    (void)hipStreamSynchronize(t->st);
    ticket_free(t);
    return CAT_EDEVICE;
  }
  uint32_t derr = 0;
  memcpy(&derr, b->pin + bpin_err(), 4);
  cat_status first = CAT_OK;
  for (uint32_t r = 0; r < b->B.k; r++) {
    uint64_t L = 0;
    memcpy(&L, b->pin + bpin_tops() + 8 * (size_t)r, 8);
    cat_status s = b->status[r];
    n_limbs[r] = s == CAT_OK ? (size_t)L : 0;
    if (s == CAT_OK) {
      if (derr || L == 0) s = CAT_EINTERNAL;
      else if (L > b->cap[r]) s = CAT_ERANGE;
    }
    if (req_status) req_status[r] = s;
    if (first == CAT_OK) first = s;
  }
  ticket_free(t);
  return first;
}

cat_status catalan_exact_noalloc(uint64_t n, uint32_t* d_limbs, size_t cap, size_t* n_limbs, void* stream) {
  if (n > CAT_N_MAX || !n_limbs || !d_limbs) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  const Layout Ly = make_layout(n);
  if (Ly.total > CAT_NOALLOC_BYTES) return CAT_ENOMEM;   // beyond the static scratch
  if (!g.scratch_ptr) return CAT_EINTERNAL;
  g.in_noalloc = true;
  const cat_status s = exact_in_workspace(n, Ly, (char*)g.scratch_ptr, d_limbs, cap, n_limbs, (hipStream_t)stream,
                                          false, false, true, 0);
  g.in_noalloc = false;
  return s;
}

cat_status catalan_noalloc_max_bytes(size_t* bytes) {
  if (!bytes) return CAT_EINVAL;
  *bytes = CAT_NOALLOC_BYTES;
  return CAT_OK;
}

cat_status catalan_exact(uint64_t n, uint32_t* d_limbs, size_t cap, size_t* n_limbs, void* d_work, size_t work_bytes,
                         void* stream) {
  return catalan_exact_ex(n, d_limbs, cap, n_limbs, d_work, work_bytes, stream, CAT_MODE_BATCHED | CAT_MODE_GRAPH);
}

cat_status factorial_ratio_sizes(const uint64_t* a, uint32_t k, const uint64_t* b, uint32_t m, size_t* max_primes,
                                 size_t* max_limbs, size_t* workspace_bytes) {
  RatioSpec r;
  STCHK(ratio_spec(a, k, b, m, &r));
  const Layout Ly = make_layout_ratio(r);
  if (max_primes) *max_primes = (size_t)Ly.Kmax;
  if (max_limbs) *max_limbs = (size_t)ratio_limbs_bound(r);
  if (workspace_bytes) *workspace_bytes = Ly.total;
  return CAT_OK;
}

cat_status factorial_ratio_factor(const uint64_t* a, uint32_t k, const uint64_t* b, uint32_t m, uint32_t* d_primes,
                                  size_t primes_cap, uint32_t* h_exps, uint64_t* h_off, uint32_t* n_groups,
                                  size_t* n_primes, void* d_work, size_t work_bytes, void* stream) {
  if (!h_exps || !h_off || !n_groups || !n_primes || !d_work) return CAT_EINVAL;
  if (!d_primes && primes_cap > 0) return CAT_EINVAL;
  RatioSpec r;
  STCHK(ratio_spec(a, k, b, m, &r));
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  const Layout Ly = make_layout_ratio(r);
  if (work_bytes < Ly.total) return CAT_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  uint64_t launches = 0;
  uint32_t dummy = 0;
  STCHK(run_phase1_ratio(Ly, r, (char*)d_work, d_primes ? d_primes : &dummy, d_primes ? primes_cap : 0, st,
                         &launches));
  GroupTable gt;
  const cat_status e = read_groups_ratio(Ly, (char*)d_work, st, &gt);
  if (e != CAT_OK && !(e == CAT_EINTERNAL && (gt.err & CAT_DEVERR_BOUNDS))) return e;
  *n_groups = gt.ngroups;
  for (uint32_t q = 0; q < gt.ngroups; q++) h_exps[q] = gt.exps[q];
  for (uint32_t q = 0; q <= gt.ngroups; q++) h_off[q] = gt.off[q];
  *n_primes = (size_t)gt.off[gt.ngroups];
  g.stats = cat_stats{};
  g.stats.launches = launches;
  g.stats.n_primes = *n_primes;
  if (*n_primes > primes_cap) return CAT_ERANGE;
  return CAT_OK;
}

cat_status factorial_ratio_exact(const uint64_t* a, uint32_t k, const uint64_t* b, uint32_t m, uint32_t* d_limbs,
                                 size_t cap, size_t* n_limbs, void* d_work, size_t work_bytes, void* stream,
                                 uint32_t flags) {
  if (!n_limbs) return CAT_EINVAL;
  RatioSpec r;
  STCHK(ratio_spec(a, k, b, m, &r));
  if (!d_limbs) {
    *n_limbs = (size_t)ratio_limbs_bound(r);
    return CAT_OK;
  }
  if (!d_work) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  const Layout Ly = make_layout_ratio(r);
  if (work_bytes < Ly.total) return CAT_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  char* wb = (char*)d_work;
  const bool plain = (flags & CAT_MODE_PLAIN) != 0;
  uint64_t launches = 0;
  STCHK(run_phase1_ratio(Ly, r, wb, (uint32_t*)wb + Ly.primes, Ly.Kmax, st, &launches));
  GroupTable gt;
  STCHK(read_groups_ratio(Ly, wb, st, &gt));
  Plan* P = nullptr;
  STCHK(make_plan(Ly, gt, &P));
  cat_status res = CAT_OK;
  if (P->result_is_one) {
    if (cap < 1) {
      *n_limbs = 1;
      res = CAT_ERANGE;
    } else {
      hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, d_limbs, (uint64_t)1, 1u);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        g.last_err = (int)e;
        res = CAT_EDEVICE;
      }
      *n_limbs = 1;
    }
    free_plan(P);
    return res;
  }
  Exec X = make_exec(Ly, wb, st);
  unsigned long long* top = (unsigned long long*)(wb + Ly.top);
  res = run_phase2(X, *P, plain);
  if (res == CAT_OK) {
    const uint32_t blocks = top_scan_blocks(P->result_cap);
    const uint64_t ncopy = std::min<uint64_t>(P->result_cap, cap);
    hipLaunchKernelGGL(k_top_nonzero, dim3(blocks), dim3(256), 0, st, X.W + P->result_pos, P->result_cap, top, d_limbs,
                       ncopy);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(g.pin, wb + Ly.top, 12, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      g.last_err = (int)e;
      res = CAT_EDEVICE;
    }
  }
  cat_stats stats{};
  stats.products = P->products;
  stats.product_limbs = P->product_limbs;
  stats.launches = launches + X.launches + 1;
  stats.n_primes = gt.off[gt.ngroups];
  stats.levels = P->levels;
  stats.outer_level = P->rins_j;
  free_plan(P);
  g.stats = stats;
  if (res != CAT_OK) return res;
  uint64_t L = 0;
  uint32_t derr = 0;
  memcpy(&L, g.pin, 8);
  memcpy(&derr, (char*)g.pin + 8, 4);
  if (derr || L == 0) return CAT_EINTERNAL;
  *n_limbs = (size_t)L;
  if (cap < L) return CAT_ERANGE;
  return CAT_OK;
}

cat_status prime_power_product_sizes(const uint32_t* h_exps, const uint64_t* h_off, uint32_t ngroups,
                                     uint32_t max_entry_bits, size_t* max_limbs, size_t* workspace_bytes) {
  GroupsIn G;
  STCHK(groups_in(h_exps, h_off, ngroups, max_entry_bits, &G));
  if (G.lbits > 32.0 * (double)((1ull << CAT_MAX_LOGN) - 64)) return CAT_ERANGE;
  const Layout Ly = make_layout_groups(G);
  if (max_limbs) *max_limbs = (size_t)(G.lbits / 32.0) + 2;
  if (workspace_bytes) *workspace_bytes = Ly.total;
  return CAT_OK;
}

cat_status prime_power_product(const uint32_t* d_entries, const uint32_t* h_exps, const uint64_t* h_off,
                               uint32_t ngroups, uint32_t max_entry_bits, uint32_t* d_limbs, size_t cap,
                               size_t* n_limbs, void* d_work, size_t work_bytes, void* stream, uint32_t flags) {
  if (!n_limbs || !d_limbs || !d_work) return CAT_EINVAL;
  GroupsIn G;
  STCHK(groups_in(h_exps, h_off, ngroups, max_entry_bits, &G));
  if (G.lbits > 32.0 * (double)((1ull << CAT_MAX_LOGN) - 64)) return CAT_ERANGE;
  if (G.total && !d_entries) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  const Layout Ly = make_layout_groups(G);
  if (work_bytes < Ly.total) return CAT_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  char* wb = (char*)d_work;
  uint32_t* W = (uint32_t*)wb;
  // control block cleared; entries into the tree's leaf buffer, group offsets
  // and the bit sums in the seed buffer (unused here)
  hipLaunchKernelGGL(k_fill, dim3((uint32_t)std::min<uint64_t>((Ly.ctl_words + 255) / 256, 1024)), dim3(256), 0, st,
                     (uint32_t*)(wb + Ly.gtab), (uint64_t)Ly.ctl_words, 0u);
  LAUNCHCHK();
  if (G.total) HIPCHK(hipMemcpyAsync(W + Ly.primes, d_entries, G.total * 4, hipMemcpyDeviceToDevice, st));
  uint64_t* d_off = (uint64_t*)(W + Ly.seeds);
  unsigned long long* d_bits = (unsigned long long*)(d_off + CAT_MAX_GROUPS + 2);
  memcpy(g.pin, G.off, sizeof(uint64_t) * (G.ng + 1));
  HIPCHK(hipMemcpyAsync(d_off, g.pin, sizeof(uint64_t) * (G.ng + 1), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, (uint32_t*)d_bits, (uint64_t)(2 * CAT_MAX_GROUPS), 0u);
  LAUNCHCHK();
  if (G.ng) {
    // enough workgroups per group to keep HBM busy on the largest group
    hipLaunchKernelGGL(k_group_bits, dim3(2048, G.ng), dim3(256), 0, st, (const uint32_t*)(W + Ly.primes),
                       (const uint64_t*)d_off, G.ng, d_bits);
    LAUNCHCHK();
  }
  HIPCHK(hipMemcpyAsync((char*)g.pin + 1024, d_bits, sizeof(uint64_t) * CAT_MAX_GROUPS, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  GroupTable gt;
  memset(&gt, 0, sizeof(gt));
  gt.ngroups = G.ng;
  double lb = 0;
  for (uint32_t q = 0; q < G.ng; q++) {
    gt.exps[q] = G.exps[q];
    gt.off[q] = G.off[q];
    memcpy(&gt.gbits[q], (char*)g.pin + 1024 + 8 * q, 8);
    if (gt.gbits[q] > (G.off[q + 1] - G.off[q]) * (uint64_t)max_entry_bits) return CAT_EINVAL;
    lb += (double)G.exps[q] * (double)gt.gbits[q];
  }
  gt.off[G.ng] = G.off[G.ng];
  if (lb > 32.0 * (double)((1ull << CAT_MAX_LOGN) - 64)) return CAT_ERANGE;
  Plan* P = nullptr;
  STCHK(make_plan(Ly, gt, &P));
  cat_status res = CAT_OK;
  if (P->result_is_one) {
    free_plan(P);
    if (cap < 1) {
      *n_limbs = 1;
      return CAT_ERANGE;
    }
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, d_limbs, (uint64_t)1, 1u);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(st));
    *n_limbs = 1;
    return CAT_OK;
  }
  Exec X = make_exec(Ly, wb, st);
  unsigned long long* top = (unsigned long long*)(wb + Ly.top);
  res = run_phase2(X, *P, (flags & CAT_MODE_PLAIN) != 0);
  if (res == CAT_OK) {
    const uint32_t blocks = top_scan_blocks(P->result_cap);
    const uint64_t ncopy = std::min<uint64_t>(P->result_cap, cap);
    hipLaunchKernelGGL(k_top_nonzero, dim3(blocks), dim3(256), 0, st, X.W + P->result_pos, P->result_cap, top, d_limbs,
                       ncopy);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(g.pin, wb + Ly.top, 12, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      g.last_err = (int)e;
      res = CAT_EDEVICE;
    }
  }
  cat_stats stats{};
  stats.products = P->products;
  stats.product_limbs = P->product_limbs;
  stats.launches = X.launches + 4;
  stats.n_primes = G.total;
  stats.levels = P->levels;
  stats.outer_level = P->rins_j;
  free_plan(P);
  g.stats = stats;
  if (res != CAT_OK) return res;
  uint64_t L = 0;
  uint32_t derr = 0;
  memcpy(&L, g.pin, 8);
  memcpy(&derr, (char*)g.pin + 8, 4);
  if (derr || L == 0) return CAT_EINTERNAL;
  *n_limbs = (size_t)L;
  if (cap < L) return CAT_ERANGE;
  return CAT_OK;
}

cat_status bigint_compare(const uint32_t* d_x, size_t lx, uint64_t shift_bits, const uint32_t* d_y, size_t ly,
                          int32_t* sign, void* d_work, size_t work_bytes, void* stream) {
  if (!sign || !d_work || work_bytes < 16 || (lx && !d_x) || (ly && !d_y)) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  hipStream_t st = (hipStream_t)stream;
  unsigned long long* top = (unsigned long long*)d_work;
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, (uint32_t*)top, (uint64_t)2, 0u);
  LAUNCHCHK();
  const uint64_t lxs = (uint64_t)lx > (shift_bits >> 5) ? (uint64_t)lx - (shift_bits >> 5) : 0;   // limbs of x >> s
  const uint64_t n = std::max<uint64_t>(lxs, ly);
  if (n) {
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_diff_top, dim3(blocks), dim3(256), 0, st, d_x, (uint64_t)lx, shift_bits, d_y, (uint64_t)ly, n,
                       top);
    LAUNCHCHK();
  }
  HIPCHK(hipMemcpyAsync(g.pin, top, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  uint64_t t = 0;
  memcpy(&t, g.pin, 8);
  if (t == 0) {
    *sign = 0;
    return CAT_OK;
  }
  // the differing limb of x >> s (one or two source limbs) and of y
  const uint64_t k = t - 1, w = k + (shift_bits >> 5);
  const uint32_t r = (uint32_t)(shift_bits & 31);
  uint32_t x2[2] = {0, 0}, b = 0;
  if (w < lx) HIPCHK(hipMemcpyAsync((char*)g.pin + 16, d_x + w, 4, hipMemcpyDeviceToHost, st));
  if (w + 1 < lx) HIPCHK(hipMemcpyAsync((char*)g.pin + 20, d_x + w + 1, 4, hipMemcpyDeviceToHost, st));
  if (k < ly) HIPCHK(hipMemcpyAsync((char*)g.pin + 24, d_y + k, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (w < lx) memcpy(&x2[0], (char*)g.pin + 16, 4);
  if (w + 1 < lx) memcpy(&x2[1], (char*)g.pin + 20, 4);
  if (k < ly) memcpy(&b, (char*)g.pin + 24, 4);
  const uint32_t a = r ? ((x2[0] >> r) | (x2[1] << (32 - r))) : x2[0];
  *sign = a > b ? 1 : -1;
  return CAT_OK;
}

// ----------------------------------------------------------------------------
// Exact decimal digit count (Table 1's 1,234,567,890 digits): d is the count
// of x > 0 exactly when 10^(d-1) <= x < 10^d, checked on the device as
// floor(x / 2^(d-1)) >= 5^(d-1) and floor(x / 2^d) < 5^d; the powers of five
// come from the Phase-2 engine ((5^13)^q * 5^r), the first guess of d from
// the top limbs in double precision, corrected by at most a few steps.
// ----------------------------------------------------------------------------
#define DD_HEAD 512   // entries (two words) and the comparison scratch
static const uint32_t kPow5_13 = 1220703125u;   // 5^13 < 2^31

// groups of 5^k for the product engine: exponent 1 on [5^r] and q on [5^13]
static uint32_t pow5_groups(uint64_t k, uint32_t* exps, uint64_t* off, uint32_t* ent) {
  const uint64_t q = k / 13, r = k % 13;
  uint32_t p5r = 1;
  for (uint64_t i = 0; i < r; i++) p5r *= 5u;
  if (q <= 1) {
    exps[0] = 1;
    off[0] = 0;
    off[1] = q ? 2 : 1;
    ent[0] = p5r;
    ent[1] = kPow5_13;
    return 1;
  }
  exps[0] = 1;
  exps[1] = (uint32_t)q;
  off[0] = 0;
  off[1] = 1;
  off[2] = 2;
  ent[0] = p5r;
  ent[1] = kPow5_13;
  return 2;
}

static uint64_t dd_max_digits(size_t n_limbs) { return (uint64_t)(32.0 * (double)n_limbs * 0.30102999566398120) + 2; }

// limbs and product-engine workspace for 5^k, k <= kmax
static cat_status dd_sizes(uint64_t kmax, size_t* p5_limbs, size_t* ppp_bytes) {
  uint32_t exps[2], ent[2];
  uint64_t off[3];
  const uint32_t ng = pow5_groups(kmax, exps, off, ent);
  size_t ml = 0, wb = 0;
  STCHK(prime_power_product_sizes(exps, off, ng, 31, &ml, &wb));
  *p5_limbs = std::max<size_t>(ml, 2);
  *ppp_bytes = wb;
  return CAT_OK;
}

cat_status bigint_decimal_digits_workspace(size_t n_limbs, size_t* workspace_bytes) {
  if (!workspace_bytes) return CAT_EINVAL;
  if (n_limbs > (1ull << CAT_MAX_LOGN)) return CAT_EINVAL;
  size_t pl = 0, pw = 0;
  STCHK(dd_sizes(dd_max_digits(n_limbs), &pl, &pw));
  *workspace_bytes = DD_HEAD + align_up(pl * 4, 256) + pw;
  return CAT_OK;
}

cat_status bigint_decimal_digits(const uint32_t* d_x, size_t n_limbs, uint64_t* digits, void* d_work,
                                 size_t work_bytes, void* stream) {
  if (!digits || !d_work || (n_limbs && !d_x) || n_limbs > (1ull << CAT_MAX_LOGN)) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  size_t need = 0;
  STCHK(bigint_decimal_digits_workspace(n_limbs, &need));
  if (work_bytes < need) return CAT_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  char* wb = (char*)d_work;
  unsigned long long* top = (unsigned long long*)(wb + 256);
  // the highest nonzero limb
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, (uint32_t*)top, (uint64_t)2, 0u);
  LAUNCHCHK();
  if (n_limbs) {
    hipLaunchKernelGGL(k_top_nonzero, dim3(top_scan_blocks(n_limbs)), dim3(256), 0, st, d_x, (uint64_t)n_limbs, top,
                       (uint32_t*)nullptr, (uint64_t)0);
    LAUNCHCHK();
  }
  HIPCHK(hipMemcpyAsync(g.pin, top, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  uint64_t L = 0;
  memcpy(&L, g.pin, 8);
  if (L == 0) {   // x = 0 has one digit
    *digits = 1;
    return CAT_OK;
  }
  const uint64_t k0 = L > 3 ? L - 3 : 0;
  HIPCHK(hipMemcpyAsync(g.pin, d_x + k0, (L - k0) * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  uint32_t tl[3] = {0, 0, 0};
  memcpy(tl, g.pin, (L - k0) * 4);
  double topv = 0;
  for (uint64_t k = L; k > k0; k--) topv = topv * 4294967296.0 + (double)tl[k - 1 - k0];
  int64_t d = (int64_t)std::floor(std::log10(topv) + 32.0 * (double)k0 * 0.30102999566398120) + 1;
  size_t pl = 0, pw = 0;
  STCHK(dd_sizes(dd_max_digits(n_limbs), &pl, &pw));
  uint32_t* d_ent = (uint32_t*)wb;
  uint32_t* d_y = (uint32_t*)(wb + DD_HEAD);
  void* ppp = wb + DD_HEAD + align_up(pl * 4, 256);
  // sign(floor(x / 2^k) - 5^k)
  auto cmp_pow5 = [&](uint64_t k, int32_t* sgn) -> cat_status {
    uint32_t exps[2], ent[2];
    uint64_t off[3];
    const uint32_t ng = pow5_groups(k, exps, off, ent);
    memcpy((char*)g.pin + 2048, ent, 8);
    HIPCHK(hipMemcpyAsync(d_ent, (char*)g.pin + 2048, 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    size_t ly = 0;
    STCHK(prime_power_product(d_ent, exps, off, ng, 31, d_y, pl, &ly, ppp, pw, stream, CAT_MODE_BATCHED));
    return bigint_compare(d_x, L, k, d_y, ly, sgn, wb + 256, 256, stream);
  };
  for (int it = 0; it < 6; it++) {
    if (d < 1) d = 1;
    int32_t s1 = 0, s2 = 0;
    STCHK(cmp_pow5((uint64_t)(d - 1), &s1));
    if (s1 < 0) {   // x < 10^(d-1)
      d--;
      continue;
    }
    STCHK(cmp_pow5((uint64_t)d, &s2));
    if (s2 >= 0) {  // x >= 10^d
      d++;
      continue;
    }
    *digits = (uint64_t)d;
    return CAT_OK;
  }
  return CAT_EINTERNAL;
}

}  // extern "C"
