// Issue rates of single VALU instruction forms (measurement only).
//
// The butterfly peak the transforms are measured against counts lane
// operations, so it rests on how fast the integer forms the butterflies are
// made of issue.  Each probe thread runs RATE_CHAINS independent dependency
// chains of one instruction (written as inline assembly, so the form is
// exactly the one named and nothing is folded), RATE_UNROLL times per loop
// trip; 8 workgroups of 4 waves per compute unit keep 8 waves on every SIMD,
// which hides each chain's latency.  The chain values are folded into one
// store per thread so that they stay live.

#define RATE_CHAINS 8
#define RATE_UNROLL 4
#define RATE_THREADS 256
#define RATE_WG_PER_CU 8

template <int OP>
__global__ void __launch_bounds__(RATE_THREADS) k_valu_rate(uint32_t iters, uint32_t seed, uint32_t* __restrict__ out) {
  uint32_t r[RATE_CHAINS];
  uint64_t w[RATE_CHAINS];
  float f[RATE_CHAINS];
  const uint32_t gid = blockIdx.x * RATE_THREADS + threadIdx.x;
  const uint32_t y = seed | 1u;
  const float fy = 1.0f + (float)(seed & 255u) * 0x1p-20f;
#pragma unroll
  for (int i = 0; i < RATE_CHAINS; i++) {
    r[i] = gid * 0x9E3779B9u + (uint32_t)i;
    w[i] = r[i];
    f[i] = (float)(r[i] & 1023u);
  }
  for (uint32_t it = 0; it < iters; it++) {
#pragma unroll
    for (int u = 0; u < RATE_UNROLL; u++) {
#pragma unroll
      for (int i = 0; i < RATE_CHAINS; i++) {
        if constexpr (OP == 0) {
          asm volatile("v_add_u32 %0, %0, %1" : "+v"(r[i]) : "v"(y));
        } else if constexpr (OP == 1) {
          asm volatile("v_min_u32 %0, %0, %1" : "+v"(r[i]) : "v"(y));
        } else if constexpr (OP == 2) {
          asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(r[i]) : "v"(y));
        } else if constexpr (OP == 3) {
          asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(r[i]) : "v"(y));
        } else if constexpr (OP == 4) {
          uint64_t c;  // carry out (unused)
          asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(w[i]), "=s"(c) : "v"(r[i]), "v"(y));
        } else {
          asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(f[i]) : "v"(fy));
        }
      }
    }
  }
  uint32_t acc = 0;
#pragma unroll
  for (int i = 0; i < RATE_CHAINS; i++) acc ^= r[i] ^ (uint32_t)w[i] ^ (uint32_t)(w[i] >> 32) ^ __float_as_uint(f[i]);
  out[gid] = acc;
}

extern "C" cat_status cat_valu_rate(int op, uint32_t iters, double* lane_ops_per_s, double* ms) {
  if (!lane_ops_per_s || op < 0 || op >= CAT_VALU_NOPS || iters == 0 || iters > (1u << 20)) return CAT_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(g.mu);
  STCHK(init_locked(-1));
  STCHK(set_device());
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const uint32_t blocks = (uint32_t)cus * RATE_WG_PER_CU;
  uint32_t* d_out = nullptr;
  HIPCHK(hipMalloc((void**)&d_out, (size_t)blocks * RATE_THREADS * sizeof(uint32_t)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  auto launch = [&](uint32_t n) {
    switch (op) {
      case 0: hipLaunchKernelGGL(k_valu_rate<0>, dim3(blocks), dim3(RATE_THREADS), 0, 0, n, 12345u, d_out); break;
      case 1: hipLaunchKernelGGL(k_valu_rate<1>, dim3(blocks), dim3(RATE_THREADS), 0, 0, n, 12345u, d_out); break;
      case 2: hipLaunchKernelGGL(k_valu_rate<2>, dim3(blocks), dim3(RATE_THREADS), 0, 0, n, 12345u, d_out); break;
      case 3: hipLaunchKernelGGL(k_valu_rate<3>, dim3(blocks), dim3(RATE_THREADS), 0, 0, n, 12345u, d_out); break;
      case 4: hipLaunchKernelGGL(k_valu_rate<4>, dim3(blocks), dim3(RATE_THREADS), 0, 0, n, 12345u, d_out); break;
      default: hipLaunchKernelGGL(k_valu_rate<5>, dim3(blocks), dim3(RATE_THREADS), 0, 0, n, 12345u, d_out); break;
    }
    return hipGetLastError();
  };
  float t = 0;
  if (err == hipSuccess) err = launch(iters);  // warm-up (clocks, code load)
  if (err == hipSuccess) err = hipEventRecord(e0, 0);
  if (err == hipSuccess) err = launch(iters);
  if (err == hipSuccess) err = hipEventRecord(e1, 0);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(d_out);
  HIPCHK(err);
  const double lane_ops = (double)blocks * RATE_THREADS * iters * RATE_UNROLL * RATE_CHAINS;
  *lane_ops_per_s = t > 0 ? lane_ops / (t * 1e-3) : 0.0;
  if (ms) *ms = t;
  return CAT_OK;
}
