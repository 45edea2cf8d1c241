// Fused kernels of the GCN layer executor.
//
// k_comb_fused computes, for every output column l < F' of one group,
//   H_l = sum_f w_{l,f} * z_f,   z_f = sum_k P_k (.) X_{k*F + f}   (Inter-CA, K > 0)
//                                z_f = X_f                          (combination only, K = 0)
// in one pass over the inputs: a thread owns one coefficient j of one limb of
// one component, so every input word is read exactly once (coalesced), z_f is
// reduced once, and the F' products w * z accumulate lazily in 128 bits
// (folded every 64 terms, safe for primes below 2^61).  This is the Inter-CA
// aggregation (Sec. 3.3.2) and the t = 1 combination (App. B) of one layer
// without writing the intermediate z_f.
#include "internal.h"

namespace ficgcn {

constexpr int FB = 256;

template <int FO>
__global__ __launch_bounds__(FB) void k_comb_fused(uint64_t* const* __restrict__ out, const uint64_t* const* __restrict__ in,
                                                   const uint64_t* const* __restrict__ pts, int K, int F, int l_first,
                                                   int n_out, int l1, const uint64_t* __restrict__ w, int log_n,
                                                   const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)FB + threadIdx.x;
  const int i = blockIdx.y, c = blockIdx.z;
  const Mod m = mods[i];
  const size_t off = ((size_t)c * l1 + i) * N + j;
  uint64_t p[16];
  for (int k = 0; k < K; ++k) p[k] = pts[k][(size_t)i * N + j];
  u128 acc[FO];
#pragma unroll
  for (int l = 0; l < FO; ++l) acc[l] = 0;
  for (int f = 0; f < F; ++f) {
    uint64_t z;
    if (K > 0) {
      u128 s = 0;
      for (int k = 0; k < K; ++k) s += (u128)p[k] * in[(size_t)k * F + f][off];
      z = reduce128(s, m);
    } else {
      z = in[f][off];
    }
    // w layout: [F'][F][l1] residues
#pragma unroll
    for (int l = 0; l < FO; ++l)
      if (l < n_out) acc[l] += (u128)z * w[(((size_t)(l_first + l)) * F + f) * l1 + i];
    if ((f & 63) == 63) {
#pragma unroll
      for (int l = 0; l < FO; ++l) acc[l] = reduce128(acc[l], m);
    }
  }
#pragma unroll
  for (int l = 0; l < FO; ++l)
    if (l < n_out) out[l_first + l][off] = reduce128(acc[l], m);
}

void comb_fused(ckks_ctx* c, uint64_t* const* out_dev_ptrs, const uint64_t* const* in_dev_ptrs,
                const uint64_t* const* pt_dev_ptrs, int K, int F, int F_out, int level, const uint64_t* w_dev,
                const char* prof_name) {
  ProfScope ps(c, prof_name);
  if (K > 16) FICGCN_THROW(EPLAN_, "more than 16 Inter-CA copies per fused launch");
  const int l1 = level + 1;
  for (int l0 = 0; l0 < F_out; l0 += 16) {
    int n = std::min(16, F_out - l0);
    dim3 grid(c->N / FB, l1, 2);
    if (n <= 8)
      hipLaunchKernelGGL(k_comb_fused<8>, grid, dim3(FB), 0, c->stream, out_dev_ptrs, in_dev_ptrs, pt_dev_ptrs, K, F,
                         l0, n, l1, w_dev, c->log_n, c->t.mods);
    else
      hipLaunchKernelGGL(k_comb_fused<16>, grid, dim3(FB), 0, c->stream, out_dev_ptrs, in_dev_ptrs, pt_dev_ptrs, K, F,
                         l0, n, l1, w_dev, c->log_n, c->t.mods);
    HIPCHECK(hipGetLastError());
  }
}

__global__ void k_zero(uint64_t* __restrict__ p, size_t n) {
  size_t i = blockIdx.x * (size_t)FB + threadIdx.x;
  if (i < n) p[i] = 0;
}

void zero_fill(ckks_ctx* c, uint64_t* p, size_t words) {
  if (!words) return;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((words + FB - 1) / FB)), dim3(FB), 0, c->stream, p, words);
  HIPCHECK(hipGetLastError());
}

}  // namespace ficgcn
