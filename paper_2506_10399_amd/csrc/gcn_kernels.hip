// Fused kernels of the GCN layer executor.
//
// The fused pass computes, for every output column l < F' of one group,
//   H_l = sum_f w_{l,f} * z_f,   z_f = sum_k P_k (.) X_{k*F + f}   (Inter-CA, K > 0)
//                                z_f = X_f                          (combination only, K = 0)
// in one pass over the inputs: a thread owns one coefficient j of one limb of
// one component, so every input word is read exactly once (coalesced), z_f is
// reduced once, and the products w * z accumulate lazily.  This is the
// Inter-CA aggregation (Sec. 3.3.2) and the one-column-per-ciphertext
// combination (App. B) of one layer without writing the intermediate z_f.
//
// Arithmetic (primes below 2^52): every operand a < 2^52 is split into 26-bit
// halves a = a1 2^26 + a0, so a partial product fits one 32x32+64 multiply-add
// and a * b = a0 b0 + (a0 b1 + a1 b0) 2^26 + a1 b1 2^52 accumulates in three
// 64-bit registers without carries: each term is below 2^53, so 2^10 terms
// per register are safe; the three are folded to one residue every 1024
// features.  Primes of 52 bits or more use the 128-bit accumulation variant.
#include "internal.h"

namespace ficgcn {

constexpr int FB = 256;
constexpr uint64_t M26 = (1ull << 26) - 1;

__device__ __forceinline__ uint64_t mad32(uint32_t a, uint32_t b, uint64_t c) { return (uint64_t)a * b + c; }

// value of a0 + a1 2^26 + a2 2^52 mod q
__device__ __forceinline__ uint64_t fold3(uint64_t a0, uint64_t a1, uint64_t a2, const Mod& m) {
  u128 v = (u128)a0 + ((u128)a1 << 26) + ((u128)a2 << 52);
  return reduce128(v, m);
}

template <int FO, bool STRIDED>
__global__ __launch_bounds__(FB) void k_fused_split(OutList out, const uint64_t* __restrict__ in_base,
                                                    size_t in_stride, const uint64_t* const* __restrict__ in_ptrs,
                                                    PtrList pts, int K, int F, int l_first, int n_out, int F_pad,
                                                    int l1, const uint32_t* __restrict__ w, int log_n,
                                                    const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)FB + threadIdx.x;
  const int i = blockIdx.y, c = blockIdx.z;
  const Mod m = mods[i];
  const size_t off = ((size_t)c * l1 + i) * N + j;
  uint32_t p0[16], p1[16];
  for (int k = 0; k < K; ++k) {
    uint64_t p = pts.p[k][(size_t)i * N + j];
    p0[k] = (uint32_t)(p & M26);
    p1[k] = (uint32_t)(p >> 26);
  }
  uint64_t b0[FO], b1[FO], b2[FO];
#pragma unroll
  for (int l = 0; l < FO; ++l) b0[l] = b1[l] = b2[l] = 0;
  // weights: [l1][F][F_pad][2] 26-bit halves, columns beyond F' are zero
  const uint32_t* wrow = w + ((size_t)i * F) * F_pad * 2 + (size_t)l_first * 2;
  for (int f = 0; f < F; ++f) {
    uint64_t z;
    if (K > 0) {
      uint64_t a0 = 0, a1 = 0, a2 = 0;
      for (int k = 0; k < K; ++k) {
        const size_t idx = (size_t)k * F + f;
        const uint64_t x = STRIDED ? in_base[idx * in_stride + off] : in_ptrs[idx][off];
        const uint32_t x0 = (uint32_t)(x & M26), x1 = (uint32_t)(x >> 26);
        a0 = mad32(p0[k], x0, a0);
        a1 = mad32(p0[k], x1, a1);
        a1 = mad32(p1[k], x0, a1);
        a2 = mad32(p1[k], x1, a2);
      }
      z = fold3(a0, a1, a2, m);
    } else {
      z = STRIDED ? in_base[(size_t)f * in_stride + off] : in_ptrs[f][off];
    }
    const uint32_t z0 = (uint32_t)(z & M26), z1 = (uint32_t)(z >> 26);
    const uint32_t* wf = wrow + (size_t)f * F_pad * 2;
    uint32_t w0[FO], w1[FO];
#pragma unroll
    for (int l = 0; l < FO; ++l) {
      w0[l] = wf[2 * l];
      w1[l] = wf[2 * l + 1];
    }
#pragma unroll
    for (int l = 0; l < FO; ++l) b0[l] = mad32(z0, w0[l], b0[l]);
#pragma unroll
    for (int l = 0; l < FO; ++l) b1[l] = mad32(z0, w1[l], b1[l]);
#pragma unroll
    for (int l = 0; l < FO; ++l) b2[l] = mad32(z1, w1[l], b2[l]);
#pragma unroll
    for (int l = 0; l < FO; ++l) b1[l] = mad32(z1, w0[l], b1[l]);
    if ((f & 1023) == 1023) {
#pragma unroll
      for (int l = 0; l < FO; ++l) {
        b0[l] = fold3(b0[l], b1[l], b2[l], m);
        b1[l] = b2[l] = 0;
      }
    }
  }
#pragma unroll
  for (int l = 0; l < FO; ++l)
    if (l < n_out) out.p[l][off] = fold3(b0[l], b1[l], b2[l], m);
}

// 128-bit accumulation variant for primes of 52 bits or more.
template <int FO>
__global__ __launch_bounds__(FB) void k_fused_wide(OutList out, const uint64_t* __restrict__ in_base,
                                                   size_t in_stride, const uint64_t* const* __restrict__ in_ptrs,
                                                   PtrList pts, int K, int F, int l_first,
                                                   int n_out, int F_out, int l1, const uint64_t* __restrict__ w,
                                                   int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)FB + threadIdx.x;
  const int i = blockIdx.y, c = blockIdx.z;
  const Mod m = mods[i];
  const size_t off = ((size_t)c * l1 + i) * N + j;
  uint64_t p[16];
  for (int k = 0; k < K; ++k) p[k] = pts.p[k][(size_t)i * N + j];
  u128 acc[FO];
#pragma unroll
  for (int l = 0; l < FO; ++l) acc[l] = 0;
  const uint64_t* wrow = w + ((size_t)i * F) * F_out + l_first;
  for (int f = 0; f < F; ++f) {
    uint64_t z;
    if (K > 0) {
      u128 s = 0;
      for (int k = 0; k < K; ++k) {
        const size_t idx = (size_t)k * F + f;
        s += (u128)p[k] * (in_base ? in_base[idx * in_stride + off] : in_ptrs[idx][off]);
      }
      z = reduce128(s, m);
    } else {
      z = in_base ? in_base[(size_t)f * in_stride + off] : in_ptrs[f][off];
    }
    const uint64_t* wf = wrow + (size_t)f * F_out;
#pragma unroll
    for (int l = 0; l < FO; ++l)
      if (l < n_out) acc[l] += (u128)z * wf[l];
    if ((f & 15) == 15) {
#pragma unroll
      for (int l = 0; l < FO; ++l) acc[l] = reduce128(acc[l], m);
    }
  }
#pragma unroll
  for (int l = 0; l < FO; ++l)
    if (l < n_out) out.p[l][off] = reduce128(acc[l], m);
}

// w: split form [l1][F][F_out][2] uint32 halves, wide form [l1][F][F_out] residues.
// outs: F_out output buffers; one launch per group of 16 columns.
void comb_fused(ckks_ctx* c, const std::vector<uint64_t*>& outs, const uint64_t* in_base, size_t in_stride,
                const uint64_t* const* in_dev_ptrs, const PtrList& pts, int K, int F, int F_out, int level,
                const void* w_dev, bool split, const char* prof_name) {
  ProfScope ps(c, prof_name);
  if (K > PtrList::MAX) FICGCN_THROW(EPLAN_, "more than 16 Inter-CA copies per fused launch");
  if ((int)outs.size() != F_out) FICGCN_THROW(EINVAL_, "output list size");
  const int l1 = level + 1;
  for (int l0 = 0; l0 < F_out; l0 += OutList::MAX) {
    const int n = std::min((int)OutList::MAX, F_out - l0);
    OutList o{};
    for (int l = 0; l < n; ++l) o.p[l] = outs[l0 + l];
    dim3 grid(c->N / FB, l1, 2);
    if (split) {
      // split weights are padded to a multiple of 16 columns
      const uint32_t* w = (const uint32_t*)w_dev;
      const int F_pad = (F_out + 15) / 16 * 16;
      if (in_base)
        hipLaunchKernelGGL((k_fused_split<16, true>), grid, dim3(FB), 0, c->stream, o, in_base, in_stride, in_dev_ptrs,
                           pts, K, F, l0, n, F_pad, l1, w, c->log_n, c->t.mods);
      else
        hipLaunchKernelGGL((k_fused_split<16, false>), grid, dim3(FB), 0, c->stream, o, in_base, in_stride,
                           in_dev_ptrs, pts, K, F, l0, n, F_pad, l1, w, c->log_n, c->t.mods);
    } else {
      const uint64_t* w = (const uint64_t*)w_dev;
      if (n <= 8)
        hipLaunchKernelGGL(k_fused_wide<8>, grid, dim3(FB), 0, c->stream, o, in_base, in_stride, in_dev_ptrs, pts,
                           K, F, l0, n, F_out, l1, w, c->log_n, c->t.mods);
      else
        hipLaunchKernelGGL(k_fused_wide<16>, grid, dim3(FB), 0, c->stream, o, in_base, in_stride, in_dev_ptrs, pts,
                           K, F, l0, n, F_out, l1, w, c->log_n, c->t.mods);
    }
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
