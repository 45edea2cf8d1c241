// Negacyclic NTT over Z_q[X]/(X^N + 1) for gfx950.
//
// Forward transform (Cooley-Tukey, twiddles psi^{brev(m+i)} merged with the
// negacyclic twist): coefficients in natural order -> evaluations at the odd
// powers psi^{2 brev(k) + 1} in bit-reversed order k.  Inverse: the
// Gentleman-Sande mirror, then a multiply by N^{-1}.
//
// A limb of N = 2^16 words (512 KiB) exceeds the 160 KiB LDS, so each
// transform runs as two passes of N = N1 * N2:
//   column pass : the stages m < N1 touch only elements j0 + k*N2 (k < N1) of
//                 one column j0; a workgroup stages 16 adjacent columns
//                 (128-byte rows, coalesced) in LDS and runs those stages;
//   row pass    : the stages m >= N1 stay inside contiguous chunks of N2
//                 words; a workgroup stages 16 chunks.
// Each pass reads and writes the limb once, so a transform moves 4 N words.
#include "internal.h"

namespace ficgcn {

constexpr int NTT_THREADS = 256;
constexpr int NTT_TILE = 16;   // columns (column pass) or chunks (row pass) per workgroup

__device__ __forceinline__ bool skip_limb(int limb, int poly, int skip_alpha, int skip_q) {
  return skip_alpha > 0 && limb < skip_q && limb / skip_alpha == poly;
}

template <int LOGC, bool INV>
__global__ __launch_bounds__(NTT_THREADS) void k_ntt_cols(uint64_t* __restrict__ base, int log_n, LimbMap map,
                                                        size_t poly_stride, const uint64_t* __restrict__ tw,
                                                        const uint64_t* __restrict__ tws, const Mod* __restrict__ mods,
                                                        const uint64_t* __restrict__ ninv,
                                                        const uint64_t* __restrict__ ninv_s, int skip_alpha,
                                                        int skip_q) {
  constexpr int C = 1 << LOGC;
  __shared__ uint64_t s[C * NTT_TILE];
  const int limb = blockIdx.y, poly = blockIdx.z;
  if (skip_limb(limb, poly, skip_alpha, skip_q)) return;
  const int N = 1 << log_n;
  const int stride = N >> LOGC;
  const int mi = lm_mod(map, limb);
  const uint64_t q = mods[mi].q;
  uint64_t* a = base + poly * poly_stride + (size_t)limb * N;
  const uint64_t* W = tw + (size_t)mi * N;
  const uint64_t* Ws = tws + (size_t)mi * N;
  const int col0 = blockIdx.x * NTT_TILE;
  for (int e = threadIdx.x; e < C * NTT_TILE; e += NTT_THREADS) {
    int r = e / NTT_TILE, cc = e % NTT_TILE;
    s[e] = a[(size_t)r * stride + col0 + cc];
  }
  __syncthreads();
#pragma unroll 1
  for (int it = 0; it < LOGC; ++it) {
    const int st = INV ? (LOGC - 1 - it) : it;
    const int m = 1 << st;
    const int t = C >> (st + 1);
    for (int b = threadIdx.x; b < (C / 2) * NTT_TILE; b += NTT_THREADS) {
      int cc = b % NTT_TILE, k = b / NTT_TILE;
      int i = k / t, r = k % t;
      int j = i * 2 * t + r;
      uint64_t w = W[m + i], ws = Ws[m + i];
      uint64_t* x = &s[j * NTT_TILE + cc];
      uint64_t* y = &s[(j + t) * NTT_TILE + cc];
      uint64_t U = *x, V = *y;
      if (!INV) {
        V = mul_shoup(V, w, ws, q);
        *x = add_mod(U, V, q);
        *y = sub_mod(U, V, q);
      } else {
        *x = add_mod(U, V, q);
        *y = mul_shoup(sub_mod(U, V, q), w, ws, q);
      }
    }
    __syncthreads();
  }
  const uint64_t ni = INV ? ninv[mi] : 0, nis = INV ? ninv_s[mi] : 0;
  for (int e = threadIdx.x; e < C * NTT_TILE; e += NTT_THREADS) {
    int r = e / NTT_TILE, cc = e % NTT_TILE;
    uint64_t v = s[e];
    if (INV) v = mul_shoup(v, ni, nis, q);
    a[(size_t)r * stride + col0 + cc] = v;
  }
}

template <int LOGC, bool INV>
__global__ __launch_bounds__(NTT_THREADS) void k_ntt_rows(uint64_t* __restrict__ base, int log_n, LimbMap map,
                                                        size_t poly_stride, const uint64_t* __restrict__ tw,
                                                        const uint64_t* __restrict__ tws, const Mod* __restrict__ mods,
                                                        int skip_alpha, int skip_q) {
  constexpr int C = 1 << LOGC;
  __shared__ uint64_t s[C * NTT_TILE];
  const int limb = blockIdx.y, poly = blockIdx.z;
  if (skip_limb(limb, poly, skip_alpha, skip_q)) return;
  const int N = 1 << log_n;
  const int N1 = N >> LOGC;   // number of chunks = first-pass length
  const int mi = lm_mod(map, limb);
  const uint64_t q = mods[mi].q;
  uint64_t* a = base + poly * poly_stride + (size_t)limb * N;
  const uint64_t* W = tw + (size_t)mi * N;
  const uint64_t* Ws = tws + (size_t)mi * N;
  const int ch0 = blockIdx.x * NTT_TILE;
  uint64_t* g = a + (size_t)ch0 * C;
  for (int e = threadIdx.x; e < C * NTT_TILE; e += NTT_THREADS) s[e] = g[e];
  __syncthreads();
#pragma unroll 1
  for (int it = 0; it < LOGC; ++it) {
    const int st = INV ? (LOGC - 1 - it) : it;
    const int m = N1 << st;   // global stage
    const int t = C >> (st + 1);
    for (int b = threadIdx.x; b < (C / 2) * NTT_TILE; b += NTT_THREADS) {
      int cc = b / (C / 2), k = b % (C / 2);
      int il = k / t, r = k % t;
      int j = il * 2 * t + r;
      int ti = m + (ch0 + cc) * (1 << st) + il;
      uint64_t w = W[ti], ws = Ws[ti];
      uint64_t* x = &s[cc * C + j];
      uint64_t* y = x + t;
      uint64_t U = *x, V = *y;
      if (!INV) {
        V = mul_shoup(V, w, ws, q);
        *x = add_mod(U, V, q);
        *y = sub_mod(U, V, q);
      } else {
        *x = add_mod(U, V, q);
        *y = mul_shoup(sub_mod(U, V, q), w, ws, q);
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < C * NTT_TILE; e += NTT_THREADS) g[e] = s[e];
}

template <bool INV>
static void launch_cols(int logc, dim3 grid, hipStream_t st, uint64_t* base, int log_n, LimbMap map, size_t ps,
                        const uint64_t* tw, const uint64_t* tws, const Mod* mods, const uint64_t* ni,
                        const uint64_t* nis, int sa, int sq) {
  switch (logc) {
#define CASE(L)                                                                                                \
  case L:                                                                                                      \
    hipLaunchKernelGGL((k_ntt_cols<L, INV>), grid, dim3(NTT_THREADS), 0, st, base, log_n, map, ps, tw, tws, mods, \
                       ni, nis, sa, sq);                                                                       \
    break;
    CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: FICGCN_THROW(EINVAL_, "unsupported ring degree");
  }
}

template <bool INV>
static void launch_rows(int logc, dim3 grid, hipStream_t st, uint64_t* base, int log_n, LimbMap map, size_t ps,
                        const uint64_t* tw, const uint64_t* tws, const Mod* mods, int sa, int sq) {
  switch (logc) {
#define CASE(L)                                                                                                 \
  case L:                                                                                                       \
    hipLaunchKernelGGL((k_ntt_rows<L, INV>), grid, dim3(NTT_THREADS), 0, st, base, log_n, map, ps, tw, tws, mods, \
                       sa, sq);                                                                                 \
    break;
    CASE(5) CASE(6) CASE(7) CASE(8) CASE(9)
#undef CASE
    default: FICGCN_THROW(EINVAL_, "unsupported ring degree");
  }
}

static void split(int log_n, int& l1, int& l2) {
  l1 = log_n / 2;
  l2 = log_n - l1;
}

void ntt_fwd(ckks_ctx* c, uint64_t* base, int n_limbs, LimbMap map, int n_polys, size_t poly_stride, int skip_alpha,
             int skip_q) {
  ProfScope ps(c, "ntt");
  if (n_limbs <= 0 || n_polys <= 0) return;
  int l1, l2;
  split(c->log_n, l1, l2);
  dim3 g1((c->N >> l1) / NTT_TILE, n_limbs, n_polys);
  launch_cols<false>(l1, g1, c->stream, base, c->log_n, map, poly_stride, c->t.psi, c->t.psi_s, c->t.mods, nullptr,
                     nullptr, skip_alpha, skip_q);
  dim3 g2((c->N >> l2) / NTT_TILE, n_limbs, n_polys);
  launch_rows<false>(l2, g2, c->stream, base, c->log_n, map, poly_stride, c->t.psi, c->t.psi_s, c->t.mods, skip_alpha,
                     skip_q);
  HIPCHECK(hipGetLastError());
}

void ntt_inv(ckks_ctx* c, uint64_t* base, int n_limbs, LimbMap map, int n_polys, size_t poly_stride) {
  ProfScope ps(c, "ntt");
  if (n_limbs <= 0 || n_polys <= 0) return;
  int l1, l2;
  split(c->log_n, l1, l2);
  dim3 g2((c->N >> l2) / NTT_TILE, n_limbs, n_polys);
  launch_rows<true>(l2, g2, c->stream, base, c->log_n, map, poly_stride, c->t.ipsi, c->t.ipsi_s, c->t.mods, 0, 0);
  dim3 g1((c->N >> l1) / NTT_TILE, n_limbs, n_polys);
  launch_cols<true>(l1, g1, c->stream, base, c->log_n, map, poly_stride, c->t.ipsi, c->t.ipsi_s, c->t.mods,
                    c->t.ninv, c->t.ninv_s, 0, 0);
  HIPCHECK(hipGetLastError());
}

}  // namespace ficgcn
