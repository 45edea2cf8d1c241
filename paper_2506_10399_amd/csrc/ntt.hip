// Negacyclic NTT over Z_q[X]/(X^N + 1) for gfx950.
//
// Forward transform (Cooley-Tukey, twiddles psi^{brev(m+i)} merged with the
// negacyclic twist): coefficients in natural order -> evaluations at the odd
// powers psi^{2 brev(k) + 1} in bit-reversed order k.  Inverse: the
// Gentleman-Sande mirror, then a multiply by N^{-1}.
//
// A limb of N = 2^16 words (512 KiB) exceeds the LDS, so each transform runs
// as two passes of N = N1 * N2:
//   column pass: the stages m < N1 touch only the N1 elements j0 + k*N2 of one
//                column j0 (a C = N1-point sub-transform);
//   row pass   : the stages m >= N1 stay inside one contiguous chunk of C = N2
//                words.
// Inside a pass, TPC = 2^floor(log C / 2) threads share one sub-transform and
// each holds EPT = C / TPC elements in registers:
//   strided layout     thread r holds elements r + TPC*u  (u < EPT): the
//                      stages with butterfly distance t >= TPC are local;
//   contiguous layout  thread r holds elements r*EPT + v (v < EPT): the stages
//                      with t < TPC are local.
// One LDS transpose switches layouts (a second one in the row pass keeps the
// global loads and stores coalesced).  Every twiddle a thread needs is read
// before its stages run.  A workgroup handles COLS columns (column pass) or
// chunks (row pass); COLS is picked per ring degree by the autotuner.
// For the 50-bit Q primes (fp64 residue arithmetic below) the limb travels
// between the two passes as the bit patterns of its doubles: the first pass
// converts on load, the second on store.
#include "internal.h"
#include "fpmod.h"

namespace ficgcn {

// ModUp output: digit d of a source owns limbs d*alpha .. d*alpha+alpha-1, which
// hold evaluation-form input already; polys run digit-fastest over sources
__device__ __forceinline__ bool skip_limb(int limb, int poly, int skip_alpha, int skip_q) {
  return skip_alpha > 0 && limb < skip_q && limb / skip_alpha == poly % ((skip_q + skip_alpha - 1) / skip_alpha);
}

// Integer butterflies with lazy reduction (Harvey's, for q < 2^62): inside a forward
// transform the values lie in [0, 4q), inside an inverse one in [0, 2q).  Shoup's
// product without its correction lands in [0, 2q) for any 64-bit input, so
//   forward CT: x <- x mod 2q (one conditional subtract), t = y w in [0, 2q),
//               (x, y) <- (x + t, x - t + 2q), both in [0, 4q);
//   inverse GS: (x, y) <- (x + y reduced to [0, 2q), (x - y + 2q) w in [0, 2q)).
// The forward transform's last pass and the inverse's scaling by 1/N return [0, q).
__device__ __forceinline__ void bf_fwd(uint64_t& x, uint64_t& y, uint64_t w, uint64_t ws, uint64_t q) {
  const uint64_t q2 = 2 * q;
  const uint64_t a = x >= q2 ? x - q2 : x;
  const uint64_t t = mul_shoup_lazy(y, w, ws, q);
  x = a + t;
  y = a - t + q2;
}
__device__ __forceinline__ void bf_inv(uint64_t& x, uint64_t& y, uint64_t w, uint64_t ws, uint64_t q) {
  const uint64_t q2 = 2 * q;
  const uint64_t s = x + y;
  const uint64_t d = x - y + q2;
  x = s >= q2 ? s - q2 : s;
  y = mul_shoup_lazy(d, w, ws, q);
}
// [0, 4q) -> [0, q)
__device__ __forceinline__ uint64_t canon4(uint64_t x, uint64_t q) {
  x = x >= 2 * q ? x - 2 * q : x;
  return x >= q ? x - q : x;
}


template <bool FP>
__device__ __forceinline__ void bfly_fwd(uint64_t& x, uint64_t& y, uint64_t w, uint64_t ws, uint64_t q, double qd,
                                         double qinv, bool red = true) {
  if (FP) {
    const double xd = b2f(x), v = fmulmod_s(b2f(y), b2f(w), qd, qinv);
    x = f2b(red ? sred(xd + v, qd, qinv) : xd + v);
    y = f2b(red ? sred(xd - v, qd, qinv) : xd - v);
  } else {
    bf_fwd(x, y, w, ws, q);
  }
}

template <bool FP>
__device__ __forceinline__ void bfly_inv(uint64_t& x, uint64_t& y, uint64_t w, uint64_t ws, uint64_t q, double qd,
                                         double qinv, bool red = true) {
  if (FP) {
    const double xd = b2f(x), yd = b2f(y);
    x = f2b(red ? sred(xd + yd, qd, qinv) : xd + yd);
    y = f2b(fmulmod_s(red ? sred(xd - yd, qd, qinv) : xd - yd, b2f(w), qd, qinv));
  } else {
    bf_inv(x, y, w, ws, q);
  }
}

// One pass over one sub-transform set of a limb; FP selects the fp64 residue arithmetic.
template <int LOGC, int COLS, bool INV, bool ROW, bool FP>
__device__ __forceinline__ void ntt_pass_body(uint64_t* s, uint64_t* a, const uint64_t* __restrict__ W,
                                              const uint64_t* __restrict__ Ws, const double* __restrict__ Wf,
                                              uint64_t q, int N, int mi,
                                              const uint64_t* __restrict__ ninv,
                                              const uint64_t* __restrict__ ninv_s) {
  constexpr int C = 1 << LOGC;
  constexpr int LT = LOGC / 2;
  constexpr int TPC = 1 << LT;
  constexpr int LE = LOGC - LT;
  constexpr int EPT = 1 << LE;
  const double qd = (double)q, qinv = 1.0 / qd;
  auto twv = [&](int k) { return FP ? f2b(Wf[k]) : W[k]; };
  auto tws = [&](int k) { return FP ? (uint64_t)0 : Ws[k]; };
  const int tid = threadIdx.x;
  // column pass: consecutive threads = consecutive columns (coalesced rows);
  // row pass: consecutive threads = consecutive elements of one chunk
  const int col = ROW ? tid / TPC : tid % COLS;
  const int r = ROW ? tid % TPC : tid / COLS;
  const int unit = blockIdx.x * COLS + col;           // column index j0 or chunk index
  const int stride = ROW ? 1 : (N >> LOGC);           // element step inside the sub-transform
  uint64_t* g = ROW ? a + (size_t)unit * C : a + unit;
  // global twiddle index of group i at local stage st
  auto twi = [&](int st, int i) { return ROW ? ((N >> LOGC) << st) + unit * (1 << st) + i : (1 << st) + i; };
  // LDS element index of element e of this unit
  auto sidx = [&](int e) { return ROW ? col * (C + TPC) + e + e / EPT : e * COLS + col + (e / EPT) * COLS; };
  uint64_t x[EPT];

  if (!INV) {
    // ---- load strided: x[u] = element r + TPC u
#pragma unroll
    for (int u = 0; u < EPT; ++u) x[u] = FP && !ROW ? to_fbits(g[(size_t)(r + TPC * u) * stride]) : g[(size_t)(r + TPC * u) * stride];
    // ---- stages 0..LE-1 (t >= TPC) in registers
    {
      uint64_t w[EPT], ws[EPT];
#pragma unroll
      for (int st = 0; st < LE; ++st)
#pragma unroll
        for (int i = 0; i < (1 << st); ++i) {
          int k = twi(st, i);
          w[(1 << st) + i - 1] = twv(k);
          ws[(1 << st) + i - 1] = tws(k);
        }
#pragma unroll
      for (int st = 0; st < LE; ++st) {
        const int tu = EPT >> (st + 1);
#pragma unroll
        for (int u = 0; u < EPT; ++u)
          if ((u & tu) == 0) {
            const int i = u / (2 * tu);
            bfly_fwd<FP>(x[u], x[u + tu], w[(1 << st) + i - 1], ws[(1 << st) + i - 1], q, qd, qinv,
                         (st & 1) || st == LOGC - 1);
          }
      }
    }
    // ---- transpose to the contiguous layout
#pragma unroll
    for (int u = 0; u < EPT; ++u) s[sidx(r + TPC * u)] = x[u];
    __syncthreads();
#pragma unroll
    for (int v = 0; v < EPT; ++v) x[v] = s[sidx(r * EPT + v)];
    // ---- stages LE..LOGC-1 (t < TPC), element r*EPT + v
    {
      uint64_t w[EPT], ws[EPT];   // at most EPT - 1 twiddles in these stages
      int pos = 0;
#pragma unroll
      for (int st = LE; st < LOGC; ++st) {
        const int t = C >> (st + 1);
        const int ng = EPT / (2 * t) > 0 ? EPT / (2 * t) : 1;   // groups touched by this thread
#pragma unroll
        for (int gi = 0; gi < ng; ++gi) {
          int i = (r * EPT) / (2 * t) + gi;
          int k = twi(st, i);
          w[pos] = twv(k);
          ws[pos] = tws(k);
          ++pos;
        }
      }
      pos = 0;
#pragma unroll
      for (int st = LE; st < LOGC; ++st) {
        const int t = C >> (st + 1);
        const int ng = EPT / (2 * t) > 0 ? EPT / (2 * t) : 1;
#pragma unroll
        for (int v = 0; v < EPT; ++v)
          if ((v & t) == 0) {
            const int gi = v / (2 * t);
            bfly_fwd<FP>(x[v], x[v + t], w[pos + gi], ws[pos + gi], q, qd, qinv, (st & 1) || st == LOGC - 1);
          }
        pos += ng;
      }
    }
    if (FP && ROW) {
#pragma unroll
      for (int v = 0; v < EPT; ++v) x[v] = from_fbits(f2b(canon(b2f(x[v]), qd)));
    }
    if (!FP && ROW) {
#pragma unroll
      for (int v = 0; v < EPT; ++v) x[v] = canon4(x[v], q);
    }
    if (ROW) {
      // back to the strided layout for a coalesced store
      __syncthreads();
#pragma unroll
      for (int v = 0; v < EPT; ++v) s[sidx(r * EPT + v)] = x[v];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < EPT; ++u) g[(size_t)(r + TPC * u) * stride] = s[sidx(r + TPC * u)];
    } else {
#pragma unroll
      for (int v = 0; v < EPT; ++v) g[(size_t)(r * EPT + v) * stride] = x[v];
    }
  } else {
    // ---- inverse: load in the contiguous layout
    if (ROW) {
#pragma unroll
      for (int u = 0; u < EPT; ++u) s[sidx(r + TPC * u)] = g[(size_t)(r + TPC * u) * stride];
      __syncthreads();
#pragma unroll
      for (int v = 0; v < EPT; ++v) x[v] = s[sidx(r * EPT + v)];
      __syncthreads();
    } else {
#pragma unroll
      for (int v = 0; v < EPT; ++v) x[v] = g[(size_t)(r * EPT + v) * stride];
    }
    if (FP && ROW) {
#pragma unroll
      for (int v = 0; v < EPT; ++v) x[v] = to_fbits(x[v]);
    }
    // ---- stages LOGC-1..LE (t < TPC) in registers
    {
      uint64_t w[EPT], ws[EPT];   // at most EPT - 1 twiddles in these stages
      int pos = 0;
#pragma unroll
      for (int st = LOGC - 1; st >= LE; --st) {
        const int t = C >> (st + 1);
        const int ng = EPT / (2 * t) > 0 ? EPT / (2 * t) : 1;
#pragma unroll
        for (int gi = 0; gi < ng; ++gi) {
          int i = (r * EPT) / (2 * t) + gi;
          int k = twi(st, i);
          w[pos] = twv(k);
          ws[pos] = tws(k);
          ++pos;
        }
      }
      pos = 0;
#pragma unroll
      for (int st = LOGC - 1; st >= LE; --st) {
        const int t = C >> (st + 1);
        const int ng = EPT / (2 * t) > 0 ? EPT / (2 * t) : 1;
#pragma unroll
        for (int v = 0; v < EPT; ++v)
          if ((v & t) == 0) {
            const int gi = v / (2 * t);
            bfly_inv<FP>(x[v], x[v + t], w[pos + gi], ws[pos + gi], q, qd, qinv, ((LOGC - 1 - st) & 1) || st == 0);
          }
        pos += ng;
      }
    }
    // ---- transpose to the strided layout
#pragma unroll
    for (int v = 0; v < EPT; ++v) s[sidx(r * EPT + v)] = x[v];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < EPT; ++u) x[u] = s[sidx(r + TPC * u)];
    // ---- stages LE-1..0 (t >= TPC)
    {
      uint64_t w[EPT], ws[EPT];
#pragma unroll
      for (int st = 0; st < LE; ++st)
#pragma unroll
        for (int i = 0; i < (1 << st); ++i) {
          int k = twi(st, i);
          w[(1 << st) + i - 1] = twv(k);
          ws[(1 << st) + i - 1] = tws(k);
        }
#pragma unroll
      for (int st = LE - 1; st >= 0; --st) {
        const int tu = EPT >> (st + 1);
#pragma unroll
        for (int u = 0; u < EPT; ++u)
          if ((u & tu) == 0) {
            const int i = u / (2 * tu);
            bfly_inv<FP>(x[u], x[u + tu], w[(1 << st) + i - 1], ws[(1 << st) + i - 1], q, qd, qinv,
                         ((LOGC - 1 - st) & 1) || st == 0);
          }
      }
    }
    if (!ROW) {
      const uint64_t ni = ninv[mi], nis = ninv_s[mi];
      const double nid = (double)ni;
#pragma unroll
      for (int u = 0; u < EPT; ++u) x[u] = FP ? f2b(fmulmod(b2f(x[u]), nid, qd, qinv)) : mul_shoup(x[u], ni, nis, q);
    }
    if (FP && !ROW) {
#pragma unroll
      for (int u = 0; u < EPT; ++u) x[u] = from_fbits(x[u]);
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) g[(size_t)(r + TPC * u) * stride] = x[u];
  }
}

// ROW: row pass (sub-transform = contiguous chunk), else column pass.
template <int LOGC, int COLS, bool INV, bool ROW>
__global__ __launch_bounds__((1 << (LOGC / 2)) * COLS) void k_ntt_pass(
    uint64_t* __restrict__ base, int log_n, LimbMap map, size_t poly_stride, const uint64_t* __restrict__ tw,
    const uint64_t* __restrict__ tws, const double* __restrict__ twf, const Mod* __restrict__ mods,
    const uint64_t* __restrict__ ninv, const uint64_t* __restrict__ ninv_s, int skip_alpha, int skip_q) {
  constexpr int C = 1 << LOGC;
  constexpr int TPC = 1 << (LOGC / 2);
  // one pad word per EPT elements (row pass) or one group width per EPT rows
  // (column pass) keeps the contiguous-layout accesses off a single bank set
  __shared__ uint64_t s[COLS * (C + TPC)];
  const int limb = blockIdx.y, poly = blockIdx.z;
  if (skip_limb(limb, poly, skip_alpha, skip_q)) return;
  const int N = 1 << log_n;
  const int mi = lm_mod(map, limb);
  const uint64_t q = mods[mi].q;
  uint64_t* a = base + poly * poly_stride + (size_t)limb * N;
  const uint64_t* W = tw + (size_t)mi * N;
  const uint64_t* Ws = tws + (size_t)mi * N;
  const double* Wf = twf + (size_t)mi * N;
  if (q > (1ull << 49) && q < (1ull << 50))
    ntt_pass_body<LOGC, COLS, INV, ROW, true>(s, a, W, Ws, Wf, q, N, mi, ninv, ninv_s);
  else
    ntt_pass_body<LOGC, COLS, INV, ROW, false>(s, a, W, Ws, Wf, q, N, mi, ninv, ninv_s);
}

// ---- launch selection --------------------------------------------------------
template <bool INV, bool ROW, int COLS>
static void launch_c(int logc, dim3 grid, hipStream_t st, uint64_t* base, int log_n, LimbMap map, size_t ps,
                     const Tables& t, int sa, int sq) {
  const uint64_t* tw = INV ? t.ipsi : t.psi;
  const uint64_t* tws = INV ? t.ipsi_s : t.psi_s;
  const double* twf = INV ? t.ipsi_f : t.psi_f;
  switch (logc) {
#define CASE(L)                                                                                                   \
  case L:                                                                                                         \
    hipLaunchKernelGGL((k_ntt_pass<L, COLS, INV, ROW>), grid, dim3((1 << (L / 2)) * COLS), 0, st, base, log_n, map, \
                       ps, tw, tws, twf, t.mods, t.ninv, t.ninv_s, sa, sq);                                       \
    break;
    CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9)
#undef CASE
    default: FICGCN_THROW(EINVAL_, "unsupported ring degree");
  }
}

template <bool INV, bool ROW>
static void launch(ckks_ctx* c, int logc, int cols, uint64_t* base, int n_limbs, LimbMap map, int n_polys,
                   size_t ps, int sa, int sq) {
  const int units = c->N >> logc;   // columns (column pass) or chunks (row pass)
  if (units % cols) cols = 1;
  dim3 grid(units / cols, n_limbs, n_polys);
  switch (cols) {
    case 1: launch_c<INV, ROW, 1>(logc, grid, c->stream, base, c->log_n, map, ps, c->t, sa, sq); break;
    case 2: launch_c<INV, ROW, 2>(logc, grid, c->stream, base, c->log_n, map, ps, c->t, sa, sq); break;
    case 4: launch_c<INV, ROW, 4>(logc, grid, c->stream, base, c->log_n, map, ps, c->t, sa, sq); break;
    case 8: launch_c<INV, ROW, 8>(logc, grid, c->stream, base, c->log_n, map, ps, c->t, sa, sq); break;
    default: launch_c<INV, ROW, 16>(logc, grid, c->stream, base, c->log_n, map, ps, c->t, sa, sq); break;
  }
}

// N = 2^l1 (column pass) * 2^l2 (row pass); each pass between 2^4 and 2^9 points
static void split(const ckks_ctx* c, int& l1, int& l2) {
  l1 = c->ntt_split ? c->ntt_split : c->log_n / 2;
  l2 = c->log_n - l1;
  if (l1 < 4 || l1 > 9 || l2 < 4 || l2 > 9) FICGCN_THROW(EINVAL_, "NTT split outside 2^4..2^9 points per pass");
}

void ntt_fwd(ckks_ctx* c, uint64_t* base, int n_limbs, LimbMap map, int n_polys, size_t poly_stride, int skip_alpha,
             int skip_q) {
  ProfScope ps(c, "ntt");
  if (n_limbs <= 0 || n_polys <= 0) return;
  int l1, l2;
  split(c, l1, l2);
  launch<false, false>(c, l1, c->ntt_cols[0], base, n_limbs, map, n_polys, poly_stride, skip_alpha, skip_q);
  launch<false, true>(c, l2, c->ntt_cols[1], base, n_limbs, map, n_polys, poly_stride, skip_alpha, skip_q);
  HIPCHECK(hipGetLastError());
}

void ntt_inv(ckks_ctx* c, uint64_t* base, int n_limbs, LimbMap map, int n_polys, size_t poly_stride) {
  ProfScope ps(c, "ntt");
  if (n_limbs <= 0 || n_polys <= 0) return;
  int l1, l2;
  split(c, l1, l2);
  launch<true, true>(c, l2, c->ntt_cols[1], base, n_limbs, map, n_polys, poly_stride, 0, 0);
  launch<true, false>(c, l1, c->ntt_cols[0], base, n_limbs, map, n_polys, poly_stride, 0, 0);
  HIPCHECK(hipGetLastError());
}

}  // namespace ficgcn
