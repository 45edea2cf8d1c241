// Canonical-embedding encoder on the device (server-side plaintexts: masks,
// weights; the client's inputs).  Same transform as the host encoder: slot j
// of m(X) is m(zeta^(5^j)), the N FFT inputs are the slot values at the odd
// powers of zeta (conjugates at zeta^(-5^j)), and
//   m_i = round_half_even( Re(exp(-i pi i / N) * FFT(v)_i) / N * scale ).
// The N-point FFT runs as two passes of N = N1 * N2 points (four-step form):
//   column pass: for each s2 < N2, the N1-point DFT over s1 of v[N2 s1 + s2],
//                times w^(s2 i1) (w = exp(-2 pi i / N)), back in place at N2 i1 + s2;
//   row pass   : for each i1 < N1, the N2-point DFT over s2 of that row, written
//                in natural order, FFT(v)_{i1 + N1 i2}.
// Each sub-DFT is an in-LDS radix-2 transform (bit-reversed load) of a block of
// COLS columns or rows.  Then one kernel rounds, checks the 63-bit range and
// writes the residues of every limb, and the NTT takes them to evaluation form.
// Independent fp64 FFTs can round a coefficient differently when its scaled
// value sits within the FFT's error of a half-integer; decoding absorbs it.
#include "internal.h"

namespace ficgcn {

typedef double2 cplx;

__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return make_double2(a.x - b.x, a.y - b.y); }

constexpr int ET = 256;           // threads per block
constexpr int ENC_LDS = 32768;    // bytes of LDS per block: COLS * C complex values

// v[b][pos[2j]] = z_j, v[b][pos[2j+1]] = conj(z_j), z_j = (re, im) (zero past n)
__global__ void k_enc_scatter(const double* __restrict__ re, const double* __restrict__ im, size_t n,
                              const uint32_t* __restrict__ pos, cplx* __restrict__ v, int N) {
  const size_t j = blockIdx.x * (size_t)ET + threadIdx.x;
  const size_t b = blockIdx.y;
  if (j >= (size_t)N / 2) return;
  const double x = j < n ? re[b * n + j] : 0.0;
  const double y = j < n && im ? im[b * n + j] : 0.0;
  cplx* vb = v + b * (size_t)N;
  vb[pos[2 * j]] = make_double2(x, y);
  vb[pos[2 * j + 1]] = make_double2(x, -y);
}

__device__ __forceinline__ uint32_t brev_bits(uint32_t x, int bits) { return __brev(x) >> (32 - bits); }

// w^e for e in [0, N): root holds w^k for k < N/2, and w^(k + N/2) = -w^k
__device__ __forceinline__ cplx wpow(const cplx* __restrict__ root, uint32_t e, int N) {
  const uint32_t h = (uint32_t)N / 2;
  const cplx r = root[e < h ? e : e - h];
  return e < h ? r : make_double2(-r.x, -r.y);
}

// One pass: COLS sub-DFTs of C points per block.  Column pass (ROW false):
// unit u = column s2, element s1 at N2 s1 + s2, result times w^(s2 i1) back in
// place.  Row pass: unit u = row i1, element s2 at N2 i1 + s2, result i2 to
// out[i1 + N1 i2].
template <bool ROW>
__global__ __launch_bounds__(ET) void k_enc_fft(cplx* __restrict__ v, cplx* __restrict__ out,
                                                const cplx* __restrict__ root, int N, int N1, int N2, int logC,
                                                int COLS) {
  extern __shared__ cplx sh[];
  const int C = 1 << logC;
  const size_t b = blockIdx.y;
  const int u0 = blockIdx.x * COLS;
  cplx* vb = v + b * (size_t)N;
  const int total = COLS * C;
  // load, bit-reversed inside each unit; consecutive threads read consecutive words
  for (int t = threadIdx.x; t < total; t += ET) {
    int col, e;
    size_t g;
    if (ROW) {
      col = t / C;
      e = t % C;
      g = (size_t)N2 * (u0 + col) + e;
    } else {
      col = t % COLS;
      e = t / COLS;
      g = (size_t)N2 * e + u0 + col;
    }
    sh[col * C + brev_bits((uint32_t)e, logC)] = vb[g];
  }
  __syncthreads();
  // radix-2 stages, twiddles w_C^k = w^(k N / C)
  const int half_total = COLS * (C / 2);
  for (int len = 2; len <= C; len <<= 1) {
    const int half = len / 2;
    const int tstep = N / len;
    for (int t = threadIdx.x; t < half_total; t += ET) {
      const int col = t / (C / 2);
      const int bi = t % (C / 2);
      const int k = bi % half;
      const int i = (bi / half) * len + k;
      cplx* s = sh + col * C;
      const cplx w = root[k * tstep];
      const cplx x0 = s[i], x1 = cmul(s[i + half], w);
      s[i] = cadd(x0, x1);
      s[i + half] = csub(x0, x1);
    }
    __syncthreads();
  }
  // store
  for (int t = threadIdx.x; t < total; t += ET) {
    if (ROW) {
      const int col = t % COLS, i2 = t / COLS;   // consecutive threads: consecutive rows i1
      out[b * (size_t)N + (size_t)(u0 + col) + (size_t)N1 * i2] = sh[col * C + i2];
    } else {
      const int col = t % COLS, i1 = t / COLS;
      const uint32_t e = (uint32_t)(((uint64_t)(u0 + col) * (uint64_t)i1) % (uint64_t)N);
      vb[(size_t)N2 * i1 + u0 + col] = cmul(sh[col * C + i1], wpow(root, e, N));
    }
  }
}

// m_i = Re(twist_i * V_i) / N * scale, rounded half to even; residues of every limb
__global__ void k_enc_final(const cplx* __restrict__ V, const cplx* __restrict__ twist, double scale, int N,
                            LimbMap map, int n_limbs, const Mod* __restrict__ mods, uint64_t* __restrict__ pt,
                            int* __restrict__ flag) {
  const size_t i = blockIdx.x * (size_t)ET + threadIdx.x;
  const size_t b = blockIdx.y;
  if (i >= (size_t)N) return;
  const cplx x = V[b * (size_t)N + i], t = twist[i];
  const double m = (t.x * x.x - t.y * x.y) / (double)N * scale;
  int64_t r = 0;
  if (fabs(m) < 9.2e18)
    r = (int64_t)rint(m);
  else
    *flag = 1;
  uint64_t* out = pt + b * (size_t)n_limbs * N;
  for (int l = 0; l < n_limbs; ++l) {
    const Mod md = mods[lm_mod(map, l)];
    const uint64_t a = r >= 0 ? reduce128((u128)(uint64_t)r, md) : md.q - 1 - reduce128((u128)(uint64_t)(-(r + 1)), md);
    out[(size_t)l * N + i] = a;
  }
}

static void ensure_enc_tables(ckks_ctx* c) {
  if (c->enc_root) return;
  std::vector<double> root, twist;
  std::vector<uint32_t> pos;
  encode_tables(c->N, root, twist, pos);
  HIPCHECK(hipMalloc(&c->enc_root, root.size() * 8));
  HIPCHECK(hipMemcpy(c->enc_root, root.data(), root.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMalloc(&c->enc_twist, twist.size() * 8));
  HIPCHECK(hipMemcpy(c->enc_twist, twist.data(), twist.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMalloc(&c->enc_pos, pos.size() * 4));
  HIPCHECK(hipMemcpy(c->enc_pos, pos.data(), pos.size() * 4, hipMemcpyHostToDevice));
  HIPCHECK(hipMalloc(&c->enc_flag, sizeof(int)));
}

static void launch_pass(ckks_ctx* c, bool row, cplx* v, cplx* out, int n_pt, int N1, int N2) {
  const int C = row ? N2 : N1;
  const int units = row ? N1 : N2;
  int logC = 0;
  while ((1 << logC) < C) ++logC;
  int cols = ENC_LDS / (int)(C * sizeof(cplx));
  if (cols > units) cols = units;
  if (cols < 1 || units % cols) FICGCN_THROW(EINVAL_, "encoder FFT shape");
  const dim3 grid(units / cols, n_pt);
  const size_t lds = (size_t)cols * C * sizeof(cplx);
  if (row)
    hipLaunchKernelGGL(k_enc_fft<true>, grid, dim3(ET), lds, c->stream, v, out, (const cplx*)c->enc_root, c->N, N1, N2,
                       logC, cols);
  else
    hipLaunchKernelGGL(k_enc_fft<false>, grid, dim3(ET), lds, c->stream, v, out, (const cplx*)c->enc_root, c->N, N1,
                       N2, logC, cols);
  HIPCHECK(hipGetLastError());
}

void encode_gpu(ckks_ctx* c, const double* re, const double* im, size_t count, size_t n, double scale, int n_limbs,
                LimbMap map, uint64_t* dev) {
  if (count == 0) return;
  if (n > (size_t)c->N / 2) FICGCN_THROW(EINVAL_, "more values than slots");
  if (!re && n > 0) FICGCN_THROW(EINVAL_, "null slot values");
  ensure_enc_tables(c);
  const int N = c->N;
  int l1 = 0;
  while ((1 << (2 * (l1 + 1))) <= N) ++l1;   // N1 = 2^floor(log N / 2)
  const int N1 = 1 << l1, N2 = N / N1;
  // chunks of plaintexts: slot values, the FFT buffer and its natural-order output
  const size_t CH = 32;
  const size_t nn = n > 0 ? n : 1;
  double* d_re = (double*)dev_scratch(c, 17, CH * nn * 8 * (im ? 2 : 1));
  double* d_im = im ? d_re + CH * nn : nullptr;
  cplx* v = (cplx*)dev_scratch(c, 18, CH * (size_t)N * sizeof(cplx));
  cplx* V = (cplx*)dev_scratch(c, 19, CH * (size_t)N * sizeof(cplx));
  HIPCHECK(hipMemsetAsync(c->enc_flag, 0, sizeof(int), c->stream));
  for (size_t b0 = 0; b0 < count; b0 += CH) {
    const int nb = (int)std::min(CH, count - b0);
    if (n > 0) {
      HIPCHECK(hipMemcpyAsync(d_re, re + b0 * n, (size_t)nb * n * 8, hipMemcpyHostToDevice, c->stream));
      if (im) HIPCHECK(hipMemcpyAsync(d_im, im + b0 * n, (size_t)nb * n * 8, hipMemcpyHostToDevice, c->stream));
    }
    hipLaunchKernelGGL(k_enc_scatter, dim3((N / 2 + ET - 1) / ET, nb), dim3(ET), 0, c->stream, d_re, d_im, n,
                       c->enc_pos, v, N);
    HIPCHECK(hipGetLastError());
    launch_pass(c, false, v, nullptr, nb, N1, N2);
    launch_pass(c, true, v, V, nb, N1, N2);
    uint64_t* pt = dev + b0 * (size_t)n_limbs * N;
    hipLaunchKernelGGL(k_enc_final, dim3((N + ET - 1) / ET, nb), dim3(ET), 0, c->stream, V, (const cplx*)c->enc_twist,
                       scale, N, map, n_limbs, c->t.mods, pt, c->enc_flag);
    HIPCHECK(hipGetLastError());
    ntt_fwd(c, pt, n_limbs, map, nb, (size_t)n_limbs * N);
    // the host slot values of this chunk are re-read by the next chunk's copy only after this point
    HIPCHECK(hipStreamSynchronize(c->stream));
  }
  int flag = 0;
  HIPCHECK(hipMemcpy(&flag, c->enc_flag, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) FICGCN_THROW(ESCALE_, "encoded coefficient exceeds 63 bits");
}

}  // namespace ficgcn
