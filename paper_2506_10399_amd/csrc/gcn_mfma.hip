// Fused Inter-CA aggregation + combination with the contraction on the
// int8 matrix cores.
//
// For one output group (F' <= 16 columns) the pass computes
//   H_l = sum_k P_k (.) T_{k,l},   T_{k,l} = sum_f w_{f,l} X_{k*F + f}   (Inter-CA, K > 0)
//   H_l = sum_f w_{f,l} X_f                                              (combination, K = 0)
// in one read of the inputs: the Inter-CA aggregation of Sec. 3.3.2 fused
// with the one-column-per-ciphertext combination of App. B.  Modular
// arithmetic is a ring, so applying P_k after the contraction gives the same
// residues as sum_f w_{f,l} (sum_k P_k (.) X_{k,f}).
//
// The contraction over f is, per wave, a dense [16 coefficients x F] x
// [F x 16 columns] product computed exactly in integers: an input residue
// x (< 2^50) and a signed integer weight w (|w| < 2^55) are written in
// balanced base-256 digits in [-128, 127],
//   x = sum_{a<7} x_a 256^a,   w = sum_{b<7} w_b 256^b,
// so sum_f x_f w_f = sum_{s<13} 256^s D_s with D_s = sum_{a+b=s} sum_f x_{a,f} w_{b,f}.
// Each digit pair (a, b) is one v_mfma_i32_16x16x64_i8 over 64 features into
// the i32 accumulator of diagonal s = a + b; |D_s| <= 7 * 2^14 * F stays below
// 2^31 for F <= 16384.  After the features of one copy the diagonals are
// folded to residues, T = sum_s [D_s]_q [256^s]_q mod q, and P_k (.) T is
// added to the output residues.
//
// Wave layout: one wave owns 16 consecutive coefficients j of one limb of one
// component and loops over the copies k and 64-feature blocks.  Lane
// (r = lane % 16, g = lane / 16) reads coefficient j0 + r of features
// 16g .. 16g+15 of each block; the digit planes of those 16 words are its A
// operands.  The B operands (weight digit planes) are laid out per block on
// the host in the same lane order.  The output tile lands as lane
// (n = lane % 16, g): column n, coefficients j0 + 4g .. j0 + 4g + 3.
#include "internal.h"

namespace ficgcn {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int MW = 256;   // 4 waves per workgroup
constexpr uint64_t DIG_C = 0x0080808080808080ull;   // 128 in each of bytes 0..6

// balanced base-256 digits of x (requires x + DIG_C in [0, 2^56)):
// byte a of the result is digit a as an int8, byte 7 is zero
__device__ __forceinline__ uint64_t bal_digits(uint64_t x) { return (x + DIG_C) ^ DIG_C; }

// 4 x 4 byte transpose: out[a] byte u = byte a of s[u].  v_perm_b32 picks
// bytes 0..3 from its second operand and 4..7 from its first.
__device__ __forceinline__ void byte_transpose(const uint32_t (&s)[4], uint32_t (&o)[4], int n_out) {
  const uint32_t t0 = __builtin_amdgcn_perm(s[1], s[0], 0x06020400u);   // s0.b0 s1.b0 s0.b2 s1.b2
  const uint32_t t1 = __builtin_amdgcn_perm(s[1], s[0], 0x07030501u);   // s0.b1 s1.b1 s0.b3 s1.b3
  const uint32_t t2 = __builtin_amdgcn_perm(s[3], s[2], 0x06020400u);
  const uint32_t t3 = __builtin_amdgcn_perm(s[3], s[2], 0x07030501u);
  o[0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
  o[1] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
  o[2] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
  if (n_out > 3) o[3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
}

// 16 words -> 7 digit planes: plane a, dword w holds digit a of words 4w..4w+3
// (byte u = word 4w+u); this fills dword w of every plane
__device__ __forceinline__ void digit_planes_w(const uint64_t (&x)[16], v4i (&A)[7], int w) {
  uint32_t lo[4], hi[4], o[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const uint64_t d = bal_digits(x[4 * w + u]);
    lo[u] = (uint32_t)d;
    hi[u] = (uint32_t)(d >> 32);
  }
  byte_transpose(lo, o, 4);
#pragma unroll
  for (int a = 0; a < 4; ++a) A[a][w] = (int)o[a];
  byte_transpose(hi, o, 3);   // byte 7 of a digit word is zero: three planes
#pragma unroll
  for (int a = 0; a < 3; ++a) A[4 + a][w] = (int)o[a];
}

template <bool STRIDED>
__global__ __launch_bounds__(MW) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_fused_mfma(OutList out, int n_out, const uint64_t* __restrict__ in_base,
                                                   size_t in_stride, const uint64_t* const* __restrict__ in_ptrs,
                                                   PtrList pts, int K, int F, int n_fb, int l1,
                                                   const v4i* __restrict__ wd, const uint64_t* __restrict__ pow256,
                                                   int log_n, const Mod* __restrict__ mods) {
  const int lane = threadIdx.x & 63;
  const size_t N = (size_t)1 << log_n;
  const size_t tiles = N >> 4;
  // wave-uniform indices (scalar registers): the wave's number within the grid
  const size_t wave = (size_t)blockIdx.x * (MW / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const size_t tile = wave % tiles;
  const int rest = (int)(wave / tiles);
  const int i = rest % l1, comp = rest / l1;
  const int r = lane & 15, g = lane >> 4;
  const size_t limb_off = ((size_t)comp * l1 + i) * N;
  const size_t off = limb_off + tile * 16 + r;
  const Mod m = mods[i];
  const bool q50 = m.q > (1ull << 49) && m.q < (1ull << 50);
  const int KK = K > 0 ? K : 1;
  const int n_steps = KK * n_fb;   // (copy, block) steps, block-fastest
  // Strided inputs are read with buffer loads: one wave-uniform resource per
  // step in scalar registers, based at the step's first feature (copy k,
  // feature 64 fb) and ranging over the features of the block below F, and a
  // fixed per-lane byte offset per load e: feature 16 g + e of the block,
  // coefficient `off`.  Features past F, and steps past the end (empty
  // range), read 0, so the prefetch is issued unconditionally and the wait
  // counts stay static.
  const size_t feat_bytes = in_stride * 8;
  uint32_t voff[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) voff[e] = STRIDED ? (uint32_t)(((size_t)(g * 16 + e) * in_stride + off) * 8) : 0u;
  auto block_rsrc = [&](int k, int fb, bool live) {
    const int nf = live ? (F - fb * 64 < 64 ? F - fb * 64 : 64) : 0;
    const char* b = (const char*)in_base + ((size_t)k * F + (size_t)fb * 64) * feat_bytes;
    return __builtin_amdgcn_make_buffer_rsrc((void*)b, 0, (int)((size_t)nf * feat_bytes), 0x00020000);
  };
  // words e0 .. e0+n-1 of a block
  auto load_words = [&](uint64_t (&x)[16], __amdgpu_buffer_rsrc_t rs, int k, int fb, bool live, int e0, int n) {
#pragma unroll
    for (int e = e0; e < e0 + n; ++e) {
      if (STRIDED) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff[e], 0, 2);   // read once: nontemporal
        x[e] = ((uint64_t)w[1] << 32) | w[0];
      } else {
        const int f = fb * 64 + e + g * 16;
        x[e] = live && f < F ? in_ptrs[(size_t)k * F + f][off] : 0;
      }
    }
  };
  const uint64_t* pw = pow256 + (size_t)i * 13;
  uint64_t h[4] = {0, 0, 0, 0};   // output residues: column lane % 16, coefficients j0 + 4g + rr
  v4i acc[13];
#pragma unroll
  for (int s = 0; s < 13; ++s) acc[s] = v4i{0, 0, 0, 0};
  uint64_t xa[16], xb[16];
  {
    const auto rs0 = block_rsrc(0, 0, n_steps > 0);
    load_words(xa, rs0, 0, 0, n_steps > 0, 0, 16);
  }
  // (copy, block) of the current step, advanced without divisions
  int k = 0, fb = 0;
  for (int step = 0; step < n_steps; step += 2) {
    // two steps per iteration so the register buffers alternate statically
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int st = step + half;
      if (st >= n_steps) break;
      uint64_t (&cur)[16] = half ? xb : xa;
      uint64_t (&nxt)[16] = half ? xa : xb;
      const bool last = fb == n_fb - 1;
      const int kn = last ? k + 1 : k, fbn = last ? 0 : fb + 1;
      // this step's weight planes (and the copy's plaintext words on its last
      // block) are requested before the next block: loads retire in order, so
      // waiting for them leaves the prefetch in flight
      v4i B[7];
#pragma unroll
      for (int b = 0; b < 7; ++b) B[b] = wd[((size_t)fb * 7 + b) * 64 + lane];
      uint64_t pk[4] = {1, 1, 1, 1};
      if (K > 0 && last) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) pk[rr] = pts.p[k][(size_t)i * N + tile * 16 + 4 * g + rr];
      }
      // keep the order: these loads, then the prefetch spread over the digit
      // planes of this block and the first matrix products (two words at a time)
      __builtin_amdgcn_sched_barrier(0);
      const bool nlive = st + 1 < n_steps;
      const auto rs = block_rsrc(kn, fbn, nlive);
      v4i A[7];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        load_words(nxt, rs, kn, fbn, nlive, 2 * w, 2);
        __builtin_amdgcn_sched_barrier(0);
        digit_planes_w(cur, A, w);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int b = 0; b < 7; ++b) {
#pragma unroll
        for (int a = 0; a < 7; ++a) acc[a + b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[a], B[b], acc[a + b], 0, 0, 0);
        if (b < 4) {
          __builtin_amdgcn_sched_barrier(0);
          load_words(nxt, rs, kn, fbn, nlive, 8 + 2 * b, 2);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      if (last) {
        // copy k done: fold the diagonals and add P_k (.) T
        if (q50) {
          // T = sum_d D_d [256^d]_q with the weights split as p0 + p1 2^25 (both below 2^25):
          // s0 = sum_d D_d p0_d and s1 = sum_d D_d p1_d are exact in 64 bits (13 terms below
          // 2^56 in magnitude), X = s0 + s1 2^25 lies in (-2^86, 2^86), and X + q 2^37 (a
          // multiple of q, at least 2^86 for q > 2^49) is reduced once
          uint32_t p0[13], p1[13];
#pragma unroll
          for (int d = 0; d < 13; ++d) {
            const uint64_t w = pw[d];
            p0[d] = (uint32_t)w & ((1u << 25) - 1);
            p1[d] = (uint32_t)(w >> 25);
          }
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            int64_t s0 = 0, s1 = 0;
#pragma unroll
            for (int d = 0; d < 13; ++d) {
              const int64_t v = acc[d][rr];
              s0 += v * (int64_t)p0[d];
              s1 += v * (int64_t)p1[d];
            }
            uint64_t lo = (uint64_t)s1 << 25, hi = (uint64_t)(s1 >> 39);
            const uint64_t l2 = lo + (uint64_t)s0;
            hi += (uint64_t)(s0 >> 63) + (l2 < lo ? 1u : 0u);
            lo = l2;
            const uint64_t l3 = lo + (m.q << 37);
            hi += (m.q >> 27) + (l3 < lo ? 1u : 0u);
            lo = l3;
            uint64_t t = reduce128(hi, lo, m);
            if (K > 0) t = reduce128((u128)t * pk[rr], m);
            h[rr] = add_mod(h[rr], t, m.q);
          }
        } else {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            u128 sum = 0;
#pragma unroll
            for (int d = 0; d < 13; ++d) {
              const int v = acc[d][rr];
              const uint64_t res = v >= 0 ? (uint64_t)v : m.q - (uint64_t)(-(int64_t)v);
              sum += (u128)res * pw[d];
            }
            uint64_t t = reduce128(sum, m);
            if (K > 0) t = reduce128((u128)t * pk[rr], m);
            h[rr] = add_mod(h[rr], t, m.q);
          }
        }
#pragma unroll
        for (int s = 0; s < 13; ++s) acc[s] = v4i{0, 0, 0, 0};
      }
      k = kn;
      fb = fbn;
    }
  }
  const int n = lane & 15;
  if (n >= n_out) return;
  uint64_t* o = out.p[n] + limb_off + tile * 16 + 4 * g;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) o[rr] = h[rr];
}

// ---- inputs stored as the pass's matrix operands ---------------------------
// The layer-1 inputs rearranged once into what the pass feeds the matrix
// cores: for every wave (the pass's wave order: tile, limb, component) and
// every (copy, 64-feature block) step, the digit planes of its 64 lanes.
// Digits 0..5 are full int8 planes, [plane][lane] x 16 bytes; digit 6 of a
// residue below 2^51 lies in [0, 8], so its plane is stored as 4-bit values,
// one 8-byte word per lane: byte k of the low dword holds the values of bytes
// k (low nibble) and 4 + k (high nibble) of the plane's first two dwords, the
// high dword likewise for the last two.  A step is PK_STEP_WORDS 64-bit words
// (6.5 bytes per residue instead of 8, no digit work in the pass).  Features
// past F hold zero digits.
constexpr size_t PK_STEP_WORDS = 6 * 64 * 2 + 64;

bool mfma_pack_supported(ckks_ctx* c) { return c->mod[0] < (1ull << 51); }

size_t mfma_packed_words(ckks_ctx* c, int K, int F, int level) {
  const size_t waves = ((size_t)c->N >> 4) * (size_t)(level + 1) * 2;
  const size_t steps = (size_t)(K > 0 ? K : 1) * (size_t)((F + 63) / 64);
  return waves * steps * PK_STEP_WORDS;
}

__device__ __forceinline__ uint64_t nibble_pack(v4i a) {
  const uint32_t lo = ((uint32_t)a.x & 0x0F0F0F0Fu) | (((uint32_t)a.y & 0x0F0F0F0Fu) << 4);
  const uint32_t hi = ((uint32_t)a.z & 0x0F0F0F0Fu) | (((uint32_t)a.w & 0x0F0F0F0Fu) << 4);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ v4i nibble_unpack(uint64_t v) {
  const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  return v4i{(int)(lo & 0x0F0F0F0Fu), (int)((lo >> 4) & 0x0F0F0F0Fu), (int)(hi & 0x0F0F0F0Fu),
             (int)((hi >> 4) & 0x0F0F0F0Fu)};
}

// one wave per (pass wave, step): the 16 words of each lane, their digit planes
template <bool STRIDED>
__global__ __launch_bounds__(MW) void k_mfma_pack(const uint64_t* __restrict__ in_base, size_t in_stride,
                                                  const uint64_t* const* __restrict__ in_ptrs, int K, int F, int n_fb,
                                                  int l1, int log_n, uint64_t* __restrict__ packed) {
  const int lane = threadIdx.x & 63;
  const size_t N = (size_t)1 << log_n;
  const size_t tiles = N >> 4;
  const size_t n_steps = (size_t)(K > 0 ? K : 1) * n_fb;
  const size_t gw = (size_t)blockIdx.x * (MW / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const size_t wave = gw / n_steps;
  if (wave >= tiles * (size_t)l1 * 2) return;
  const int st = (int)(gw % n_steps);
  const size_t tile = wave % tiles;
  const int rest = (int)(wave / tiles);
  const int i = rest % l1, comp = rest / l1;
  const int k = st / n_fb, fb = st % n_fb;
  const int r = lane & 15, g = lane >> 4;
  const size_t off = ((size_t)comp * l1 + i) * N + tile * 16 + r;
  uint64_t x[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int f = fb * 64 + g * 16 + e;
    x[e] = f < F ? (STRIDED ? in_base[((size_t)k * F + f) * in_stride + off] : in_ptrs[(size_t)k * F + f][off]) : 0;
  }
  v4i A[7];
#pragma unroll
  for (int w = 0; w < 4; ++w) digit_planes_w(x, A, w);
  uint64_t* step = packed + gw * PK_STEP_WORDS;
  v4i* dst = (v4i*)step + lane;
#pragma unroll
  for (int a = 0; a < 6; ++a) dst[(size_t)a * 64] = A[a];
  step[6 * 64 * 2 + lane] = nibble_pack(A[6]);
}

void mfma_pack(ckks_ctx* c, const uint64_t* in_base, size_t in_stride, const uint64_t* const* in_ptrs, int K, int F,
               int level, uint64_t* packed) {
  const int l1 = level + 1;
  const int n_fb = (F + 63) / 64;
  const size_t items = ((size_t)c->N >> 4) * l1 * 2 * (size_t)(K > 0 ? K : 1) * n_fb;
  const size_t blocks = (items + MW / 64 - 1) / (MW / 64);
  if (blocks >= ((size_t)1 << 31)) FICGCN_THROW(EINVAL_, "input block too large to rearrange in one launch");
  if (!mfma_pack_supported(c)) FICGCN_THROW(EINVAL_, "rearranged inputs need primes below 2^51");
  if (in_base)
    hipLaunchKernelGGL(k_mfma_pack<true>, dim3((unsigned)blocks), dim3(MW), 0, c->stream, in_base, in_stride, in_ptrs, K,
                       F, n_fb, l1, c->log_n, packed);
  else
    hipLaunchKernelGGL(k_mfma_pack<false>, dim3((unsigned)blocks), dim3(MW), 0, c->stream, in_base, in_stride, in_ptrs,
                       K, F, n_fb, l1, c->log_n, packed);
  HIPCHECK(hipGetLastError());
}

// The pass on rearranged inputs: per step six 16-byte plane loads and one
// 8-byte load of the top digit's nibbles (the next step's issued before this
// step's matrix products), the nibbles widened to bytes in registers, then the
// same products, folds and output as the pass on ciphertext words.
__global__ __launch_bounds__(MW) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_fused_mfma_packed(
    OutList out, int n_out, const uint64_t* __restrict__ packed, PtrList pts, int K, int n_fb, int l1,
    const v4i* __restrict__ wd, const uint64_t* __restrict__ pow256, int log_n, const Mod* __restrict__ mods) {
  const int lane = threadIdx.x & 63;
  const size_t N = (size_t)1 << log_n;
  const size_t tiles = N >> 4;
  const size_t wave = (size_t)blockIdx.x * (MW / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const size_t tile = wave % tiles;
  const int rest = (int)(wave / tiles);
  const int i = rest % l1, comp = rest / l1;
  const int g = lane >> 4;
  const size_t limb_off = ((size_t)comp * l1 + i) * N;
  const Mod m = mods[i];
  const int KK = K > 0 ? K : 1;
  const int n_steps = KK * n_fb;
  const uint64_t* src = packed + wave * (size_t)n_steps * PK_STEP_WORDS;
  const uint64_t* pw = pow256 + (size_t)i * 13;
  uint64_t h[4] = {0, 0, 0, 0};
  v4i acc[13];
#pragma unroll
  for (int s = 0; s < 13; ++s) acc[s] = v4i{0, 0, 0, 0};
  // per step: planes 0..5 as 16-byte loads, plane 6 as one 8-byte nibble word
  v4i Aa[6], Ab[6];
  uint64_t Ta, Tb;
  auto load_step = [&](int st, v4i (&A)[6], uint64_t& T) {
    const uint64_t* w = src + (size_t)st * PK_STEP_WORDS;
#pragma unroll
    for (int a = 0; a < 6; ++a) A[a] = ((const v4i*)w)[(size_t)a * 64 + lane];
    T = w[6 * 64 * 2 + lane];
  };
  load_step(0, Aa, Ta);
  int k = 0, fb = 0;
  for (int step = 0; step < n_steps; step += 2) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int st = step + half;
      if (st >= n_steps) break;
      v4i (&A6)[6] = half ? Ab : Aa;
      v4i (&An)[6] = half ? Aa : Ab;
      const uint64_t T = half ? Tb : Ta;
      uint64_t& Tn = half ? Ta : Tb;
      const bool last = fb == n_fb - 1;
      v4i B[7];
#pragma unroll
      for (int b = 0; b < 7; ++b) B[b] = wd[((size_t)fb * 7 + b) * 64 + lane];
      uint64_t pk[4] = {1, 1, 1, 1};
      if (K > 0 && last) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) pk[rr] = pts.p[k][(size_t)i * N + tile * 16 + 4 * g + rr];
      }
      __builtin_amdgcn_sched_barrier(0);
      if (st + 1 < n_steps) load_step(st + 1, An, Tn);
      __builtin_amdgcn_sched_barrier(0);
      const v4i A[7] = {A6[0], A6[1], A6[2], A6[3], A6[4], A6[5], nibble_unpack(T)};
#pragma unroll
      for (int b = 0; b < 7; ++b)
#pragma unroll
        for (int a = 0; a < 7; ++a) acc[a + b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[a], B[b], acc[a + b], 0, 0, 0);
      if (last) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          u128 sum = 0;
#pragma unroll
          for (int d = 0; d < 13; ++d) {
            const int v = acc[d][rr];
            const uint64_t res = v >= 0 ? (uint64_t)v : m.q - (uint64_t)(-(int64_t)v);
            sum += (u128)res * pw[d];
          }
          uint64_t t = reduce128(sum, m);
          if (K > 0) t = reduce128((u128)t * pk[rr], m);
          h[rr] = add_mod(h[rr], t, m.q);
        }
#pragma unroll
        for (int s = 0; s < 13; ++s) acc[s] = v4i{0, 0, 0, 0};
        k = k + 1;
        fb = 0;
      } else {
        fb = fb + 1;
      }
    }
  }
  const int n = lane & 15;
  if (n >= n_out) return;
  uint64_t* o = out.p[n] + limb_off + tile * 16 + 4 * g;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) o[rr] = h[rr];
}

void comb_mfma_packed(ckks_ctx* c, const std::vector<uint64_t*>& outs, const uint64_t* packed, const PtrList& pts, int K,
                      int F, int level, const void* wd, const uint64_t* pw, const char* prof_name) {
  ProfScope ps(c, prof_name);
  const int n_out = (int)outs.size();
  if (n_out > 16 || K > PtrList::MAX || F > 16384 || !packed) FICGCN_THROW(EINVAL_, "shape outside the matrix-core pass");
  if (!mfma_pack_supported(c)) FICGCN_THROW(EINVAL_, "rearranged inputs need primes below 2^51");
  const int l1 = level + 1;
  OutList o{};
  for (int l = 0; l < n_out; ++l) o.p[l] = outs[l];
  const int n_fb = (F + 63) / 64;
  const size_t waves = ((size_t)c->N >> 4) * l1 * 2;
  hipLaunchKernelGGL(k_fused_mfma_packed, dim3((unsigned)(waves / (MW / 64))), dim3(MW), 0, c->stream, o, n_out,
                     packed, pts, K, n_fb, l1, (const v4i*)wd, pw, c->log_n, c->t.mods);
  HIPCHECK(hipGetLastError());
}

// Weight digit planes of one 16-column group: [n_fb][7][64 lanes] x 16 bytes;
// lane (n, g), byte e holds digit b of w[f = 64 fb + 16 g + e][l0 + n] (zero
// outside F x F').  Returns false when a weight is outside the digit range.
bool mfma_weight_planes(const std::vector<int64_t>& w_int, int F, int F_out, int l0, std::vector<uint8_t>& planes,
                        int& n_fb) {
  n_fb = (F + 63) / 64;
  planes.assign((size_t)n_fb * 7 * 64 * 16, 0);
  for (int f = 0; f < F; ++f)
    for (int n = 0; n < 16 && l0 + n < F_out; ++n) {
      const int64_t w = w_int[(size_t)f * F_out + l0 + n];
      const int64_t lim = (int64_t)DIG_C;
      if (w < -lim || w >= (int64_t)(1ull << 56) - lim) return false;
      const uint64_t d = ((uint64_t)w + DIG_C) ^ DIG_C;
      const int fb = f / 64, g = (f % 64) / 16, e = f % 16;
      const int lane = g * 16 + n;
      for (int b = 0; b < 7; ++b) planes[(((size_t)fb * 7 + b) * 64 + lane) * 16 + e] = (uint8_t)(d >> (8 * b));
    }
  return true;
}

// 256^s mod q_i, s < 13, for the limbs of one level: [l1][13]
void mfma_pow256(ckks_ctx* c, int l1, std::vector<uint64_t>& out) {
  out.resize((size_t)l1 * 13);
  for (int i = 0; i < l1; ++i) {
    const uint64_t q = c->mod[i];
    uint64_t v = 1;
    for (int s = 0; s < 13; ++s) {
      out[(size_t)i * 13 + s] = v;
      v = (uint64_t)((u128)v * 256 % q);
    }
  }
}

constexpr int MFMA_MAX_K = PtrList::MAX;

bool mfma_supported(ckks_ctx* c, int K, int F, int F_out) {
  return c->mod[0] < (1ull << 52) && K <= MFMA_MAX_K && F <= 16384 && F_out <= 16 && c->log_n >= 6;
}

// outs: F' <= 16 buffers [2][l+1][N]; wd: digit planes of this group; pw: [l1][13] on the device
void comb_mfma(ckks_ctx* c, const std::vector<uint64_t*>& outs, const uint64_t* in_base, size_t in_stride,
               const uint64_t* const* in_dev_ptrs, const PtrList& pts, int K, int F, int level, const void* wd,
               const uint64_t* pw, const char* prof_name) {
  ProfScope ps(c, prof_name);
  const int n_out = (int)outs.size();
  if (n_out > 16 || K > MFMA_MAX_K || F > 16384 || (in_base && in_stride >= ((size_t)1 << 22)))
    FICGCN_THROW(EINVAL_, "shape outside the matrix-core pass");
  const int l1 = level + 1;
  OutList o{};
  for (int l = 0; l < n_out; ++l) o.p[l] = outs[l];
  const int n_fb = (F + 63) / 64;
  const size_t waves = ((size_t)c->N >> 4) * l1 * 2;
  dim3 grid((unsigned)(waves / (MW / 64)));
  if (in_base)
    hipLaunchKernelGGL(k_fused_mfma<true>, grid, dim3(MW), 0, c->stream, o, n_out, in_base, in_stride, in_dev_ptrs, pts,
                       K, F, n_fb, l1, (const v4i*)wd, pw, c->log_n, c->t.mods);
  else
    hipLaunchKernelGGL(k_fused_mfma<false>, grid, dim3(MW), 0, c->stream, o, n_out, in_base, in_stride, in_dev_ptrs,
                       pts, K, F, n_fb, l1, (const v4i*)wd, pw, c->log_n, c->t.mods);
  HIPCHECK(hipGetLastError());
}

}  // namespace ficgcn
