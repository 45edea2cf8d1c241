// Batched key switching and batched ciphertext kernels (ks_batch.hip).
#pragma once
#include <vector>

#include "internal.h"

namespace ficgcn {

// One key switch of a batch.  With acc = sum_d sigma_g(D_{src,d}) * key_d over
// Q_l and P (D = ModUp of source `src`), the switched ciphertext is
//   KS = ( ModDown(acc_0) + sigma_g(add0),  ModDown(acc_1) + add1 )
// (a missing add term counts as zero).  Jobs are grouped: the group output
// receives the sum over its jobs of KS, or of KS (.) pt when pt is set.
struct KSJob {
  const uint64_t* key;    // [beta][2][L+alpha][N]
  const uint64_t* add0;   // [l+1][N] or null; read through sigma_g (a rotation's c0)
  const uint64_t* add1;   // [l+1][N] or null
  const uint64_t* pt;     // [l+1][N] or null: plaintext multiplied into KS
  uint64_t g;             // Galois element (1: no automorphism)
  int32_t src;            // index into the batch's sources
  int32_t grp;            // output group; jobs are sorted by group
};

struct TensorJob {
  const uint64_t* x;
  const uint64_t* y;
  uint64_t* d;            // [3][l+1][N]
};

struct MacTerm {
  const uint64_t* ct;     // [2][l+1][N], or [2][l1][N] when l1 is set
  const uint64_t* pt;     // [l+1][N], null = plain addition
  int64_t l1 = 0;         // limbs per component of ct (0: l+1); a larger value reads ct dropped to level l
};

// sources: polynomials [l+1][N] in evaluation form (a ciphertext's c1 or a
// tensor product's d2).  outs[grp] (accumulate ? += : =) the group's sum;
// every group in [0, outs.size()) is written, a group without jobs with 0
// (or left as it is when accumulating).
void keyswitch_batch(ckks_ctx* c, int level, const std::vector<const uint64_t*>& sources,
                     const std::vector<KSJob>& jobs, const std::vector<uint64_t*>& outs, bool accumulate);
// Masked sums of key switches with one ModDown per output (double hoisting):
// for every output group, A = sum over its jobs of acc_r (.) pt_r on the key
// basis (pt_r: [l+1+alpha][N], Q_l limbs then P limbs), then
//   out_grp (+)= ( ModDown(A_0) + sum_r sigma_g(add0_r) (.) pt_r,  ModDown(A_1) ).
// A job without pt is taken unmasked (the plain sum of its rotation: the
// giant steps of the baby-step/giant-step form); add1 is ignored.
void keyswitch_masked_sum(ckks_ctx* c, int level, const std::vector<const uint64_t*>& sources,
                          const std::vector<KSJob>& jobs, const std::vector<uint64_t*>& outs, bool accumulate);
void tensor_batch(ckks_ctx* c, int level, const std::vector<TensorJob>& jobs);
// rounding rescale of each ciphertext in place ([2][l+1][N] -> [2][l][N])
void rescale_batch(ckks_ctx* c, int level, const std::vector<uint64_t*>& cts);
// two rescales in a row (level, then level - 1) in one pass over the limbs;
// the same words as two rescale_batch calls
void rescale2_batch(ckks_ctx* c, int level, const std::vector<uint64_t*>& cts);
// a term of a sum over up to four ciphertexts under one shared plaintext
struct MacTermNP {
  enum { MAX = 4 };
  const uint64_t* ct[MAX];   // [2][l+1][N] each
  const uint64_t* pt;        // [l+1][N], null = plain addition
};
// outs[g * np + c] (accumulate ? += : =) sum over groups[g]'s terms of ct[c] (.) pt
void group_mac_np(ckks_ctx* c, int level, int np, const std::vector<std::vector<MacTermNP>>& groups,
                  const std::vector<uint64_t*>& outs, bool accumulate);
// outs[g] (accumulate ? += : =) sum of groups[g]'s terms
void group_mac(ckks_ctx* c, int level, const std::vector<std::vector<MacTerm>>& groups,
               const std::vector<uint64_t*>& outs, bool accumulate);

}  // namespace ficgcn
