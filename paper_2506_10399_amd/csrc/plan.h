// Plan object of the encrypted GCN (library side).
#pragma once
#include <vector>

#include "internal.h"

namespace ficgcn {

// Radix-2 SpIntra-CA program (paper Sec. 3.3, CPOO of Sec. 3.3.1): working
// ciphertexts ("registers") stepped round by round through masks.
struct R2Term {
  int dst = -1;                    // Keep/Move term: register written; Fin term: -1
  int64_t m = 0;                   // rotation amount of the source register (0: none)
  std::vector<int32_t> slot;       // block-local slots, ascending
  std::vector<double> val;         // mask values at those slots
};
struct R2Step {
  int lane = 0, r0 = 0, r1 = 0;    // rounds [r0, r1)
  int depth = 0;                   // levels below the aggregation level of the source register
  int src = 0;                     // register read (0 = the packed input)
  std::vector<R2Term> keep;        // by (dst, m)
  std::vector<R2Term> fin;         // by m
};
struct R2Program {
  R2Term self;                     // the self terms, multiplied into the input
  std::vector<R2Step> steps;
  std::vector<int> reg_depth;      // per register
  int depth = 1;                   // levels the aggregation consumes
  int n_lanes = 0;
  int64_t n_moved = 0;
  // operand j: step (-1 = self), term index (keep first, then fin), depth
  struct Ref { int step, term, depth; };
  std::vector<Ref> ops;
};
// The program of one packed layout: node order pi, CSR adjacency (diagonal
// included), M slots, column block B (wrap: t = 1, shifts AOO-reduced),
// CPOO threshold theta (0 = off).
void build_radix2(const std::vector<int32_t>& pi, const std::vector<int32_t>& rowptr, const std::vector<int32_t>& col,
                  const std::vector<double>& val, int M, int B, bool wrap, double theta, R2Program& out);

struct LayerPlan {
  int kind = 0;              // 0 = Inter-CA (client copies), 1 = SpIntra-CA
  int f_in = 0, f_out = 0;
  bool act = false;
  // Inter-CA
  int K = 0;
  std::vector<int> copy_src;       // [K][n_v], -1 = none
  std::vector<double> copy_val;    // [K][n_v]
  // SpIntra-CA
  int t = 1, B = 0;
  std::vector<int64_t> shifts;     // sorted distinct
  int family = 1, G = 1;
  std::vector<int64_t> pack_steps; // sorted distinct, negative
  R2Program r2;                    // family 3
  double cpoo = 0;                 // family 3: CPOO threshold (0 = off)
  // Inter-CA packing: 0 = one input column per ciphertext (weights as integer sums), 1 = the
  // case-1 layout of Sec. 3.2 / App. B (t input columns per ciphertext, each repeated for the
  // F' output columns in blocks of B slots; operands A_hat_k (x) W-slice, ceil(log2 t) folds)
  int pack = 0;
  std::vector<int64_t> fold_steps;
  // SpIntra-CA combination: 0 = columns by integer weights then packed by rotations, 1 = input
  // already packed in blocks of B, output block c = sum over s of Rot_{sB}(in) (.) cm_s
  int comb = 0;
  std::vector<int64_t> comb_shifts;
  std::vector<double> w;           // [f_in][f_out] weights (case-1 operands, combination masks)
  // Sec. 3.3.2's aggregation-mode formula (later layers): -1 not evaluated, 0 Inter-CA, 1 SpIntra-CA
  int paper_mode = -1;
  double mode_cost_inter = 0, mode_cost_spintra = 0;
  // schedule
  int level_in = 0, level_agg = 0, level_out = 0, n_rescale_comb = 0;
  double scale_in = 0, sP = 0, sW = 0, sM = 0, scale_agg = 0, scale_out = 0;
  bool squared_out = false;
  std::vector<int64_t> w_int;      // [f_in][f_out]
  // operands on the device: Inter-CA: K plaintexts at level_in;
  // SpIntra-CA: n_packed * n_shifts masks at level_agg
  int op_level = 0;
  double op_scale = 0;
  std::vector<char> op_x;          // operand on the key basis (level+1+alpha limbs): family 4 masks,
                                   // the nonzero-offset block-combination masks
  std::vector<int32_t> op_alias;   // operand whose memory this one shares (-1: its own): the masks of
                                   // packed ciphertexts with as many columns as the first one are equal
  std::vector<int32_t> op_lv;      // level of each operand
  std::vector<size_t> op_off;      // word offset of each operand in ops_block
  size_t op_words = 0;
  std::vector<uint64_t*> ops;
  uint64_t* ops_block = nullptr;   // one allocation for all operands
  // device constants for the fused kernels (built on first use)
  uint64_t* w_dev = nullptr;       // [f_out][f_in][level+1][2] residues + Shoup (per-operation form)
  void* wf_dev = nullptr;          // fused-pass weights [level+1][f_in][f_out] (split halves or residues)
  bool wf_split = false;
  // matrix-core pass: weight digit planes per 16-column group, 256^s mod q_i
  int wm_state = 0;                // 0 not built, 1 built, -1 shape or weights outside the pass
  uint8_t* wm_dev = nullptr;       // [groups][n_fb][7][64][16]
  size_t wm_group_bytes = 0;
  uint64_t* pw_dev = nullptr;      // [level+1][13]
  // inputs rearranged as the matrix-core pass's operands (caller-owned buffer,
  // registered by ficgcn_plan_pack_inputs; read when the layer is called
  // without input ciphertexts)
  const uint64_t* packed_in = nullptr;
  int n_packed() const { return kind == 0 ? (pack ? 1 : f_out) : (f_out + t - 1) / t; }
  int n_in_cts() const { return kind == 0 ? K * (pack ? (f_in + t - 1) / t : f_in) : (comb ? 1 : f_in); }
  size_t n_agg_ops() const;        // aggregation masks (SpIntra-CA): the first operands of the layer
};

}  // namespace ficgcn

namespace ficgcn {
// One layer's batched launch sequence captured in a HIP graph, for fixed
// input and output buffers.
struct LayerGraph {
  std::vector<const uint64_t*> in;
  std::vector<uint64_t*> out;
  const ckks_keys* keys = nullptr;
  ckks_ctx* ctx = nullptr;
  Recorder rec;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool failed = false;   // capture not possible: the layer runs eagerly
  ~LayerGraph();
};
}  // namespace ficgcn

struct ficgcn_plan {
  ckks_ctx* ctx = nullptr;
  std::vector<std::unique_ptr<ficgcn::LayerGraph>> graphs;   // per layer, built on first graph-mode call
  int n_v = 0, M = 0, B_pi = 0;
  std::vector<int32_t> pi;
  std::vector<int32_t> rowptr, col;
  std::vector<double> val;
  std::vector<std::vector<int>> regions;
  std::vector<ficgcn::LayerPlan> layers;
  std::vector<int64_t> rot_steps;
  bool low_level = false;    // inputs at the lowest level the layers need
  ~ficgcn_plan();
};

namespace ficgcn {
// operand slot vector i of layer li (M doubles)
void plan_operand_slots(const ficgcn_plan* p, int li, size_t i, std::vector<double>& out);
size_t plan_operand_count(const ficgcn_plan* p, int li);
// level and encoding scale of operand i of layer li
int plan_operand_level(const ficgcn_plan* p, int li, size_t i);
double plan_operand_scale(const ficgcn_plan* p, int li, size_t i);
// operand i held on the key basis (level+1+alpha limbs: Q_l residues, then the special primes')
bool plan_operand_ext(const ficgcn_plan* p, int li, size_t i);
void run_layer(ckks_ctx* c, const ckks_keys* ek, ficgcn_plan* p, int li, const uint64_t* const* in, size_t n_in,
               uint64_t* const* out, size_t n_out, int mode);
// frees the plan's device memory (operands and layer constants); the plan can be encoded again
void release_plan_device(ficgcn_plan* p);
// builds every table the layers would build on first use, so that running the plan only reads it
// (several requests may then run one plan at once)
void prepare_plan_device(ckks_ctx* c, ficgcn_plan* p);
// rotation steps a layer's batched execution switches keys for
std::vector<int64_t> layer_rotation_steps(const LayerPlan& lp);
// device bytes the plan's operands take once encoded
size_t plan_operand_bytes(const ficgcn_plan* p);
}  // namespace ficgcn
