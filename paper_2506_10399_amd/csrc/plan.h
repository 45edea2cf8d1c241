// Plan object of the encrypted GCN (library side).
#pragma once
#include <vector>

#include "internal.h"

namespace ficgcn {

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
  // schedule
  int level_in = 0, level_agg = 0, level_out = 0, n_rescale_comb = 0;
  double scale_in = 0, sP = 0, sW = 0, sM = 0, scale_agg = 0, scale_out = 0;
  bool squared_out = false;
  std::vector<int64_t> w_int;      // [f_in][f_out]
  // operands on the device: Inter-CA: K plaintexts at level_in;
  // SpIntra-CA: n_packed * n_shifts masks at level_agg
  int op_level = 0;
  double op_scale = 0;
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
  int n_packed() const { return kind == 0 ? f_out : (f_out + t - 1) / t; }
  int n_in_cts() const { return kind == 0 ? K * f_in : f_in; }
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
  ~ficgcn_plan();
};

namespace ficgcn {
// operand slot vector i of layer li (M doubles)
void plan_operand_slots(const ficgcn_plan* p, int li, size_t i, std::vector<double>& out);
size_t plan_operand_count(const ficgcn_plan* p, int li);
void run_layer(ckks_ctx* c, const ckks_keys* ek, ficgcn_plan* p, int li, const uint64_t* const* in, size_t n_in,
               uint64_t* const* out, size_t n_out, int mode);
// frees the plan's device memory (operands and layer constants); the plan can be encoded again
void release_plan_device(ficgcn_plan* p);
// device bytes the plan's operands take once encoded
size_t plan_operand_bytes(const ficgcn_plan* p);
}  // namespace ficgcn
