// Host-side plan of one factorization: the recursion of Algorithms 1-3 unrolled
// into an ordered list of kernel launches with their descriptor arrays.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mpchol.h"
#include "internal.h"

namespace mpc {

struct Launch {
  enum Kind { POTRF, TRSM, MAXABS, CAST, GEMM, TRINV, INVJOIN } kind;
  int prec;
  int64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;  // POTRF / TRINV: i0, m (POTRF a2 = 1: also
                                          // the inverse); TRSM: r0, m, c0, k;
                                          // CAST: a0 = 1 single-pass (scale 1 + max-abs)
  int first = 0, count = 0, total = 0;    // descriptor range, workgroups; POTRF / TRINV /
                                          // TRSM / INVJOIN: leaf-inverse slot (TRSM: -1 =
                                          // substitution)
  int64_t off = 0;                        // POTRF / TRINV / TRSM: element offset in the slot
                                          // (INVJOIN: a0 = i0, a1 = m, a2 = m1)
  int tile = 128;                         // GEMM output tile (32, 64, 128 or 256)
  // Lookahead (single-matrix path): side = 1 runs the launch on the side
  // stream once the caller's stream has reached it; wait_side = 1 makes the
  // caller's stream wait for the side stream's work before this launch.
  int side = 0, wait_side = 0;
};

struct PlanStats {
  double flops[4] = {0, 0, 0, 0};  // GEMM/SYRK flops by precision (E4M3, F16, F32, F64)
  double leaf_flops = 0;           // leaf POTRF + leaf TRSM
  double cast_bytes = 0;           // algorithmic bytes of quantize casts
  int64_t n_launch = 0;
};

constexpr int kInvLd = 2 * kKernelLeaf;   // leaf-inverse slot: up to two joined kernel leaves

struct Plan {
  int64_t n = 0, ldl = 0;
  mpchol_tree tree{};
  std::vector<int8_t> node_prec;
  std::vector<Launch> launches;
  std::vector<MaxabsJob> maxabs;
  std::vector<CastJob> casts;
  std::vector<GemmProb> gemms;
  size_t ws_bytes = 0;     // quantized-operand workspace needed
  int64_t parts = 0;       // maxabs partial slots needed
  int ninv = 0;            // leaf-inverse slots (kInvLd x kInvLd doubles each)
  int64_t split1 = 0;      // order of the top-level A11 (0: the root is a leaf)
  int first_outer = -1;    // first launch that touches rows >= split1
  int n_side = 0;          // launches on the side stream (lookahead tails)
  PlanStats stats;
  // device copies of the descriptor arrays
  MaxabsJob* d_maxabs = nullptr;
  CastJob* d_casts = nullptr;
  GemmProb* d_gemms = nullptr;
};

// Validates the descriptor; returns 0 or a negative/positive mpchol code.
int validate_tree(const mpchol_tree* t);
std::string plan_key(int64_t n, int64_t ldl, const mpchol_tree* t);
// single_wg: the plan runs inside one workgroup (batched executor); GEMM
// tiles are chosen for per-workgroup efficiency instead of chip occupancy.
// tile: 0 automatic, 64 or 128 forces the GEMM output tile.
// lookahead: split each Tree-SYRK of Algorithm 1 into the part that updates
// A22's leading block (the block Tree-POTRF(A22) factors first) and the rest,
// run the rest on a side stream while the leading block is factored, and join
// before the Tree-TRSM of A22 (one tail in flight at a time; its operand
// copies live in a second workspace bank).  lookahead 1: every Tree-SYRK;
// 2: only FP32 / FP64 ones (FP16 / E4M3 GEMMs never share the GPU); 0: off.
// Ignored with single_wg.
void build_plan(Plan& P, int64_t n, int64_t ldl, const mpchol_tree* t, bool single_wg = false,
                int tile = 0, int lookahead = 0);
int64_t split_rule(int64_t m, int32_t align);
// The block-scale mode the kernels apply to an operand of precision prec:
// scale_mode 2 (E4M3 scaled both ways, the other formats only down) is
// resolved here, per launch, into 1 for E4M3 and 0 otherwise, so that the
// device-side block scale keeps its two modes.
inline int operand_scale_mode(int scale_mode, int prec) {
  return scale_mode == 2 ? (prec == MPCHOL_E4M3 ? 1 : 0) : scale_mode;
}
// Tree-TRSM (Algorithm 2) / Tree-SYRK (Algorithm 3) on their own, on blocks of
// one matrix (ld ldl) as Algorithm 1 calls them: TRSM A21 = (k, 0, m x k)
// against L11 = (0, 0, k x k); SYRK A22 = (k, k, n x n) -= A21 A21^T with
// A21 = (k, 0, n x k).  The precision list is read by their own recursion
// depth; FP64 leaf TRSMs go through inverses of L11's leaf blocks formed first.
void build_trsm_plan(Plan& P, int64_t m, int64_t k, int64_t ldl, const mpchol_tree* t);
void build_syrk_plan(Plan& P, int64_t n, int64_t k, int64_t ldl, const mpchol_tree* t);


// Internal Tree-POTRF nodes (order > leaf) of an order-n factorization in
// preorder: {i0, m, m1, depth} each.
struct PolicyNodeRec {
  int64_t i0;
  int64_t m, m1;
  int32_t depth;
};
void tree_nodes(int64_t n, const mpchol_tree* t, std::vector<PolicyNodeRec>& out);

}  // namespace mpc
