// C-ABI of libmpchol: context, plan cache, executor and the refinement loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <sstream>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mpchol.h"
#include "batched.h"
#include "internal.h"
#include "numfmt.h"
#include "plan.h"
#include "policy.h"

using namespace mpc;

#define HIPCHK(x)                          \
  do {                                     \
    hipError_t e_ = (x);                   \
    if (e_ != hipSuccess) return MPCHOL_HIP_ERROR; \
  } while (0)

namespace {
constexpr int kNormParts = 64;
constexpr int kMaxRhs = 16;
}  // namespace

struct mpchol_ctx_s {
  int device = 0;
  DevStatus* dst = nullptr;   // device status words
  DevStatus* hst = nullptr;   // pinned host copy
  void* ws = nullptr;         // quantized operand copies
  size_t ws_bytes = 0;
  double* inv = nullptr;      // FP64 leaf inverses (KL x KL per slot)
  int ninv = 0;
  double* part = nullptr;     // max-abs partials
  int64_t part_count = 0;
  double* rbuf = nullptr;     // refinement residual / correction (n x nrhs)
  int64_t rbuf_count = 0;
  double* rpart = nullptr;    // residual partial sums (residual_part_bytes(n))
  size_t rpart_bytes = 0;
  // block solves: published solution blocks and diagonal-block inverses
  double* tsv_x = nullptr;    // published solution blocks (n x kMaxRhs)
  size_t tsv_x_count = 0;
  double* tsv_yd = nullptr;   // inverses of the 64 x 64 diagonal blocks of L, then
                              // the chain-step matrices of both solve directions
  size_t tsv_yd_count = 0;
  double* npart = nullptr;    // norm partials (device)
  double* hnpart = nullptr;   // norm partials (pinned host)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // copy of A's rows below the top-level A11 into L, overlapped with A11's
  // factorization
  hipStream_t side = nullptr;
  hipEvent_t ev_in = nullptr, ev_copy = nullptr;
  // lookahead: a Tree-SYRK tail on the side stream (ev_la_main: the caller's
  // stream has reached it; ev_la_side: the side stream's work is done)
  hipEvent_t ev_la_main = nullptr, ev_la_side = nullptr;
  std::map<std::string, std::unique_ptr<Plan>> plans;
  // per-launch-class event timing (mpchol_profile)
  uint32_t prof_mask = 0;
  std::vector<hipEvent_t> prof_ev;      // pool, used in pairs
  std::vector<int> prof_kind;           // kind of each recorded pair
  std::vector<double> prof_flops;       // algorithmic flops / bytes of each pair
  size_t prof_used = 0;
  double acc_ms[MPCHOL_PROF_KINDS] = {0};
  double acc_work[MPCHOL_PROF_KINDS] = {0};
  int64_t acc_n[MPCHOL_PROF_KINDS] = {0};
  // leaf choice by size for the batched path (mpchol_set_tune_table)
  std::vector<mpchol_tune_entry> tune;   // per-size plan choices of the batched path
  // batched program cache: device arrays and the captured graph of the last call
  struct Batch {
    std::string key;
    std::vector<void*> bufs;        // device allocations owned by the program
    BatchProgram prog{};
    BatchInfo* hinfo = nullptr;     // pinned
    int64_t batch = 0;
    int nwg = 0;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t cap = nullptr;
  } bt;
  // policy buffers (features, labels, training), grown on demand
  std::vector<std::pair<void*, size_t>> pbuf;
};

static_assert(MPCHOL_PROF_KINDS == 11, "per-class slots of the persistent kernel's timing");

static void free_batch(mpchol_ctx c) {
  auto& B = c->bt;
  if (B.exec) (void)hipGraphExecDestroy(B.exec);
  if (B.graph) (void)hipGraphDestroy(B.graph);
  B.exec = nullptr;
  B.graph = nullptr;
  for (void* p : B.bufs) (void)hipFree(p);
  B.bufs.clear();
  if (B.hinfo) (void)hipHostFree(B.hinfo);
  B.hinfo = nullptr;
  B.key.clear();
}

static int launch_kind(const Launch& L) {
  switch (L.kind) {
    case Launch::GEMM: return MPCHOL_PROF_GEMM_E4M3 + L.prec;
    case Launch::CAST: return MPCHOL_PROF_CAST;
    case Launch::MAXABS: return MPCHOL_PROF_MAXABS;
    case Launch::POTRF: return MPCHOL_PROF_POTRF;
    case Launch::TRINV: return MPCHOL_PROF_TRINV;
    case Launch::INVJOIN: return MPCHOL_PROF_TRINV;
    default: return MPCHOL_PROF_TRSM;
  }
}

// Record a start event for a launch of `kind` when profiling it; returns the
// pair index or -1.
static int prof_begin(mpchol_ctx c, int kind, double work, hipStream_t s) {
  if (!(c->prof_mask & (1u << kind))) return -1;
  size_t i = c->prof_used;
  if (2 * i + 2 > c->prof_ev.size()) {
    for (int k = 0; k < 2; k++) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      c->prof_ev.push_back(e);
    }
    c->prof_kind.push_back(0);
    c->prof_flops.push_back(0);
  }
  c->prof_kind[i] = kind;
  c->prof_flops[i] = work;
  c->prof_used++;
  if (hipEventRecord(c->prof_ev[2 * i], s) != hipSuccess) return -1;
  return (int)i;
}
static void prof_end(mpchol_ctx c, int i, hipStream_t s) {
  if (i >= 0) (void)hipEventRecord(c->prof_ev[2 * i + 1], s);
}
// Fold the recorded pairs into the accumulators (waits for their events).
static int prof_collect(mpchol_ctx c) {
  for (size_t i = 0; i < c->prof_used; i++) {
    HIPCHK(hipEventSynchronize(c->prof_ev[2 * i + 1]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->prof_ev[2 * i], c->prof_ev[2 * i + 1]));
    int k = c->prof_kind[i];
    c->acc_ms[k] += ms;
    c->acc_work[k] += c->prof_flops[i];
    c->acc_n[k] += 1;
  }
  c->prof_used = 0;
  return 0;
}

static double launch_work(const Plan& P, const Launch& L) {
  double w = 0.0;
  if (L.kind == Launch::GEMM) {
    for (int i = 0; i < L.count; i++) {
      const GemmProb& g = P.gemms[L.first + i];
      w += g.lower ? (double)g.m * (g.m + 1) * g.k : 2.0 * g.m * g.n * g.k;
    }
  } else if (L.kind == Launch::CAST) {
    int esz = L.prec == F32 ? 4 : L.prec == F16 ? 2 : 1;
    for (int i = 0; i < L.count; i++) {
      const CastJob& j = P.casts[L.first + i];
      w += (double)j.rows * j.cols * (8.0 + esz);
    }
  } else if (L.kind == Launch::MAXABS) {
    for (int i = 0; i < L.count; i++) {
      const MaxabsJob& j = P.maxabs[L.first + i];
      w += (double)j.rows * j.cols * 8.0;
    }
  } else if (L.kind == Launch::INVJOIN) {
    w = 2.0 * (double)(L.a1 - L.a2) * L.a2 * L.a1;   // the two products
  } else if (L.kind == Launch::POTRF || L.kind == Launch::TRINV) {
    w = (double)L.a1 * L.a1 * L.a1 / 3.0;
    if (L.kind == Launch::POTRF && L.a2 == 1) w *= 2.0;   // with the inverse
  } else {
    w = (double)L.a1 * L.a3 * L.a3;
  }
  return w;
}

static void free_plan(Plan& P) {
  if (P.d_maxabs) (void)hipFree(P.d_maxabs);
  if (P.d_casts) (void)hipFree(P.d_casts);
  if (P.d_gemms) (void)hipFree(P.d_gemms);
  P.d_maxabs = nullptr;
  P.d_casts = nullptr;
  P.d_gemms = nullptr;
}

template <typename T>
static int upload(T** dptr, const std::vector<T>& v) {
  if (v.empty()) return 0;
  HIPCHK(hipMalloc((void**)dptr, sizeof(T) * v.size()));
  HIPCHK(hipMemcpy(*dptr, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return 0;
}

static int ensure_ws(mpchol_ctx c, size_t bytes, int64_t parts) {
  if (bytes > c->ws_bytes) {
    HIPCHK(hipDeviceSynchronize());
    if (c->ws) HIPCHK(hipFree(c->ws));
    c->ws = nullptr;
    HIPCHK(hipMalloc(&c->ws, bytes));
    c->ws_bytes = bytes;
  }
  if (parts > c->part_count) {
    HIPCHK(hipDeviceSynchronize());
    if (c->part) HIPCHK(hipFree(c->part));
    c->part = nullptr;
    HIPCHK(hipMalloc((void**)&c->part, sizeof(double) * parts));
    c->part_count = parts;
  }
  return 0;
}

// Lookahead mode of the single-matrix factorization (build_plan): 2 unless
// MPCHOL_LOOKAHEAD says 0 or 1 (the switch that measures what the overlap
// gains).
static int lookahead_on() {
  static const int mode = [] {
    const char* e = getenv("MPCHOL_LOOKAHEAD");
    return e && (e[0] == '0' || e[0] == '1') ? e[0] - '0' : 2;
  }();
  return mode;
}

// op 0: Tree-POTRF of order n; 1: Tree-TRSM of an n x k block against a k x k
// factor; 2: Tree-SYRK of order n with k columns.
static int get_plan(mpchol_ctx c, int64_t n, int64_t ldl, const mpchol_tree* t, Plan** out,
                    int op = 0, int64_t k = 0) {
  std::string key = plan_key(n, ldl, t);
  if (op) key = (op == 1 ? "trsm:" : "syrk:") + std::to_string(k) + ":" + key;
  auto it = c->plans.find(key);
  if (it != c->plans.end()) {
    *out = it->second.get();
    return 0;
  }
  std::unique_ptr<Plan> P(new Plan());
  if (op == 1) build_trsm_plan(*P, n, k, ldl, t);
  else if (op == 2) build_syrk_plan(*P, n, k, ldl, t);
  else build_plan(*P, n, ldl, t, false, 0, lookahead_on());
  if (upload(&P->d_maxabs, P->maxabs) || upload(&P->d_casts, P->casts) ||
      upload(&P->d_gemms, P->gemms)) {
    free_plan(*P);
    return MPCHOL_HIP_ERROR;
  }
  *out = P.get();
  c->plans[key] = std::move(P);
  return 0;
}

// wait_at >= 0: the stream waits for wait_ev before launch wait_at.
static int run_plan(mpchol_ctx c, const Plan& P, double* L, int64_t ldl, hipStream_t s,
                    int wait_at = -1, hipEvent_t wait_ev = nullptr) {
  for (size_t li = 0; li < P.launches.size(); li++) {
    const Launch& Lc = P.launches[li];
    const int sm = operand_scale_mode(P.tree.scale_mode, Lc.prec);
    if ((int)li == wait_at) HIPCHK(hipStreamWaitEvent(s, wait_ev, 0));
    if (Lc.wait_side) HIPCHK(hipStreamWaitEvent(s, c->ev_la_side, 0));
    hipStream_t ls = s;
    if (Lc.side) {
      // a lookahead tail: starts once the caller's stream has issued
      // everything before it (the casts it reads)
      HIPCHK(hipEventRecord(c->ev_la_main, s));
      HIPCHK(hipStreamWaitEvent(c->side, c->ev_la_main, 0));
      ls = c->side;
    }
    hipError_t e = hipSuccess;
    const int pk = c->prof_mask ? prof_begin(c, launch_kind(Lc), launch_work(P, Lc), ls) : -1;
    switch (Lc.kind) {
      case Launch::POTRF:
        if (Lc.a2 == 1)
          e = launch_potrf_inv(L, ldl, Lc.a0, (int)Lc.a1, c->dst,
                               c->inv + (size_t)Lc.first * kInvLd * kInvLd + Lc.off, kInvLd, ls);
        else
          e = launch_potrf_leaf(Lc.prec, L, ldl, Lc.a0, (int)Lc.a1, c->dst, ls);
        break;
      case Launch::TRSM:
        if (Lc.first >= 0)
          e = launch_trsm_inv(L, ldl, Lc.a0, Lc.a1, Lc.a2, (int)Lc.a3,
                              c->inv + (size_t)Lc.first * kInvLd * kInvLd + Lc.off, kInvLd, ls);
        else
          e = launch_trsm_leaf(Lc.prec, L, ldl, Lc.a0, Lc.a1, Lc.a2, (int)Lc.a3, ls);
        break;
      case Launch::TRINV:
        e = launch_trinv(L, ldl, Lc.a0, (int)Lc.a1,
                         c->inv + (size_t)Lc.first * kInvLd * kInvLd + Lc.off, kInvLd, ls);
        break;
      case Launch::INVJOIN:
        e = launch_inv_join(L, ldl, Lc.a0, (int)Lc.a1, (int)Lc.a2,
                            c->inv + (size_t)Lc.first * kInvLd * kInvLd, kInvLd, ls);
        break;
      case Launch::MAXABS:
        e = launch_maxabs(L, ldl, P.d_maxabs + Lc.first, Lc.count, Lc.total, c->part, ls);
        break;
      case Launch::CAST:
        if (Lc.a0 == 1)
          e = launch_cast_max(L, ldl, P.d_casts + Lc.first, Lc.count, Lc.total, c->part, Lc.prec,
                              c->ws, ls);
        else
          e = launch_cast(L, ldl, P.d_casts + Lc.first, Lc.count, Lc.total, c->part, Lc.prec, sm,
                          c->ws, c->dst, ls);
        break;
      case Launch::GEMM:
        e = launch_gemm(Lc.prec, Lc.tile, L, ldl, c->ws, P.d_gemms + Lc.first, Lc.count,
                        Lc.total, c->part, sm, c->dst, ls);
        break;
    }
    prof_end(c, pk, ls);
    if (e != hipSuccess) return MPCHOL_HIP_ERROR;
    if (Lc.side) HIPCHK(hipEventRecord(c->ev_la_side, c->side));
  }
  // every tail is joined by a later launch; joined again here so that the
  // caller's stream never runs ahead of side-stream work
  if (P.n_side > 0) HIPCHK(hipStreamWaitEvent(s, c->ev_la_side, 0));
  return 0;
}

static int status_from(const DevStatus& h, mpchol_info* info) {
  int st = MPCHOL_OK;
  int64_t fi = 0;
  if (h.failed != ~0ull) {
    st = MPCHOL_NOT_SPD;
    fi = (int64_t)h.failed;
  } else if (h.nonfinite) {
    st = MPCHOL_NONFINITE;
  } else if (h.wait_timeout) {
    st = MPCHOL_HIP_ERROR;
  }
  if (info) {
    info->status = st;
    info->failed_index = fi;
  }
  return st;
}

// Device buffer `slot` of the policy path with at least `bytes` (grown after
// the device has drained, so no queued kernel still uses the old one).
static void* pol_buf(mpchol_ctx c, size_t slot, size_t bytes) {
  if (c->pbuf.size() <= slot) c->pbuf.resize(slot + 1, {nullptr, 0});
  auto& b = c->pbuf[slot];
  if (b.second >= bytes && b.first) return b.first;
  if (hipDeviceSynchronize() != hipSuccess) return nullptr;
  if (b.first) (void)hipFree(b.first);
  b = {nullptr, 0};
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) return nullptr;
  b = {p, std::max<size_t>(bytes, 256)};
  return p;
}

static void add_stat_job(std::vector<StatJob>& jobs, int& parts, int64_t r0, int64_t c0, int64_t rows,
                         int64_t cols, int mode, int node) {
  StatJob j{};
  j.r0 = r0;
  j.c0 = c0;
  j.rows = (int32_t)rows;
  j.cols = (int32_t)cols;
  j.mode = mode;
  j.node = node;
  const int64_t np = std::max<int64_t>(1, std::min<int64_t>(128, cols));
  j.cpw = (int32_t)((cols + np - 1) / np);
  j.nparts = (int32_t)((cols + j.cpw - 1) / j.cpw);
  j.part0 = parts;
  j.wg_start = parts;
  parts += j.nparts;
  jobs.push_back(j);
}

struct PolicyTables {
  std::vector<PolicyNodeRec> rec;
  std::vector<PNode> nodes;
};

static void policy_tables(int64_t n, const mpchol_tree* t, PolicyTables& T) {
  tree_nodes(n, t, T.rec);
  T.nodes.clear();
  for (const PolicyNodeRec& r : T.rec)
    T.nodes.push_back(PNode{r.i0, (int32_t)r.m, (int32_t)r.m1, r.depth, 0});
}

template <typename T>
static int upload_async(mpchol_ctx c, size_t slot, const std::vector<T>& v, T** out, hipStream_t s) {
  *out = (T*)pol_buf(c, slot, sizeof(T) * std::max<size_t>(1, v.size()));
  if (!*out) return MPCHOL_HIP_ERROR;
  if (!v.empty())
    HIPCHK(hipMemcpyAsync(*out, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
  // the host vector must outlive the copy
  HIPCHK(hipStreamSynchronize(s));
  return 0;
}

// Features of every node of A into feat (device).
static int policy_features(mpchol_ctx c, int64_t n, const double* A, int64_t lda,
                           const PolicyTables& T, float* feat, hipStream_t s) {
  const int nn = (int)T.nodes.size();
  if (nn == 0) return 0;
  std::vector<StatJob> jobs;
  int parts = 0;
  for (int k = 0; k < nn; k++) {
    const PNode& N = T.nodes[k];
    add_stat_job(jobs, parts, N.i0 + N.m1, N.i0, N.m - N.m1, N.m1, 0, k);
  }
  const int64_t nstrip = (n + 63) / 64;
  double* rowpart = (double*)pol_buf(c, 0, sizeof(double) * (size_t)(nstrip * n));
  double* colsum = (double*)pol_buf(c, 1, sizeof(double) * (size_t)n);
  double* ratio = (double*)pol_buf(c, 2, sizeof(double) * (size_t)n);
  double* dparts = (double*)pol_buf(c, 3, sizeof(double) * 4 * (size_t)parts);
  double* rowmax = (double*)pol_buf(c, 19, sizeof(double) * (size_t)(nstrip * n));
  double* colmax = (double*)pol_buf(c, 20, sizeof(double) * (size_t)n);
  double* gap = (double*)pol_buf(c, 21, sizeof(double) * (size_t)n);
  if (!rowpart || !colsum || !ratio || !dparts || !rowmax || !colmax || !gap)
    return MPCHOL_HIP_ERROR;
  PNode* dn = nullptr;
  StatJob* dj = nullptr;
  if (upload_async(c, 4, T.nodes, &dn, s) || upload_async(c, 5, jobs, &dj, s)) return MPCHOL_HIP_ERROR;
  HIPCHK(launch_rowabs(A, lda, n, rowpart, colsum, 0, s));
  HIPCHK(launch_rowabs(A, lda, n, rowmax, colmax, 1, s));
  HIPCHK(launch_row_ratio(A, lda, n, rowpart, colsum, rowmax, colmax, ratio, gap, s));
  HIPCHK(launch_stats(A, lda, dj, (int)jobs.size(), parts, nullptr, dparts, s));
  HIPCHK(launch_node_features(dn, nn, A, lda, dj, dparts, ratio, gap, feat, s));
  return 0;
}

static const mpchol_tune_entry* tuned(mpchol_ctx c, int64_t n) {
  for (const mpchol_tune_entry& e : c->tune)
    if (n <= e.nmax) return &e;
  return nullptr;
}

template <typename T>
static int dev_upload(std::vector<void*>& keep, T** dptr, const std::vector<T>& v) {
  *dptr = nullptr;
  size_t bytes = sizeof(T) * std::max<size_t>(v.size(), 1);
  HIPCHK(hipMalloc((void**)dptr, bytes));
  keep.push_back(*dptr);
  if (!v.empty()) HIPCHK(hipMemcpy(*dptr, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return 0;
}

extern "C" {


int mpchol_backward_error(mpchol_ctx c, int64_t n, const double* A, int64_t lda, const double* L,
                          int64_t ldl, double* norms, void* stream) {
  if (!c) return -1;
  if (n < 0 || n > (int64_t)1 << 31) return -2;
  if (n > 0 && !A) return -3;
  if (lda < std::max<int64_t>(1, n)) return -4;
  if (n > 0 && !L) return -5;
  if (ldl < std::max<int64_t>(1, n)) return -6;
  if (!norms) return -7;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->device));
  const int64_t nt = llt_tiles(n);
  double* parts = (double*)pol_buf(c, 16, sizeof(double) * 2 * (size_t)std::max<int64_t>(1, nt));
  double* out = (double*)pol_buf(c, 17, sizeof(double) * 2);
  if (!parts || !out) return MPCHOL_HIP_ERROR;
  HIPCHK(launch_llt_resid(n, A, lda, L, ldl, parts, out, s));
  HIPCHK(hipMemcpyAsync(norms, out, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return 0;
}

int64_t mpchol_policy_nodes(int64_t n, const mpchol_tree* tree, int64_t* table) {
  if (n < 0) return -1;
  if (validate_tree(tree)) return -2;
  std::vector<PolicyNodeRec> rec;
  tree_nodes(n, tree, rec);
  if (table)
    for (size_t k = 0; k < rec.size(); k++) {
      table[4 * k + 0] = rec[k].i0;
      table[4 * k + 1] = rec[k].m;
      table[4 * k + 2] = rec[k].m1;
      table[4 * k + 3] = rec[k].depth;
    }
  return (int64_t)rec.size();
}

static_assert(kMlpParams == MPCHOL_MLP_PARAMS, "perceptron layout of the header");

int mpchol_policy_features(mpchol_ctx c, int64_t n, const double* A, int64_t lda,
                           const mpchol_tree* tree, float* feat, void* stream) {
  if (!c) return -1;
  if (n < 0 || n > (int64_t)1 << 31) return -2;
  if (n > 0 && !A) return -3;
  if (lda < std::max<int64_t>(1, n)) return -4;
  if (validate_tree(tree)) return -5;
  PolicyTables T;
  policy_tables(n, tree, T);
  if (!T.nodes.empty() && !feat) return -6;
  HIPCHK(hipSetDevice(c->device));
  return policy_features(c, n, A, lda, T, feat, (hipStream_t)stream);
}

int mpchol_policy_labels(mpchol_ctx c, int64_t n, const double* A, int64_t lda, const double* L,
                         int64_t ldl, const mpchol_tree* tree, double tau, int32_t scale_mode,
                         int32_t min_prec, double* err, int32_t* labels, void* stream) {
  if (!c) return -1;
  if (n < 0 || n > (int64_t)1 << 31) return -2;
  if (n > 0 && !A) return -3;
  if (lda < std::max<int64_t>(1, n)) return -4;
  if (n > 0 && !L) return -5;
  if (ldl < std::max<int64_t>(1, n)) return -6;
  if (validate_tree(tree)) return -7;
  if (!(tau > 0.0)) return -8;
  if (scale_mode < 0 || scale_mode > 2) return -9;
  PolicyTables T;
  policy_tables(n, tree, T);
  const int nn = (int)T.nodes.size();
  if (nn > 0 && !labels) return -10;
  if (min_prec < MPCHOL_E4M3 || min_prec > MPCHOL_F64) return -11;
  if (nn == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->device));
  std::vector<StatJob> xj, xj2, aj;
  int xparts = 0, xparts2 = 0, aparts = 0;
  double sum_s2 = 0.0;
  for (int k = 0; k < nn; k++) {
    const PNode& N = T.nodes[k];
    add_stat_job(xj, xparts, N.i0 + N.m1, N.i0, N.m - N.m1, N.m1, 0, k);
    add_stat_job(xj2, xparts2, N.i0 + N.m1, N.i0, N.m - N.m1, N.m1, 2, k);
    add_stat_job(aj, aparts, N.i0, N.i0, N.m, N.m, 1, k);
    sum_s2 += (double)N.m1 * (double)N.m1;
  }
  double* dx = (double*)pol_buf(c, 6, sizeof(double) * 4 * (size_t)xparts);
  double* da = (double*)pol_buf(c, 7, sizeof(double) * 4 * (size_t)aparts);
  double* sc = (double*)pol_buf(c, 8, sizeof(double) * 3 * (size_t)nn);
  double* gd = (double*)pol_buf(c, 18, sizeof(double));
  if (!dx || !da || !sc || !gd) return MPCHOL_HIP_ERROR;
  PNode* dn = nullptr;
  StatJob *dxj = nullptr, *dxj2 = nullptr, *daj = nullptr;
  if (upload_async(c, 4, T.nodes, &dn, s) || upload_async(c, 9, xj, &dxj, s) ||
      upload_async(c, 10, xj2, &dxj2, s) || upload_async(c, 11, aj, &daj, s))
    return MPCHOL_HIP_ERROR;
  HIPCHK(launch_stats(L, ldl, dxj, nn, xparts, nullptr, dx, s));
  HIPCHK(launch_node_scales(nn, dxj, dx, scale_mode, sc, s));   // mode 2 resolved per format
  HIPCHK(launch_stats(L, ldl, dxj2, nn, xparts2, sc, dx, s));
  HIPCHK(launch_stats(A, lda, daj, nn, aparts, nullptr, da, s));
  HIPCHK(launch_pivot_ratio(L, ldl, n, gd, s));
  HIPCHK(launch_node_labels(dn, nn, dxj2, dx, daj, da, tau, gd, sum_s2, min_prec, err, labels,
                            s));
  return 0;
}

int mpchol_mlp_forward(mpchol_ctx c, int64_t rows, const float* X, const float* params,
                       float* probs, int32_t* cls, void* stream) {
  if (!c) return -1;
  if (rows < 0) return -2;
  if (rows > 0 && !X) return -3;
  if (!params) return -4;
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_mlp_forward(rows, X, params, probs, cls, (hipStream_t)stream));
  return 0;
}

int mpchol_mlp_train_step(mpchol_ctx c, int64_t rows, const float* X, const int32_t* y,
                          float* params, float* m, float* v, int32_t step, float lr, float* loss,
                          float* grad, void* stream) {
  if (!c) return -1;
  if (rows < 1 || rows > ((int64_t)1 << 31)) return -2;
  if (!X) return -3;
  if (!y) return -4;
  if (!params) return -5;
  if (lr > 0.f && (!m || !v)) return -6;
  if (step < 1) return -7;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->device));
  const int nwg = (int)((rows + kMlpRows - 1) / kMlpRows);
  float* gpart = (float*)pol_buf(c, 12, sizeof(float) * (size_t)kMlpTrained * (size_t)nwg);
  float* lpart = (float*)pol_buf(c, 13, sizeof(float) * (size_t)nwg);
  if (!gpart || !lpart) return MPCHOL_HIP_ERROR;
  HIPCHK(launch_mlp_grad(rows, X, y, params, gpart, lpart, s));
  HIPCHK(launch_mlp_adam(nwg, rows, gpart, lpart, params, m, v, step, lr, loss, grad, s));
  return 0;
}

int mpchol_policy_choose(mpchol_ctx c, int64_t n, const double* A, int64_t lda,
                         const mpchol_tree* tree, const float* params, int8_t* node_prec,
                         void* stream) {
  if (!c) return -1;
  if (n < 0 || n > (int64_t)1 << 31) return -2;
  if (n > 0 && !A) return -3;
  if (lda < std::max<int64_t>(1, n)) return -4;
  if (validate_tree(tree)) return -5;
  if (!params) return -6;
  PolicyTables T;
  policy_tables(n, tree, T);
  const int nn = (int)T.nodes.size();
  if (nn == 0) return 0;
  if (!node_prec) return -7;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->device));
  float* feat = (float*)pol_buf(c, 14, sizeof(float) * kMlpIn * (size_t)nn);
  int32_t* cls = (int32_t*)pol_buf(c, 15, sizeof(int32_t) * (size_t)nn);
  if (!feat || !cls) return MPCHOL_HIP_ERROR;
  int r = policy_features(c, n, A, lda, T, feat, s);
  if (r) return r;
  HIPCHK(launch_mlp_forward(nn, feat, params, nullptr, cls, s));
  std::vector<int32_t> h((size_t)nn);
  HIPCHK(hipMemcpyAsync(h.data(), cls, sizeof(int32_t) * (size_t)nn, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int k = 0; k < nn; k++) node_prec[k] = (int8_t)h[(size_t)k];
  return 0;
}

const char* mpchol_version(void) { return "mpchol 0.1 (gfx950, HIP)"; }

int mpchol_create(mpchol_ctx* ctx, int device) {
  if (!ctx) return -1;
  *ctx = nullptr;
  std::unique_ptr<mpchol_ctx_s> c(new mpchol_ctx_s());
  c->device = device;
  HIPCHK(hipSetDevice(device));
  HIPCHK(hipMalloc((void**)&c->dst, sizeof(DevStatus)));
  HIPCHK(hipHostMalloc((void**)&c->hst, sizeof(DevStatus), hipHostMallocDefault));
  HIPCHK(hipMalloc((void**)&c->npart, sizeof(double) * kNormParts * kMaxRhs * 2));
  HIPCHK(hipHostMalloc((void**)&c->hnpart, sizeof(double) * kNormParts * kMaxRhs * 2,
                       hipHostMallocDefault));
  HIPCHK(hipEventCreate(&c->ev0));
  HIPCHK(hipEventCreate(&c->ev1));
  HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&c->ev_copy, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&c->ev_la_main, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&c->ev_la_side, hipEventDisableTiming));
  *ctx = c.release();
  return 0;
}

int mpchol_destroy(mpchol_ctx c) {
  if (!c) return 0;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : c->plans) free_plan(*kv.second);
  if (c->ws) (void)hipFree(c->ws);
  if (c->inv) (void)hipFree(c->inv);
  if (c->part) (void)hipFree(c->part);
  if (c->rbuf) (void)hipFree(c->rbuf);
  if (c->rpart) (void)hipFree(c->rpart);
  if (c->tsv_x) (void)hipFree(c->tsv_x);
  if (c->tsv_yd) (void)hipFree(c->tsv_yd);
  if (c->npart) (void)hipFree(c->npart);
  if (c->hnpart) (void)hipHostFree(c->hnpart);
  if (c->dst) (void)hipFree(c->dst);
  if (c->hst) (void)hipHostFree(c->hst);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_copy) (void)hipEventDestroy(c->ev_copy);
  if (c->ev_la_main) (void)hipEventDestroy(c->ev_la_main);
  if (c->ev_la_side) (void)hipEventDestroy(c->ev_la_side);
  if (c->side) (void)hipStreamDestroy(c->side);
  for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
  free_batch(c);
  if (c->bt.cap) (void)hipStreamDestroy(c->bt.cap);
  for (auto& b : c->pbuf) (void)hipFree(b.first);
  delete c;
  return 0;
}

int mpchol_factor(mpchol_ctx c, int64_t n, const double* A, int64_t lda, double* L, int64_t ldl,
                  const mpchol_tree* tree, void* stream, mpchol_info* info) {
  if (!c) return -1;
  if (n < 0) return -2;
  if (!A && n > 0) return -3;
  if (lda < std::max<int64_t>(1, n)) return -4;
  if (!L && n > 0) return -5;
  if (ldl < std::max<int64_t>(1, n)) return -6;
  int v = validate_tree(tree);
  if (v) return v;
  if (L == A && ldl != lda) return -6;
  if (info) std::memset(info, 0, sizeof(*info));
  if (n == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->device));
  Plan* P = nullptr;
  int r = get_plan(c, n, ldl, tree, &P);
  if (r) return r;
  r = ensure_ws(c, std::max<size_t>(P->ws_bytes, 256), std::max<int64_t>(P->parts, 1));
  if (r) return r;
  if (P->ninv > c->ninv) {
    HIPCHK(hipDeviceSynchronize());
    if (c->inv) HIPCHK(hipFree(c->inv));
    c->inv = nullptr;
    c->ninv = 0;
    HIPCHK(hipMalloc((void**)&c->inv, sizeof(double) * kInvLd * kInvLd * (size_t)P->ninv));
    c->ninv = P->ninv;
  }
  if (info) HIPCHK(hipEventRecord(c->ev0, s));
  HIPCHK(launch_status_init(c->dst, s));
  if (L != A && P->first_outer > 0) {
    // A11 on the caller's stream; the rows below it on the side stream, which
    // the caller's stream joins before the first launch that reads them
    const int64_t n1 = P->split1;
    HIPCHK(launch_copy_lower_rows(A, lda, L, ldl, 0, n1, 0, n1, s));
    HIPCHK(hipEventRecord(c->ev_in, s));
    HIPCHK(hipStreamWaitEvent(c->side, c->ev_in, 0));
    HIPCHK(launch_copy_lower_rows(A, lda, L, ldl, 0, n, n1, n, c->side));
    HIPCHK(hipEventRecord(c->ev_copy, c->side));
    r = run_plan(c, *P, L, ldl, s, P->first_outer, c->ev_copy);
  } else {
    if (L != A) HIPCHK(launch_copy_lower(A, lda, L, ldl, n, s));
    r = run_plan(c, *P, L, ldl, s);
  }
  if (r) return r;
  HIPCHK(hipMemcpyAsync(c->hst, c->dst, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  if (!info) return 0;
  HIPCHK(hipEventRecord(c->ev1, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  info->ms_factor = ms;
  return status_from(*c->hst, info);
}

// Tree-TRSM / Tree-SYRK on their own (op 1 / 2, see get_plan) on blocks of A.
static int run_subkernel(mpchol_ctx c, int op, int64_t a, int64_t k, double* A, int64_t lda,
                         const mpchol_tree* tree, void* stream, mpchol_info* info) {
  if (!c) return -1;
  if (a < 0) return -2;
  if (k < 0) return -3;
  if (!A && a > 0 && k > 0) return -4;
  if (lda < std::max<int64_t>(1, a + k)) return -5;
  int v = validate_tree(tree);
  if (v) return v == -7 ? -6 : v;
  if (tree->n_nodes != 0) return -6;
  if (info) std::memset(info, 0, sizeof(*info));
  if (a == 0 || k == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->device));
  Plan* P = nullptr;
  int r = get_plan(c, a, lda, tree, &P, op, k);
  if (r) return r;
  r = ensure_ws(c, std::max<size_t>(P->ws_bytes, 256), std::max<int64_t>(P->parts, 1));
  if (r) return r;
  if (P->ninv > c->ninv) {
    HIPCHK(hipDeviceSynchronize());
    if (c->inv) HIPCHK(hipFree(c->inv));
    c->inv = nullptr;
    c->ninv = 0;
    HIPCHK(hipMalloc((void**)&c->inv, sizeof(double) * kInvLd * kInvLd * (size_t)P->ninv));
    c->ninv = P->ninv;
  }
  if (info) HIPCHK(hipEventRecord(c->ev0, s));
  HIPCHK(launch_status_init(c->dst, s));
  r = run_plan(c, *P, A, lda, s);
  if (r) return r;
  HIPCHK(hipMemcpyAsync(c->hst, c->dst, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  if (!info) return 0;
  HIPCHK(hipEventRecord(c->ev1, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  info->ms_factor = ms;
  return status_from(*c->hst, info);
}

int mpchol_trsm(mpchol_ctx c, int64_t m, int64_t k, double* A, int64_t lda,
                const mpchol_tree* tree, void* stream, mpchol_info* info) {
  return run_subkernel(c, 1, m, k, A, lda, tree, stream, info);
}

int mpchol_syrk(mpchol_ctx c, int64_t n, int64_t k, double* A, int64_t lda,
                const mpchol_tree* tree, void* stream, mpchol_info* info) {
  return run_subkernel(c, 2, n, k, A, lda, tree, stream, info);
}

// Published-block copy and diagonal-block inverses of the block solves of order n.
static int ensure_trsv(mpchol_ctx c, int64_t n) {
  const size_t yc = (size_t)((n + 63) / 64) * 4096 * 3;
  if (yc > c->tsv_yd_count) {
    HIPCHK(hipDeviceSynchronize());
    if (c->tsv_yd) HIPCHK(hipFree(c->tsv_yd));
    c->tsv_yd = nullptr;
    c->tsv_yd_count = 0;
    HIPCHK(hipMalloc((void**)&c->tsv_yd, sizeof(double) * yc));
    c->tsv_yd_count = yc;
  }
  const size_t xc = (size_t)n * kMaxRhs;
  if (xc > c->tsv_x_count) {
    HIPCHK(hipDeviceSynchronize());
    if (c->tsv_x) HIPCHK(hipFree(c->tsv_x));
    c->tsv_x = nullptr;
    c->tsv_x_count = 0;
    HIPCHK(hipMalloc((void**)&c->tsv_x, sizeof(double) * xc));
    c->tsv_x_count = xc;
  }
  return 0;
}

// Device and host buffers of one solve call: the context's (grown on demand)
// or the allocation-free entry point's fixed scratch.
struct SolveBufs {
  int device;
  DevStatus* dst;      // device status words
  DevStatus* hst;      // host copy
  double* yd;          // diagonal-block inverses (nblk 4096), then the chain-step
  double* md;          //   matrices (2 nblk 4096)
  double* xp;          // published solution blocks (n kMaxRhs)
  double* rbuf;        // residual / correction (n nrhs)
  double* rpart;       // residual partial sums (NULL: the two-read residual)
  size_t rpart_bytes;
  double* npart;       // norm partials (kNormParts kMaxRhs 2), device
  double* hnpart;      //   and host
  mpchol_ctx prof;     // launch timing (NULL: none)
};

static int sb_prof_begin(const SolveBufs& B, int kind, double work, hipStream_t s) {
  return B.prof && B.prof->prof_mask ? prof_begin(B.prof, kind, work, s) : -1;
}
static void sb_prof_end(const SolveBufs& B, int i, hipStream_t s) {
  if (B.prof) prof_end(B.prof, i, s);
}

// X <- L^-T L^-1 X for up to kMaxRhs columns at a time (B.yd / B.md hold the
// diagonal-block inverses and chain-step matrices of L).
static int chol_solve_inplace(const SolveBufs& B, int64_t n, int64_t nrhs, const double* L,
                              int64_t ldl, double* X, int64_t ldx, hipStream_t s) {
  const double lbytes = (double)n * (n + 1) / 2 * 8.0;
  int rows = 0;
  const int P = trsv_grid(n, B.device, &rows);
  if (P <= 0) return MPCHOL_HIP_ERROR;
  for (int64_t c0 = 0; c0 < nrhs; c0 += kMaxRhs) {
    int nc = (int)std::min<int64_t>(kMaxRhs, nrhs - c0);
    for (int trans = 0; trans < 2; trans++) {
      const int pk = sb_prof_begin(B, MPCHOL_PROF_TRSV, lbytes, s);
      HIPCHK(launch_trsv(trans, L, ldl, n, nc, X + c0 * ldx, ldx, B.xp, B.yd, B.md, P, rows, B.dst,
                         s));
      sb_prof_end(B, pk, s);
    }
  }
  return 0;
}

static int solve_args(int64_t n, int64_t nrhs, const double* A, int64_t lda, const double* L,
                      int64_t ldl, const double* B, int64_t ldb, const double* X, int64_t ldx,
                      int32_t max_iter) {
  if (n < 0) return -2;
  if (nrhs < 0) return -3;
  if (A && lda < std::max<int64_t>(1, n)) return -5;
  if (!L && n > 0) return -6;
  if (ldl < std::max<int64_t>(1, n)) return -7;
  if (!B && n > 0 && nrhs > 0) return -8;
  if (ldb < std::max<int64_t>(1, n)) return -9;
  if (!X && n > 0 && nrhs > 0) return -10;
  if (ldx < std::max<int64_t>(1, n)) return -11;
  if (max_iter < 0) return -13;
  return 0;
}

// The solve and its refinement on the stream, with the buffers in Bf; returns
// the status (info filled except ms_solve).
static int solve_run(const SolveBufs& Bf, int64_t n, int64_t nrhs, const double* A, int64_t lda,
                     const double* L, int64_t ldl, const double* B, int64_t ldb, double* X,
                     int64_t ldx, double tol, int32_t max_iter, hipStream_t s, mpchol_info* info) {
  HIPCHK(launch_status_init(Bf.dst, s));
  HIPCHK(launch_copy_cols(n, (int)nrhs, B, ldb, X, ldx, s));
  {
    // used by every triangular solve of this call
    const int pk = sb_prof_begin(Bf, MPCHOL_PROF_TRINV,
                                 (double)((n + 63) / 64) * 64.0 * 64.0 * 64.0 / 3.0, s);
    HIPCHK(launch_diag_inv(L, ldl, n, Bf.yd, s));
    HIPCHK(launch_chain_mats(L, ldl, n, Bf.yd, Bf.md, s));
    sb_prof_end(Bf, pk, s);
  }
  int r = chol_solve_inplace(Bf, n, nrhs, L, ldl, X, ldx, s);
  if (r) return r;
  int status = MPCHOL_OK;
  int iters = 0;
  double corr = 0.0;
  if (A && max_iter > 0) {
    double* R = Bf.rbuf;
    double prev = INFINITY;
    int grew = 0;
    status = MPCHOL_NOT_CONVERGED;
    for (int it = 1; it <= max_iter; it++) {
      for (int64_t c0 = 0; c0 < nrhs; c0 += kMaxRhs) {
        int nc = (int)std::min<int64_t>(kMaxRhs, nrhs - c0);
        int pk = sb_prof_begin(Bf, MPCHOL_PROF_RESIDUAL, (double)n * (n + 1) / 2 * 8.0, s);
        HIPCHK(launch_residual(A, lda, n, nc, X + c0 * ldx, ldx, B + c0 * ldb, ldb, R + c0 * n, n,
                               Bf.rpart, Bf.rpart_bytes, s));
        sb_prof_end(Bf, pk, s);
      }
      r = chol_solve_inplace(Bf, n, nrhs, L, ldl, R, n, s);
      if (r) return r;
      double worst = 0.0;
      bool bad = false;
      for (int64_t c0 = 0; c0 < nrhs; c0 += kMaxRhs) {
        int nc = (int)std::min<int64_t>(kMaxRhs, nrhs - c0);
        HIPCHK(launch_update_norms(n, nc, X + c0 * ldx, ldx, R + c0 * n, n, Bf.npart, kNormParts,
                                   nullptr, s));
        HIPCHK(hipMemcpyAsync(Bf.hnpart, Bf.npart, sizeof(double) * kNormParts * nc * 2,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int cc = 0; cc < nc; cc++) {
          double dm = 0.0, xm = 0.0;
          for (int w = 0; w < kNormParts; w++) {
            dm = std::max(dm, Bf.hnpart[(w * nc + cc) * 2 + 0]);
            xm = std::max(xm, Bf.hnpart[(w * nc + cc) * 2 + 1]);
          }
          if (!std::isfinite(dm) || !std::isfinite(xm)) bad = true;
          double rr = xm > 0.0 ? dm / xm : dm;
          worst = std::max(worst, rr);
        }
      }
      iters = it;
      corr = worst;
      if (bad) {
        status = MPCHOL_NONFINITE;
        break;
      }
      if (worst <= tol) {
        status = MPCHOL_OK;
        break;
      }
      if (worst > prev) {
        if (++grew >= 2) break;
      } else {
        grew = 0;
      }
      prev = worst;
    }
  }
  HIPCHK(hipMemcpyAsync(Bf.hst, Bf.dst, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (Bf.hst->wait_timeout) status = MPCHOL_HIP_ERROR;
  if (info) {
    info->status = status;
    info->ir_iters = iters;
    info->final_rel_corr = corr;
  }
  return status;
}

int mpchol_solve(mpchol_ctx c, int64_t n, int64_t nrhs, const double* A, int64_t lda,
                 const double* L, int64_t ldl, const double* B, int64_t ldb, double* X,
                 int64_t ldx, double tol, int32_t max_iter, void* stream, mpchol_info* info) {
  if (!c) return -1;
  const int bad = solve_args(n, nrhs, A, lda, L, ldl, B, ldb, X, ldx, max_iter);
  if (bad) return bad;
  if (info) std::memset(info, 0, sizeof(*info));
  if (n == 0 || nrhs == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipEventRecord(c->ev0, s));
  int r = ensure_trsv(c, n);
  if (r) return r;
  if (A && max_iter > 0 && c->rbuf_count < n * nrhs) {
    HIPCHK(hipStreamSynchronize(s));
    if (c->rbuf) HIPCHK(hipFree(c->rbuf));
    c->rbuf = nullptr;
    HIPCHK(hipMalloc((void**)&c->rbuf, sizeof(double) * n * nrhs));
    c->rbuf_count = n * nrhs;
  }
  if (A && max_iter > 0 && c->rpart_bytes < residual_part_bytes(n)) {
    HIPCHK(hipStreamSynchronize(s));
    if (c->rpart) HIPCHK(hipFree(c->rpart));
    c->rpart = nullptr;
    c->rpart_bytes = 0;
    HIPCHK(hipMalloc((void**)&c->rpart, residual_part_bytes(n)));
    c->rpart_bytes = residual_part_bytes(n);
  }
  const SolveBufs Bf{c->device, c->dst, c->hst, c->tsv_yd,
                     c->tsv_yd + (size_t)((n + 63) / 64) * 4096, c->tsv_x, c->rbuf, c->rpart,
                     c->rpart_bytes, c->npart, c->hnpart, c};
  const int status = solve_run(Bf, n, nrhs, A, lda, L, ldl, B, ldb, X, ldx, tol, max_iter, s, info);
  if (status == MPCHOL_HIP_ERROR || status < 0) return status;
  HIPCHK(hipEventRecord(c->ev1, s));
  HIPCHK(hipStreamSynchronize(s));
  if (info) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    info->ms_solve = ms;
  }
  return status;
}

int mpchol_solve_noalloc(int device, int64_t n, int64_t nrhs, const double* A, int64_t lda,
                         const double* L, int64_t ldl, const double* B, int64_t ldb, double* X,
                         int64_t ldx, double tol, int32_t max_iter, void* stream,
                         mpchol_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  if (device < 0) return -1;
  const int bad = solve_args(n, nrhs, A, lda, L, ldl, B, ldb, X, ldx, max_iter);
  if (bad) return bad;
  if (n > MPCHOL_NOALLOC_MAX_N) return -2;
  if (nrhs > MPCHOL_NOALLOC_MAX_RHS) return -3;
  if (info) std::memset(info, 0, sizeof(*info));
  if (n == 0 || nrhs == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipSetDevice(device));
  NoAllocScratch sc;
  if (noalloc_scratch(device, &sc) != hipSuccess) return MPCHOL_HIP_ERROR;
  DevStatus hst;
  double hnpart[kNormParts * kMaxRhs * 2];
  const SolveBufs Bf{device, sc.status, &hst, sc.yd, sc.yd + (size_t)((n + 63) / 64) * 4096, sc.xp,
                     sc.rbuf, nullptr, 0, sc.npart, hnpart, nullptr};
  const int status = solve_run(Bf, n, nrhs, A, lda, L, ldl, B, ldb, X, ldx, tol, max_iter, s, info);
  if (info)
    info->ms_solve = (float)std::chrono::duration<double, std::milli>(
                         std::chrono::steady_clock::now() - t0).count();
  return status;
}

int mpchol_set_tune_table(mpchol_ctx c, int32_t count, const mpchol_tune_entry* table) {
  if (!c) return -1;
  if (count < 0) return -2;
  if (count > 0 && !table) return -3;
  for (int32_t i = 0; i < count; i++) {
    if (i > 0 && table[i].nmax <= table[i - 1].nmax) return -3;
    if (table[i].leaf < 1) return -4;
    if (table[i].split_align < 0) return -5;
    if (table[i].tile != 0 && table[i].tile != 64 && table[i].tile != 128) return -6;
  }
  c->tune.assign(table, table + count);
  return 0;
}

int mpchol_factor_batched(mpchol_ctx c, int64_t batch, const int64_t* n_host,
                          const double* const* A_dev, const int64_t* lda_host,
                          double* const* L_dev, const int64_t* ldl_host, int64_t nrhs,
                          const double* const* B_dev, double* const* X_dev, double tol,
                          int32_t max_iter, const mpchol_tree* tree, void* stream,
                          mpchol_info* info_host) {
  if (!c) return -1;
  if (batch < 0) return -2;
  if (batch > 0 && !n_host) return -3;
  if (batch > 0 && !A_dev) return -4;
  if (batch > 0 && !lda_host) return -5;
  if (batch > 0 && !L_dev) return -6;
  if (batch > 0 && !ldl_host) return -7;
  if (nrhs < 0 || nrhs > kMaxRhs) return -8;
  if (nrhs > 0 && (!B_dev || !X_dev)) return -9;
  if (max_iter < 0) return -12;
  int v = validate_tree(tree);
  if (v) return v == -7 ? -13 : v;
  if (tree->scale_mode == 2) return MPCHOL_NOT_SUPPORTED;   // one block-scale mode per batch
  for (int64_t i = 0; i < batch; i++) {
    if (n_host[i] < 1 || n_host[i] > (1 << 20)) return -3;
    if (!A_dev[i] || !L_dev[i]) return -4;
    if (lda_host[i] < n_host[i]) return -5;
    if (ldl_host[i] < n_host[i]) return -7;
    if (L_dev[i] == A_dev[i] && ldl_host[i] != lda_host[i]) return -7;
    if (nrhs > 0 && L_dev[i] == A_dev[i]) return -6;   // refinement needs A in FP64
    if (nrhs > 0 && (!B_dev[i] || !X_dev[i])) return -9;
  }
  if (info_host) std::memset(info_host, 0, sizeof(mpchol_info) * (size_t)batch);
  if (batch == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->device));
  auto& BT = c->bt;

  // cache key: everything the device program depends on
  std::ostringstream key;
  const bool bprof = c->prof_mask != 0;
  key << batch << '|' << nrhs << '|' << tol << '|' << max_iter << '|' << bprof << '|'
      << plan_key(0, 1, tree);
  for (const mpchol_tune_entry& e : c->tune)
    key << e.nmax << ':' << e.leaf << ':' << e.split_align << ':' << e.tile << ',';
  for (int64_t i = 0; i < batch; i++) {
    key << '|' << n_host[i] << ',' << lda_host[i] << ',' << ldl_host[i] << ',' << (const void*)A_dev[i]
        << ',' << (const void*)L_dev[i];
    if (nrhs > 0) key << ',' << (const void*)B_dev[i] << ',' << (const void*)X_dev[i];
  }
  if (BT.key != key.str()) {
    HIPCHK(hipDeviceSynchronize());
    free_batch(c);
    std::vector<BatchTask> tasks;
    std::vector<MaxabsJob> mj;
    std::vector<CastJob> cj;
    std::vector<GemmProb> gp;
    std::vector<BatchMat> mats((size_t)batch);
    std::map<std::string, std::pair<int32_t, int32_t>> seen;  // plan -> task range
    size_t ws_max = 256;
    int64_t parts_max = 1;
    for (int64_t i = 0; i < batch; i++) {
      mpchol_tree t = *tree;
      int tile = 0;
      if (const mpchol_tune_entry* e = tuned(c, n_host[i])) {
        t.leaf = e->leaf;
        if (e->split_align > 0) t.split_align = e->split_align;
        tile = e->tile;
      }
      std::string pk = plan_key(n_host[i], ldl_host[i], &t) + "/t" + std::to_string(tile);
      auto it = seen.find(pk);
      if (it == seen.end()) {
        Plan P;
        build_plan(P, n_host[i], ldl_host[i], &t, true, tile);
        int32_t t0 = (int32_t)tasks.size();
        for (const Launch& L : P.launches) {
          if (L.kind == Launch::TRINV || L.kind == Launch::INVJOIN ||
              (L.kind == Launch::TRSM && L.first >= 0) || (L.kind == Launch::POTRF && L.a2 == 1)) {
            free_batch(c);
            return MPCHOL_HIP_ERROR;   // workgroup-level plans never use leaf inverses
          }
          BatchTask T{};
          T.kind = (int32_t)L.kind;
          T.prec = L.prec;
          T.tile = L.tile;
          T.count = L.count;
          T.total = L.total;
          T.a0 = L.a0;
          T.a1 = L.a1;
          T.a2 = L.a2;
          T.a3 = L.a3;
          if (L.kind == Launch::MAXABS) {
            T.first = (int32_t)mj.size();
            mj.insert(mj.end(), P.maxabs.begin() + L.first, P.maxabs.begin() + L.first + L.count);
          } else if (L.kind == Launch::CAST) {
            T.first = (int32_t)cj.size();
            cj.insert(cj.end(), P.casts.begin() + L.first, P.casts.begin() + L.first + L.count);
          } else if (L.kind == Launch::GEMM) {
            T.first = (int32_t)gp.size();
            gp.insert(gp.end(), P.gemms.begin() + L.first, P.gemms.begin() + L.first + L.count);
          }
          tasks.push_back(T);
        }
        ws_max = std::max(ws_max, P.ws_bytes);
        parts_max = std::max(parts_max, P.parts);
        it = seen.emplace(pk, std::make_pair(t0, (int32_t)tasks.size())).first;
      }
      BatchMat& M = mats[(size_t)i];
      M.A = A_dev[i];
      M.L = L_dev[i];
      M.B = nrhs > 0 ? B_dev[i] : nullptr;
      M.X = nrhs > 0 ? X_dev[i] : nullptr;
      M.lda = lda_host[i];
      M.ldl = ldl_host[i];
      M.n = (int32_t)n_host[i];
      M.t0 = it->second.first;
      M.t1 = it->second.second;
    }
    std::vector<int32_t> order((size_t)batch);
    for (int64_t i = 0; i < batch; i++) order[(size_t)i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return n_host[a] > n_host[b]; });
    int64_t nmax = 0;
    for (int64_t i = 0; i < batch; i++) nmax = std::max(nmax, n_host[i]);
    int ncu = 0;
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
    const int nwg = (int)std::max<int64_t>(1, std::min<int64_t>(ncu, batch));
    BatchProgram& G = BT.prog;
    G = BatchProgram{};
    if (dev_upload(BT.bufs, (BatchTask**)&G.tasks, tasks) ||
        dev_upload(BT.bufs, (MaxabsJob**)&G.maxabs, mj) ||
        dev_upload(BT.bufs, (CastJob**)&G.casts, cj) ||
        dev_upload(BT.bufs, (GemmProb**)&G.gemms, gp) ||
        dev_upload(BT.bufs, (BatchMat**)&G.mats, mats) ||
        dev_upload(BT.bufs, (int32_t**)&G.order, order)) {
      free_batch(c);
      return MPCHOL_HIP_ERROR;
    }
    G.ws_stride = (ws_max + 255) / 256 * 256;
    G.part_stride = (size_t)parts_max;
    G.scratch_stride = (size_t)(nmax * std::max<int64_t>(nrhs, 1));
    void* p = nullptr;
    HIPCHK(hipMalloc(&p, sizeof(BatchInfo) * (size_t)batch));
    BT.bufs.push_back(p);
    G.info = (BatchInfo*)p;
    HIPCHK(hipMalloc(&p, 256));
    BT.bufs.push_back(p);
    G.queue = (unsigned int*)p;
    HIPCHK(hipMalloc(&p, G.ws_stride * (size_t)nwg));
    BT.bufs.push_back(p);
    G.ws = (char*)p;
    HIPCHK(hipMalloc(&p, sizeof(double) * G.part_stride * (size_t)nwg));
    BT.bufs.push_back(p);
    G.part = (double*)p;
    HIPCHK(hipMalloc(&p, sizeof(double) * G.scratch_stride * (size_t)nwg));
    BT.bufs.push_back(p);
    G.scratch = (double*)p;
    HIPCHK(hipMalloc(&p, sizeof(DevStatus) * (size_t)nwg));
    BT.bufs.push_back(p);
    G.status = (DevStatus*)p;
    if (bprof) {
      HIPCHK(hipMalloc(&p, sizeof(unsigned long long) * 2 * MPCHOL_PROF_KINDS));
      BT.bufs.push_back(p);
      G.prof = (unsigned long long*)p;
    }
    G.batch = (int32_t)batch;
    G.nrhs = (int32_t)nrhs;
    G.max_iter = max_iter;
    G.scale_mode = tree->scale_mode;   // 0 or 1 (2 is rejected above)
    G.tol = tol;
    HIPCHK(hipHostMalloc((void**)&BT.hinfo, sizeof(BatchInfo) * (size_t)batch,
                         hipHostMallocDefault));
    BT.batch = batch;
    BT.nwg = nwg;
    // one graph: queue reset + persistent kernel + status copy-back
    if (!BT.cap) HIPCHK(hipStreamCreateWithFlags(&BT.cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(BT.cap, hipStreamCaptureModeThreadLocal));
    hipError_t le = launch_batched(G, nwg, BT.cap);
    hipError_t me = hipMemcpyAsync(BT.hinfo, G.info, sizeof(BatchInfo) * (size_t)batch,
                                   hipMemcpyDeviceToHost, BT.cap);
    hipError_t ee = hipStreamEndCapture(BT.cap, &BT.graph);
    if (le != hipSuccess || me != hipSuccess || ee != hipSuccess) {
      free_batch(c);
      return MPCHOL_HIP_ERROR;
    }
    HIPCHK(hipGraphInstantiate(&BT.exec, BT.graph, nullptr, nullptr, 0));
    BT.key = key.str();
  }
  HIPCHK(hipEventRecord(c->ev0, s));
  HIPCHK(hipGraphLaunch(BT.exec, s));
  HIPCHK(hipEventRecord(c->ev1, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  if (BT.prog.prof) {
    // per task class: workgroup-milliseconds (wall clock summed over workgroups) and task counts
    unsigned long long h[2 * MPCHOL_PROF_KINDS];
    int khz = 0;
    HIPCHK(hipMemcpy(h, BT.prog.prof, sizeof(h), hipMemcpyDeviceToHost));
    HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device));
    for (int k = 0; k < MPCHOL_PROF_KINDS; k++) {
      if (c->prof_mask & (1u << k)) {
        c->acc_ms[k] += khz > 0 ? (double)h[2 * k] / (double)khz : 0.0;
        c->acc_n[k] += (int64_t)h[2 * k + 1];
      }
    }
  }
  int worst = 0;
  for (int64_t i = 0; i < batch; i++) {
    const BatchInfo& I = BT.hinfo[i];
    if (info_host) {
      info_host[i].status = I.status;
      info_host[i].ir_iters = I.ir_iters;
      info_host[i].failed_index = I.failed_index;
      info_host[i].final_rel_corr = I.final_rel_corr;
      info_host[i].ms_factor = ms;
    }
    worst = std::max(worst, (int)I.status);
  }
  return worst;
}

// Quantize one column-major block with its power-of-two block scale into a
// K-contiguous copy (the operation every low-precision GEMM operand goes
// through).  Synchronizes the stream.
int mpchol_quantize(mpchol_ctx c, int64_t rows, int64_t cols, const double* src, int64_t lds,
                    int32_t prec, int32_t scale_mode, void* dst, int64_t ldq, double* scale_out,
                    void* stream) {
  if (!c) return -1;
  if (rows < 0) return -2;
  if (cols < 0) return -3;
  if (!src && rows > 0 && cols > 0) return -4;
  if (lds < std::max<int64_t>(1, rows)) return -5;
  if (prec != MPCHOL_F16 && prec != MPCHOL_E4M3) return -6;
  if (scale_mode < 0 || scale_mode > 2) return -7;
  if (!dst && rows > 0) return -8;
  if (ldq < ((cols + 15) / 16) * 16) return -9;
  if (rows > INT32_MAX || cols > INT32_MAX || ldq > INT32_MAX) return -2;
  scale_mode = operand_scale_mode(scale_mode, prec);
  if (rows == 0 || cols == 0) {
    if (scale_out) *scale_out = 1.0;
    return 0;
  }
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->device));
  MaxabsJob mj{};
  mj.src = 0;
  mj.rows = (int)rows;
  mj.cols = (int)cols;
  int np = (int)std::min<int64_t>(128, cols);
  mj.cpw = (int)((cols + np - 1) / np);
  mj.nparts = (int)((cols + mj.cpw - 1) / mj.cpw);
  mj.part0 = 0;
  mj.wg_start = 0;
  CastJob cj{};
  cj.src = 0;
  cj.dst = 0;
  cj.rows = (int)rows;
  cj.cols = (int)cols;
  cj.ldq = (int)ldq;
  cj.part0 = 0;
  cj.nparts = mj.nparts;
  cj.tiles_r = (int)((rows + 63) / 64);
  cj.tiles_c = (int)((ldq + 63) / 64);
  cj.wg_start = 0;
  int r = ensure_ws(c, 256, mj.nparts);
  if (r) return r;
  MaxabsJob* dm = nullptr;
  CastJob* dc = nullptr;
  HIPCHK(hipMalloc((void**)&dm, sizeof(mj)));
  HIPCHK(hipMalloc((void**)&dc, sizeof(cj)));
  HIPCHK(hipMemcpyAsync(dm, &mj, sizeof(mj), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dc, &cj, sizeof(cj), hipMemcpyHostToDevice, s));
  HIPCHK(launch_status_init(c->dst, s));
  HIPCHK(launch_maxabs(src, lds, dm, 1, mj.nparts, c->part, s));
  HIPCHK(launch_cast(src, lds, dc, 1, cj.tiles_r * cj.tiles_c, c->part, prec, scale_mode, dst,
                     c->dst, s));
  std::vector<double> hp(mj.nparts);
  HIPCHK(hipMemcpyAsync(hp.data(), c->part, sizeof(double) * mj.nparts, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(c->hst, c->dst, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipFree(dm));
  HIPCHK(hipFree(dc));
  double mx = 0.0;
  for (double v : hp) mx = std::max(mx, v);
  bool bad = !(mx <= 1.7976931348623157e308);
  if (scale_out) *scale_out = bad ? 1.0 : block_scale(mx, prec, scale_mode);
  return c->hst->nonfinite ? MPCHOL_NONFINITE : 0;
}

int mpchol_profile(mpchol_ctx c, uint32_t kind_mask) {
  if (!c) return -1;
  if (prof_collect(c)) return MPCHOL_HIP_ERROR;
  c->prof_mask = kind_mask;
  for (int k = 0; k < MPCHOL_PROF_KINDS; k++) {
    c->acc_ms[k] = 0.0;
    c->acc_work[k] = 0.0;
    c->acc_n[k] = 0;
  }
  return 0;
}

int mpchol_profile_read(mpchol_ctx c, double* ms, double* work, int64_t* launches) {
  if (!c) return -1;
  if (prof_collect(c)) return MPCHOL_HIP_ERROR;
  for (int k = 0; k < MPCHOL_PROF_KINDS; k++) {
    if (ms) ms[k] = c->acc_ms[k];
    if (work) work[k] = c->acc_work[k];
    if (launches) launches[k] = c->acc_n[k];
  }
  return 0;
}

// Plan introspection (host only, no device needed): flops by precision,
// leaf flops, quantize-cast bytes, launch count and workspace of (n, ldl, tree).
int mpchol_plan_stats(int64_t n, int64_t ldl, const mpchol_tree* tree, double* flops4,
                      double* leaf_flops, double* cast_bytes, int64_t* launches,
                      int64_t* ws_bytes) {
  if (n < 0) return -1;
  if (ldl < std::max<int64_t>(1, n)) return -2;
  int v = validate_tree(tree);
  if (v) return v;
  Plan P;
  build_plan(P, n, ldl, tree, false, 0, lookahead_on());
  for (int i = 0; i < 4; i++) flops4[i] = P.stats.flops[i];
  *leaf_flops = P.stats.leaf_flops;
  *cast_bytes = P.stats.cast_bytes;
  *launches = P.stats.n_launch;
  *ws_bytes = (int64_t)P.ws_bytes;
  return 0;
}

}  // extern "C"
