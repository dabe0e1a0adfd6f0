// Planner: walks Tree-POTRF (Algorithm 1), Tree-TRSM (Algorithm 2) and
// Tree-SYRK (Algorithm 3) on the host once per (n, ldl, descriptor) and emits
// the launches that carry them out on the GPU, in an order that respects every
// data dependency of the recursion (one stream):
//
//  - a GEMM issued by a Tree-POTRF node at depth l runs in that node's
//    precision (offdiag[min(l, nlevels-1)] or node_prec[node]); FP16 / E4M3
//    operands are quantized first (max-abs, power-of-two scale, cast), FP32
//    operands are scaled and rounded while loaded, FP64 operands are used as is;
//  - every GEMM and leaf SYRK of one Tree-SYRK is independent of the others
//    (disjoint outputs, read-only operand panel), so each Tree-SYRK becomes one
//    max-abs launch, one cast launch and one grouped GEMM launch per precision;
//  - Tree-TRSM is a chain (each GEMM consumes the previous leaf solve);
//  - a leaf of the precision tree larger than the kernel leaf (128) is factored
//    / solved by an all-leaf-precision sub-recursion down to 128; this is a
//    leaf-precision Cholesky (resp. triangular solve) of that leaf;
//  - GEMM launches use 128 x 128 output tiles (256 x 256 for large FP16
//    groups), or 64 x 64 when 128-tiles would
//    leave most of the 256 compute units idle.
#include "plan.h"

#include <algorithm>
#include <cstring>
#include <map>
#include <sstream>

namespace mpc {

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int64_t rup(int64_t a, int64_t b) { return cdiv(a, b) * b; }

int64_t split_rule(int64_t m, int32_t align) {
  int64_t h = m / 2;
  if (align > 1) h = cdiv(h, align) * align;
  if (h < 1) h = 1;
  if (h > m - 1) h = m - 1;
  return h;
}

int validate_tree(const mpchol_tree* t) {
  if (!t) return -7;
  if (t->abi_version != MPCHOL_ABI_VERSION) return -7;
  if (t->leaf < 1 || t->split_align < 1) return -7;
  if (t->nlevels < 1 || t->nlevels > MPCHOL_MAX_LEVELS) return -7;
  for (int i = 0; i < t->nlevels; i++)
    if (t->offdiag[i] < MPCHOL_E4M3 || t->offdiag[i] > MPCHOL_F64) return -7;
  if (t->leaf_prec != MPCHOL_F32 && t->leaf_prec != MPCHOL_F64) return -7;
  if (t->syrk_leaf_mode < 0 || t->syrk_leaf_mode > 1) return -7;
  if (t->scale_mode < 0 || t->scale_mode > 2) return -7;
  if (t->scale_tile != 0) return MPCHOL_NOT_SUPPORTED;
  if (t->leaf_trsm != 0 && t->leaf_trsm != 1) return -7;
  if (t->n_nodes < 0 || (t->n_nodes > 0 && !t->node_prec)) return -7;
  for (int64_t i = 0; i < t->n_nodes; i++)
    if (t->node_prec[i] > MPCHOL_F64) return -7;
  return 0;
}

std::string plan_key(int64_t n, int64_t ldl, const mpchol_tree* t) {
  std::ostringstream o;
  o << n << ':' << ldl << ':' << t->leaf << ':' << t->split_align << ':' << t->leaf_prec << ':'
    << t->syrk_leaf_mode << ':' << t->scale_mode << ':' << t->leaf_trsm << ':';
  for (int i = 0; i < t->nlevels; i++) o << t->offdiag[i] << ',';
  o << ':';
  for (int64_t i = 0; i < t->n_nodes; i++) o << (int)t->node_prec[i] << ',';
  return o.str();
}

namespace {

constexpr int kMaxParts = 128;

struct Builder {
  Plan& P;
  const mpchol_tree& t;
  int64_t ldl;
  bool single_wg = false;
  int tile_force = 0;
  // (origin, order) of a diagonal block with an inverse -> (slot, element offset)
  std::map<std::pair<int64_t, int64_t>, std::pair<int, int64_t>> inv_slot;

  // FP64 leaves of the single-matrix path solve their TRSMs through the inverse
  bool use_inverse() const { return !single_wg && t.leaf_prec == F64 && t.leaf_trsm == 0; }
  int64_t next_node = 0;
  size_t ws_cursor = 0;   // bytes used by the current group of quantized copies
  int64_t part_cursor = 0;
  // lookahead: groups whose copies and partials go to bank 1 (offset past
  // bank 0's high-water marks once the plan is complete)
  int lookahead = 0;   // 0 off; 1 every Tree-SYRK; 2 only FP32 / FP64 ones
  bool tail_pending = false;
  int bank = 0;
  size_t ws_max[2] = {0, 0};
  int64_t parts_max[2] = {0, 0};
  struct BankRange { size_t mj0, mj1, cj0, cj1, gp0, gp1; int esz; bool quant; };
  std::vector<BankRange> bank1;

  Builder(Plan& p, const mpchol_tree& tr, int64_t ld) : P(p), t(tr), ldl(ld) {}

  int64_t off(int64_t r, int64_t c) const { return r + c * ldl; }

  int node_prec(int64_t id, int depth) const {
    if (id < (int64_t)P.node_prec.size() && P.node_prec[id] >= 0) return P.node_prec[id];
    return t.offdiag[std::min(depth, t.nlevels - 1)];
  }

  void begin_group() {
    ws_cursor = 0;
    part_cursor = 0;
  }
  void end_group() {
    ws_max[bank] = std::max(ws_max[bank], ws_cursor);
    parts_max[bank] = std::max(parts_max[bank], part_cursor);
    P.ws_bytes = std::max(P.ws_bytes, ws_cursor);
    P.parts = std::max(P.parts, part_cursor);
  }

  // Bank 1 after bank 0: shift the offsets of every bank-1 group.
  void place_banks() {
    if (bank1.empty()) return;
    const size_t ws0 = (size_t)rup((int64_t)ws_max[0], 256);
    const int64_t p0 = parts_max[0];
    for (const BankRange& r : bank1) {
      for (size_t i = r.mj0; i < r.mj1; i++) P.maxabs[i].part0 += (int)p0;
      for (size_t i = r.cj0; i < r.cj1; i++) {
        P.casts[i].dst += (int64_t)(ws0 / r.esz);
        P.casts[i].part0 += (int)p0;
      }
      for (size_t i = r.gp0; i < r.gp1; i++) {
        GemmProb& g = P.gemms[i];
        if (r.quant) {
          g.x += (int64_t)(ws0 / r.esz);
          g.y += (int64_t)(ws0 / r.esz);
        }
        if (g.xnparts > 0) g.xpart0 += (int)p0;
        if (g.ynparts > 0) g.ypart0 += (int)p0;
      }
    }
    P.ws_bytes = ws0 + ws_max[1];
    P.parts = p0 + parts_max[1];
  }

  // Max-abs job for block (r, c, rows, cols); returns (part0, nparts).
  std::pair<int, int> add_maxabs(std::vector<MaxabsJob>& jobs, int64_t r, int64_t c, int rows,
                                 int cols) {
    MaxabsJob j{};
    j.src = off(r, c);
    j.rows = rows;
    j.cols = cols;
    int np = std::min(kMaxParts, cols);
    j.cpw = (int)cdiv(cols, np);
    j.nparts = (int)cdiv(cols, j.cpw);
    j.part0 = (int)part_cursor;
    part_cursor += j.nparts;
    jobs.push_back(j);
    return {j.part0, j.nparts};
  }

  int64_t add_cast(std::vector<CastJob>& jobs, int prec, int64_t r, int64_t c, int rows, int cols,
                   std::pair<int, int> parts, int* ldq_out) {
    int esz = prec == F32 ? 4 : prec == F16 ? 2 : 1;
    CastJob j{};
    j.src = off(r, c);
    j.rows = rows;
    j.cols = cols;
    j.ldq = (int)rup(cols, 16);
    ws_cursor = (size_t)rup((int64_t)ws_cursor, 256);
    j.dst = (int64_t)(ws_cursor / esz);
    ws_cursor += (size_t)rows * j.ldq * esz;
    j.part0 = parts.first;
    j.nparts = parts.second;
    j.tiles_r = (int)cdiv(rows, 64);
    j.tiles_c = (int)cdiv(j.ldq, 64);
    j.tpu = 0;
    jobs.push_back(j);
    P.stats.cast_bytes += (double)rows * cols * (8.0 + esz);
    *ldq_out = j.ldq;
    return j.dst;
  }

  struct Node {
    int64_t cr, cc;  // C block origin
    int m, n;        // C block size
    int64_t xr, xc;  // X block origin (m x k)
    int64_t yr, yc;  // Y block origin (n x k)
    int k;
    int lower;
    int prec;
  };

  // Emit maxabs / cast / grouped GEMM launches for independent GEMM nodes that
  // share one precision.
  // head_count >= 0: the first head_count nodes form the GEMM launch of the
  // caller's stream and the rest a launch on the side stream, issued first
  // (after the casts both read), with the group's copies in bank 1.
  void emit_group(const std::vector<Node>& nodes, int prec, bool with_parts,
                  int head_count = -1) {
    if (nodes.empty()) return;
    begin_group();
    const size_t mj_first = P.maxabs.size(), cj_first = P.casts.size(),
                 gp_first = P.gemms.size();
    std::vector<MaxabsJob> mj;
    std::vector<CastJob> cj;
    std::vector<GemmProb> gp;
    // FP32 operands of the multi-workgroup path are copied too (4 bytes per
    // element and K-contiguous instead of the FP64 factor), always in one
    // pass: FP32 blocks are never scaled up, so a block's scale is 1 unless
    // its max-abs exceeds the FP32 range
    const bool quant = prec == F16 || prec == E4M3 || (prec == F32 && !single_wg);
    // FP16 without upward scaling (scale_mode 0 or 2) and FP32: one pass casts
    // at scale 1 and records the max-abs
    const bool single_pass =
        (prec == F16 && t.scale_mode != 1) || (prec == F32 && !single_wg);
    if (single_pass) with_parts = false;
    // Single pass: operands of the group with the same columns whose rows
    // overlap or touch share one scale-1 copy of the union of their rows (a
    // SYRK's sub-products read every row of its operand once per recursion
    // level).  Each operand keeps its own block scale: the GEMM reduces the
    // copy's 64 x 64 tile maxima over the operand's rows, and when that
    // scale is not 1 it quantizes the operand from the factor instead of
    // reading the copy.  Sharing needs operand rows on 64-row tile
    // boundaries of the union, so the tiles reduced are exactly the
    // operand's; an operand that is not aligned gets a copy of its own.
    struct OpView { int64_t dst, src; int part0, nparts, ldq; };
    std::vector<OpView> views;
    std::vector<int> node_x(nodes.size(), -1), node_y(nodes.size(), -1);
    if (single_pass) {
      struct Opd { int64_t r, c; int rows, k; };
      std::vector<Opd> ops;
      for (size_t i = 0; i < nodes.size(); i++) {
        const Node& nd = nodes[i];
        node_x[i] = (int)ops.size();
        ops.push_back({nd.xr, nd.xc, nd.m, nd.k});
        if (nd.lower) {
          node_y[i] = node_x[i];
        } else {
          node_y[i] = (int)ops.size();
          ops.push_back({nd.yr, nd.yc, nd.n, nd.k});
        }
      }
      std::vector<int> opd_view(ops.size(), -1);
      std::vector<int64_t> base_row;   // first row of each shared copy (index = cast job)
      std::map<std::pair<int64_t, int>, std::vector<int>> cls;
      for (int i = 0; i < (int)ops.size(); i++) cls[{ops[i].c, ops[i].k}].push_back(i);
      auto make_base = [&](int64_t r, int64_t c, int rows, int k) {
        int ldq = 0;
        add_cast(cj, prec, r, c, rows, k, {0, 0}, &ldq);
        CastJob& j = cj.back();
        // work units of tpu tiles along a tile row, one partial each (unit
        // row-major), so that an operand's rows are a contiguous range of at
        // most about 1024 partials
        j.tpu = (int)std::min<int64_t>(j.tiles_c, cdiv((int64_t)j.tiles_r * j.tiles_c, 1024));
        j.part0 = (int)part_cursor;
        j.nparts = j.tiles_r * (int)cdiv(j.tiles_c, j.tpu);
        part_cursor += j.nparts;
        base_row.resize(cj.size(), 0);
        base_row.back() = r;
        return (int)cj.size() - 1;
      };
      auto make_view = [&](int oi, int bi) {
        const Opd& o = ops[oi];
        const CastJob& b = cj[bi];
        const int64_t dr = o.r - base_row[bi];
        OpView v{};
        v.dst = b.dst + dr * b.ldq;
        v.src = off(o.r, o.c);
        const int units_r = (int)cdiv(b.tiles_c, b.tpu);   // units per tile row
        v.part0 = b.part0 + (int)(dr / 64) * units_r;
        v.nparts = (int)(cdiv(dr + o.rows, 64) - dr / 64) * units_r;
        v.ldq = b.ldq;
        opd_view[oi] = (int)views.size();
        views.push_back(v);
      };
      for (auto& kv : cls) {
        std::vector<int>& idx = kv.second;
        std::sort(idx.begin(), idx.end(), [&](int a, int b) {
          return ops[a].r != ops[b].r ? ops[a].r < ops[b].r : ops[a].rows > ops[b].rows;
        });
        size_t i = 0;
        while (i < idx.size()) {
          // union of rows overlapping or touching
          int64_t u0 = ops[idx[i]].r, u1 = u0 + ops[idx[i]].rows;
          size_t j = i + 1;
          while (j < idx.size() && ops[idx[j]].r <= u1) {
            u1 = std::max(u1, ops[idx[j]].r + ops[idx[j]].rows);
            j++;
          }
          std::vector<int> aligned, other;
          for (size_t q = i; q < j; q++) {
            const Opd& o = ops[idx[q]];
            const int64_t a0 = o.r - u0, a1 = o.r + o.rows - u0;
            if (a0 % 64 == 0 && (a1 % 64 == 0 || o.r + o.rows == u1)) aligned.push_back(idx[q]);
            else other.push_back(idx[q]);
          }
          if (aligned.size() == 1 && ops[aligned[0]].r == u0 && ops[aligned[0]].rows == u1 - u0) {
            other.push_back(aligned[0]);
            aligned.clear();
          }
          if (!aligned.empty()) {
            // the shared copy spans the aligned operands' rows only
            int64_t s0 = INT64_MAX, s1 = INT64_MIN;
            for (int oi : aligned) {
              s0 = std::min(s0, ops[oi].r);
              s1 = std::max(s1, ops[oi].r + ops[oi].rows);
            }
            bool ok = true;
            for (int oi : aligned) {
              const int64_t a0 = ops[oi].r - s0, a1 = ops[oi].r + ops[oi].rows - s0;
              if (a0 % 64 != 0 || (a1 % 64 != 0 && ops[oi].r + ops[oi].rows != s1)) ok = false;
            }
            if (ok) {
              const int bi = make_base(s0, kv.first.first, (int)(s1 - s0), kv.first.second);
              for (int oi : aligned) make_view(oi, bi);
            } else {
              other.insert(other.end(), aligned.begin(), aligned.end());
            }
          }
          for (int oi : other) {
            if (opd_view[oi] >= 0) continue;
            const int bi = make_base(ops[oi].r, ops[oi].c, ops[oi].rows, ops[oi].k);
            make_view(oi, bi);
          }
          i = j;
        }
      }
      for (size_t i = 0; i < nodes.size(); i++) {
        node_x[i] = opd_view[node_x[i]];
        node_y[i] = opd_view[node_y[i]];
      }
    }
    for (size_t ni = 0; ni < nodes.size(); ni++) {
      const Node& nd = nodes[ni];
      GemmProb g{};
      g.c = off(nd.cr, nd.cc);
      g.m = nd.m;
      g.n = nd.n;
      g.k = nd.k;
      g.lower = nd.lower;
      std::pair<int, int> px{0, 0}, py{0, 0};
      if (with_parts) {
        px = add_maxabs(mj, nd.xr, nd.xc, nd.m, nd.k);
        py = nd.lower ? px : add_maxabs(mj, nd.yr, nd.yc, nd.n, nd.k);
      }
      g.xpart0 = px.first;
      g.xnparts = px.second;
      g.ypart0 = py.first;
      g.ynparts = py.second;
      if (single_pass) {
        const OpView& vx = views[node_x[ni]];
        const OpView& vy = views[node_y[ni]];
        g.x = vx.dst;
        g.xsrc = vx.src;
        g.ldx = vx.ldq;
        g.xpart0 = vx.part0;
        g.xnparts = vx.nparts;
        g.y = vy.dst;
        g.ysrc = vy.src;
        g.ldy = vy.ldq;
        g.ypart0 = vy.part0;
        g.ynparts = vy.nparts;
      } else if (quant) {
        int ldx = 0, ldy = 0;
        g.x = add_cast(cj, prec, nd.xr, nd.xc, nd.m, nd.k, px, &ldx);
        g.ldx = ldx;
        if (nd.lower) {
          g.y = g.x;
          g.ldy = ldx;
        } else {
          g.y = add_cast(cj, prec, nd.yr, nd.yc, nd.n, nd.k, py, &ldy);
          g.ldy = ldy;
        }
        g.xsrc = g.ysrc = -1;
      } else {
        g.x = off(nd.xr, nd.xc);
        g.y = off(nd.yr, nd.yc);
        g.xsrc = g.ysrc = -1;
        g.ldx = g.ldy = (int)ldl;
      }
      double fl = nd.lower ? (double)nd.m * (nd.m + 1) * nd.k : 2.0 * nd.m * nd.n * nd.k;
      P.stats.flops[prec] += fl;
      gp.push_back(g);
    }
    if (!mj.empty()) {
      Launch L{Launch::MAXABS, prec};
      L.first = (int)P.maxabs.size();
      L.count = (int)mj.size();
      int wg = 0;
      for (auto& j : mj) {
        j.wg_start = wg;
        wg += j.nparts;
      }
      L.total = wg;
      P.maxabs.insert(P.maxabs.end(), mj.begin(), mj.end());
      P.launches.push_back(L);
    }
    if (!cj.empty()) {
      Launch L{Launch::CAST, prec};
      L.first = (int)P.casts.size();
      L.count = (int)cj.size();
      L.a0 = single_pass ? 1 : 0;
      int wg = 0;
      for (auto& j : cj) {
        j.wg_start = wg;
        wg += single_pass ? j.tiles_r * (int)cdiv(j.tiles_c, j.tpu) : j.tiles_r * j.tiles_c;
      }
      L.total = wg;
      P.casts.insert(P.casts.end(), cj.begin(), cj.end());
      P.launches.push_back(L);
    }
    // GEMM launch over the problems [g0, g1) of gp (side: on the side stream)
    auto gemm_launch = [&](size_t g0, size_t g1, int side) {
      Launch L{Launch::GEMM, prec};
      L.side = side;
      L.first = (int)P.gemms.size();
      L.count = (int)(g1 - g0);
      std::vector<GemmProb> sub(gp.begin() + g0, gp.begin() + g1);
      auto tiles_of = [&](int T) {
        int64_t tot = 0;
        for (auto& g : sub) {
          int64_t tm = cdiv(g.m, T);
          tot += g.lower ? tm * (tm + 1) / 2 : tm * cdiv(g.n, T);
        }
        return tot;
      };
      if (tile_force) {
        L.tile = tile_force;
      } else if (single_wg) {
        int mn = 1 << 30;
        for (auto& g : sub) mn = std::min(mn, std::min(g.m, g.n));
        L.tile = mn >= 128 ? 128 : 64;
      } else {
        // 128 x 128 tiles unless that leaves most of the 256 CUs idle; FP32 /
        // FP64 groups with fewer than 256 64-tiles take 32-tiles.  Large FP16
        // groups take the 256 x 256 kernel (operands loaded straight into
        // LDS), which needs K % 64 == 0 and operand blocks addressable with
        // 31-bit byte offsets
        L.tile = tiles_of(128) >= 256 ? 128 : 64;
        if (L.tile == 64 && (prec == F32 || prec == F64) && tiles_of(64) < 256) L.tile = 32;
        if (prec == F16 && tiles_of(256) >= 256) {
          bool ok = true;
          for (auto& g : sub)
            ok = ok && g.k % 64 == 0 && (int64_t)g.m * g.ldx * 2 < ((int64_t)1 << 31) &&
                 (int64_t)g.n * g.ldy * 2 < ((int64_t)1 << 31);
          if (ok) L.tile = 256;
        }
      }
      int tiles = 0;
      for (auto& g : sub) {
        g.tiles_m = (int)cdiv(g.m, L.tile);
        g.tiles_n = (int)cdiv(g.n, L.tile);
        g.tile_start = tiles;
        tiles += g.lower ? g.tiles_m * (g.tiles_m + 1) / 2 : g.tiles_m * g.tiles_n;
      }
      L.total = tiles;
      P.gemms.insert(P.gemms.end(), sub.begin(), sub.end());
      P.launches.push_back(L);
      if (side) P.n_side++;
    };
    if (head_count >= 0 && head_count < (int)gp.size()) {
      gemm_launch((size_t)head_count, gp.size(), 1);
      if (head_count > 0) gemm_launch(0, (size_t)head_count, 0);
    } else {
      gemm_launch(0, gp.size(), 0);
    }
    end_group();
    if (bank == 1) {
      const int esz = prec == F32 ? 4 : prec == F16 ? 2 : 1;
      bank1.push_back({mj_first, P.maxabs.size(), cj_first, P.casts.size(), gp_first,
                       P.gemms.size(), esz, quant});
    }
  }

  void gemm_one(const Node& nd, bool with_parts) { emit_group({nd}, nd.prec, with_parts); }

  // ---- leaf precision: kernels of size <= kKernelLeaf, sub-recursion above
  int64_t leaf_split(int64_t m) const {
    int64_t h = cdiv(m / 2, kKernelLeaf) * kKernelLeaf;
    return std::max<int64_t>(1, std::min(h, m - 1));
  }

  // slot >= 0: the inverse goes into that slot at element offset off (the
  // second half of a joined 256-leaf); otherwise a new slot
  void leaf_potrf(int64_t i0, int64_t m, int slot = -1, int64_t off = 0) {
    if (m <= 0) return;
    if (m <= kKernelLeaf) {
      Launch L{Launch::POTRF, t.leaf_prec};
      L.a0 = i0;
      L.a1 = m;
      if (use_inverse()) {
        // the inverse is formed by the same launch (a2 = 1) into slot `first`
        L.a2 = 1;
        L.first = slot >= 0 ? slot : P.ninv++;
        L.off = slot >= 0 ? off : 0;
        inv_slot[{i0, m}] = {L.first, L.off};
      }
      P.launches.push_back(L);
      P.stats.leaf_flops += (double)m * m * m / 3.0;
      return;
    }
    int64_t m1 = leaf_split(m), m2 = m - m1;
    // a leaf of two kernel leaves gets one inverse: the halves' inverses joined
    const bool join = use_inverse() && m <= kInvLd;
    const int js = join ? P.ninv++ : -1;
    leaf_potrf(i0, m1, js, 0);
    leaf_trsm(i0 + m1, m2, i0, m1);
    gemm_one(Node{i0 + m1, i0 + m1, (int)m2, (int)m2, i0 + m1, i0, i0 + m1, i0, (int)m1, 1,
                  t.leaf_prec},
             false);
    leaf_potrf(i0 + m1, m2, js, m1 + m1 * (int64_t)kInvLd);
    if (join) {
      Launch J{Launch::INVJOIN, F64};
      J.a0 = i0;
      J.a1 = m;
      J.a2 = m1;
      J.first = js;
      P.launches.push_back(J);
      inv_slot[{i0, m}] = {js, 0};
    }
  }

  void leaf_trsm(int64_t r0, int64_t m, int64_t c0, int64_t k) {
    if (m <= 0 || k <= 0) return;
    auto it = use_inverse() ? inv_slot.find({c0, k}) : inv_slot.end();
    if (it != inv_slot.end() || k <= kKernelLeaf) {
      Launch L{Launch::TRSM, t.leaf_prec};
      L.a0 = r0;
      L.a1 = m;
      L.a2 = c0;
      L.a3 = k;
      L.first = -1;
      if (it != inv_slot.end()) {
        L.first = it->second.first;
        L.off = it->second.second;
      }
      P.launches.push_back(L);
      P.stats.leaf_flops += (double)m * k * k;
      return;
    }
    int64_t k1 = leaf_split(k), k2 = k - k1;
    leaf_trsm(r0, m, c0, k1);
    gemm_one(Node{r0, c0 + k1, (int)m, (int)k2, r0, c0, c0 + k1, c0, (int)k1, 0, t.leaf_prec},
             false);
    leaf_trsm(r0, m, c0 + k1, k2);
  }

  // ---- Algorithm 2: B <- B L^{-T}, B = (r0, c0, m x k), L = (c0, c0, k x k)
  void trsm(int64_t r0, int64_t m, int64_t c0, int64_t k, int prec) {
    if (m <= 0 || k <= 0) return;
    if (std::min(m, k) <= t.leaf) {
      leaf_trsm(r0, m, c0, k);
      return;
    }
    int64_t k1 = split_rule(k, t.split_align), k2 = k - k1;
    trsm(r0, m, c0, k1, prec);
    gemm_one(Node{r0, c0 + k1, (int)m, (int)k2, r0, c0, c0 + k1, c0, (int)k1, 0, prec},
             prec != F64);
    trsm(r0, m, c0 + k1, k2, prec);
  }

  // ---- Algorithm 3: C <- C - P P^T (lower), C = (c0, c0, s x s), P = (c0, p0, s x K)
  void syrk_collect(int64_t c0, int64_t s, int64_t p0, int64_t K, int prec,
                    std::vector<Node>& out) {
    if (s <= 0) return;
    if (s <= t.leaf) {
      int p = t.syrk_leaf_mode ? t.leaf_prec : prec;
      out.push_back(Node{c0, c0, (int)s, (int)s, c0, p0, c0, p0, (int)K, 1, p});
      return;
    }
    int64_t s1 = split_rule(s, t.split_align), s2 = s - s1;
    syrk_collect(c0, s1, p0, K, prec, out);
    out.push_back(Node{c0 + s1, c0, (int)s2, (int)s1, c0 + s1, p0, c0, p0, (int)K, 0, prec});
    syrk_collect(c0 + s1, s2, p0, K, prec, out);
  }

  // Returns true when the Tree-SYRK was split for lookahead (its tail is then
  // in flight on the side stream).
  bool syrk(int64_t c0, int64_t s, int64_t p0, int64_t K, int prec, bool split = false) {
    if (s <= 0 || K <= 0) return false;
    std::vector<Node> all;
    if (split && s > t.leaf) {
      // head: the leading block [c0, c0 + s1) that Tree-POTRF of this block
      // factors first; tail: the block below it and the trailing block
      const int64_t s1 = split_rule(s, t.split_align), s2 = s - s1;
      syrk_collect(c0, s1, p0, K, prec, all);
      const int head = (int)all.size();
      all.push_back(Node{c0 + s1, c0, (int)s2, (int)s1, c0 + s1, p0, c0, p0, (int)K, 0, prec});
      syrk_collect(c0 + s1, s2, p0, K, prec, all);
      bool one_prec = true;
      for (auto& nd : all) one_prec = one_prec && nd.prec == prec;
      if (one_prec) {
        bank = 1;
        emit_group(all, prec, prec != F64, head);
        bank = 0;
        return true;
      }
      all.clear();
    }
    syrk_collect(c0, s, p0, K, prec, all);
    for (int q = E4M3; q <= F64; q++) {
      std::vector<Node> sel;
      for (auto& nd : all)
        if (nd.prec == q) sel.push_back(nd);
      emit_group(sel, q, q != F64);
    }
    return false;
  }

  // ---- Tree-TRSM / Tree-SYRK on their own: the precision list is read by
  // the depth of their own recursion (the GEMM at depth d, and a leaf SYRK
  // reached at depth d, in offdiag[min(d, nlevels - 1)])
  int level_prec(int depth) const { return t.offdiag[std::min(depth, t.nlevels - 1)]; }

  // Inverse of the FP64 diagonal block (i0, m), m <= kInvLd, for the leaf
  // TRSMs that follow (a kernel leaf, or two joined).
  void leaf_inverse(int64_t i0, int64_t m) {
    if (!use_inverse() || m > kInvLd || inv_slot.count({i0, m})) return;
    auto trinv = [&](int64_t a0, int64_t mm, int slot, int64_t off) {
      Launch L{Launch::TRINV, F64};
      L.a0 = a0;
      L.a1 = mm;
      L.first = slot;
      L.off = off;
      P.launches.push_back(L);
      P.stats.leaf_flops += (double)mm * mm * mm / 3.0;
    };
    const int js = P.ninv++;
    if (m <= kKernelLeaf) {
      trinv(i0, m, js, 0);
    } else {
      const int64_t m1 = leaf_split(m), m2 = m - m1;
      trinv(i0, m1, js, 0);
      trinv(i0 + m1, m2, js, m1 + m1 * (int64_t)kInvLd);
      Launch J{Launch::INVJOIN, F64};
      J.a0 = i0;
      J.a1 = m;
      J.a2 = m1;
      J.first = js;
      P.launches.push_back(J);
    }
    inv_slot[{i0, m}] = {js, 0};
  }

  void trsm_leaf_blocks(int64_t m, int64_t c0, int64_t k) {
    if (m <= 0 || k <= 0) return;
    if (std::min(m, k) <= t.leaf) {
      leaf_inverse(c0, k);
      return;
    }
    const int64_t k1 = split_rule(k, t.split_align);
    trsm_leaf_blocks(m, c0, k1);
    trsm_leaf_blocks(m, c0 + k1, k - k1);
  }

  void trsm_depth(int64_t r0, int64_t m, int64_t c0, int64_t k, int depth) {
    if (m <= 0 || k <= 0) return;
    if (std::min(m, k) <= t.leaf) {
      leaf_trsm(r0, m, c0, k);
      return;
    }
    const int prec = level_prec(depth);
    const int64_t k1 = split_rule(k, t.split_align), k2 = k - k1;
    trsm_depth(r0, m, c0, k1, depth + 1);
    gemm_one(Node{r0, c0 + k1, (int)m, (int)k2, r0, c0, c0 + k1, c0, (int)k1, 0, prec},
             prec != F64);
    trsm_depth(r0, m, c0 + k1, k2, depth + 1);
  }

  void syrk_collect_depth(int64_t c0, int64_t s, int64_t p0, int64_t K, int depth,
                          std::vector<Node>& out) {
    if (s <= 0) return;
    if (s <= t.leaf) {
      const int p = t.syrk_leaf_mode ? t.leaf_prec : level_prec(depth);
      out.push_back(Node{c0, c0, (int)s, (int)s, c0, p0, c0, p0, (int)K, 1, p});
      return;
    }
    const int64_t s1 = split_rule(s, t.split_align), s2 = s - s1;
    syrk_collect_depth(c0, s1, p0, K, depth + 1, out);
    out.push_back(Node{c0 + s1, c0, (int)s2, (int)s1, c0 + s1, p0, c0, p0, (int)K, 0,
                       level_prec(depth)});
    syrk_collect_depth(c0 + s1, s2, p0, K, depth + 1, out);
  }

  void syrk_depth(int64_t c0, int64_t s, int64_t p0, int64_t K) {
    if (s <= 0 || K <= 0) return;
    std::vector<Node> all;
    syrk_collect_depth(c0, s, p0, K, 0, all);
    for (int q = E4M3; q <= F64; q++) {
      std::vector<Node> sel;
      for (auto& nd : all)
        if (nd.prec == q) sel.push_back(nd);
      emit_group(sel, q, q != F64);
    }
  }

  // ---- Algorithm 1.  join_tail: the Tree-SYRK that updated this block left
  // its tail (everything but the leading block) on the side stream; the
  // Tree-TRSM below the leading block waits for it.
  void potrf(int64_t i0, int64_t m, int depth, bool join_tail = false) {
    if (m <= 0) return;
    if (m <= t.leaf) {
      leaf_potrf(i0, m);
      return;
    }
    int64_t id = next_node++;
    int p = node_prec(id, depth);
    int64_t m1 = split_rule(m, t.split_align), m2 = m - m1;
    potrf(i0, m1, depth + 1);
    if (depth == 0) {
      P.split1 = m1;
      P.first_outer = (int)P.launches.size();
    }
    const size_t first_trsm = P.launches.size();
    trsm(i0 + m1, m2, i0, m1, p);
    if (join_tail) {
      P.launches[first_trsm].wait_side = 1;
      tail_pending = false;
    }
    const bool split = lookahead && !single_wg && !tail_pending && m2 > t.leaf &&
                       (lookahead == 1 || p == F32 || p == F64);
    const bool tail = syrk(i0 + m1, m2, i0, m1, p, split);
    if (tail) tail_pending = true;
    potrf(i0 + m1, m2, depth + 1, tail);
  }
};

}  // namespace

static void tree_nodes_rec(int64_t i0, int64_t m, int32_t depth, const mpchol_tree* t,
                           std::vector<PolicyNodeRec>& out) {
  if (m <= 0 || m <= t->leaf) return;
  const int64_t m1 = split_rule(m, t->split_align);
  out.push_back({i0, m, m1, depth});
  tree_nodes_rec(i0, m1, depth + 1, t, out);
  tree_nodes_rec(i0 + m1, m - m1, depth + 1, t, out);
}

void tree_nodes(int64_t n, const mpchol_tree* t, std::vector<PolicyNodeRec>& out) {
  out.clear();
  tree_nodes_rec(0, n, 0, t, out);
}

static void plan_init(Plan& P, int64_t n, int64_t ldl, const mpchol_tree* t) {
  P.n = n;
  P.ldl = ldl;
  P.tree = *t;
  P.node_prec.clear();
  P.tree.node_prec = nullptr;
  P.tree.n_nodes = 0;
}

void build_trsm_plan(Plan& P, int64_t m, int64_t k, int64_t ldl, const mpchol_tree* t) {
  plan_init(P, m + k, ldl, t);
  Builder B(P, P.tree, ldl);
  B.trsm_leaf_blocks(m, 0, k);
  B.trsm_depth(k, m, 0, k, 0);
  P.stats.n_launch = (int64_t)P.launches.size();
}

void build_syrk_plan(Plan& P, int64_t n, int64_t k, int64_t ldl, const mpchol_tree* t) {
  plan_init(P, n + k, ldl, t);
  Builder B(P, P.tree, ldl);
  B.syrk_depth(k, n, 0, k);
  P.stats.n_launch = (int64_t)P.launches.size();
}

void build_plan(Plan& P, int64_t n, int64_t ldl, const mpchol_tree* t, bool single_wg, int tile,
                int lookahead) {
  P.n = n;
  P.ldl = ldl;
  P.tree = *t;
  P.node_prec.assign(t->node_prec, t->node_prec + t->n_nodes);
  P.tree.node_prec = nullptr;
  Builder B(P, P.tree, ldl);
  B.single_wg = single_wg;
  B.tile_force = tile;
  B.lookahead = single_wg ? 0 : lookahead;
  B.potrf(0, n, 0);
  B.place_banks();
  P.stats.n_launch = (int64_t)P.launches.size();
}

}  // namespace mpc
