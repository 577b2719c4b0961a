// Planner: turns (algorithm, depth, cutoff, n, dtype) into the descriptors of
// one fused level - the pre-addition stage, the grouped leaf products with
// their epilogue post-additions, and the outer post-addition stage - plus
// the workspace size.  Plans are immutable and cached; their descriptors live
// in one device allocation made on first use.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include <algorithm>

#include "mf_internal.h"

namespace mf {

Plan::~Plan() {
  if (dev) (void)hipFree(dev);
}

namespace {

// Leaf products allowed in one plan.
constexpr int64_t kMaxLeafProducts = 1 << 16;

int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }
int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  while (e-- > 0) r *= b;
  return r;
}

// A block of the recursion: a view (src, offset, ld) of a matrix or of a
// workspace buffer, valid over vr x vc (virtual zeros beyond), standing for
// scale times the viewed entries.
struct Blk {
  int32_t src = SRC_A;
  int64_t off = 0;
  int32_t ld = 0;
  int32_t vr = 0, vc = 0;
  double scale = 1.0;
  bool zero = true;
  // BF16 leaves: the staging set that forms this leaf operand and its
  // coefficients (see Plan::bf_sets)
  int32_t stage_set = -1, stage_coef = -1;
};

// Part k (row-major in a split into pc columns of parts) of block b; every
// part is sr x sc.
Blk quarter(const Blk& b, int k, int pc, int64_t sr, int64_t sc) {
  Blk q = b;
  const int64_t r0 = (int64_t)(k / pc) * sr, c0 = (int64_t)(k % pc) * sc;
  q.vr = (int32_t)std::max<int64_t>(0, std::min<int64_t>(sr, b.vr - r0));
  q.vc = (int32_t)std::max<int64_t>(0, std::min<int64_t>(sc, b.vc - c0));
  q.zero = b.zero || q.vr == 0 || q.vc == 0;
  if (q.zero) {
    q.vr = q.vc = 0;
    q.off = 0;
  } else {
    q.off = b.off + r0 * b.ld + c0;
  }
  return q;
}
Blk quarter(const Blk& b, int k, int p, int64_t s) { return quarter(b, k, p, s, s); }

CombIn as_input(const Blk& b) {
  CombIn in{};
  in.off = b.off;
  in.src = b.src;
  in.ld = b.ld;
  in.vr = b.zero ? 0 : b.vr;
  in.vc = b.zero ? 0 : b.vc;
  return in;
}

// A three-factor Kronecker composition of <2,2,2;7> algorithms (<8,8,8;343>):
// its levels run on the factor-by-factor combination kernels.
bool is_kron3(const Algo& a) {
  if (a.factors.size() != 3) return false;
  for (const Algo& f : a.factors)
    if (f.p != 2 || f.R != 7) return false;
  return true;
}

// Block index (row-major in the 8 x 8 split) of factor-order index
// t = 16 t1 + 4 t2 + t3, where t_f = 2 i_f + j_f is the block of factor f.
int kron3_block(int t) {
  const int t1 = t / 16, t2 = (t / 4) % 4, t3 = t % 4;
  const int I = 4 * (t1 / 2) + 2 * (t2 / 2) + t3 / 2;
  const int J = 4 * (t1 % 2) + 2 * (t2 % 2) + t3 % 2;
  return I * 8 + J;
}

// The three 4 x 7 factor matrices of X (U, V or W of each factor), the
// first scaled by `scale`.
void kron3_coef(const Algo& a, char which, double scale, std::vector<double>* out) {
  for (int f = 0; f < 3; ++f)
    for (int t = 0; t < 4; ++t)
      for (int r = 0; r < 7; ++r) {
        const Algo& F = a.factors[(size_t)f];
        const double x = which == 'u' ? F.u(t, r) : which == 'v' ? F.v(t, r) : F.w(t, r);
        out->push_back(f == 0 ? x * scale : x);
      }
}

// Appends a set whose blocks are rows x cols.
void finish_set(CombineStage* st, CombSet set, int64_t rows, int64_t cols) {
  set.rows = (int32_t)rows;
  set.cols = (int32_t)cols;
  bool full = true;
  for (int k = 0; k < st->nin; ++k) {
    const CombIn& v = st->ins[(size_t)set.in_beg + k];
    full = full && v.vr == rows && v.vc == cols;
  }
  for (int o = set.out_beg; o < set.out_end; ++o) full = full && st->outs[o].vr == rows && st->outs[o].vc == cols;
  set.full = full ? 1 : 0;
  st->nout_max = std::max(st->nout_max, set.out_end - set.out_beg);
  st->elems_max = std::max(st->elems_max, rows * cols);
  st->sets.push_back(set);
}

// Granule of the leaf sizes of a stored-product plan (see kLeafStep).
int64_t leaf_granule(int dtype);

bool bf16_leaves(int dtype) {
  const int leaf = (dtype >> 8) & 0xff;
  return leaf == 2 || leaf == 3;
}

int64_t leaf_granule(int dtype) { return bf16_leaves(dtype) ? kLeafTile : kLeafStep; }

// Smallest M, N and K for which a classical product copies operands with
// unaligned rows: below it the copy's launch costs more than the masked K
// loop (FP64 n = 129: 0.035 ms without, 0.039 with the copy; n = 193: 0.048
// and 0.043; n = 1037: 0.215 and 0.142).
constexpr int64_t kAlignCopyMin = 192;

// BF16 leaves: reserve the staged operands (see Plan::bf_base) after
// everything else in the workspace, and list the outputs of every staging
// set: ops_a[z] / ops_b[z] are the leaf blocks of product z.
void finish_bf16(Plan* pl, const std::vector<Blk>& ops_a, const std::vector<Blk>& ops_b) {
  if (!bf16_leaves(pl->dtype)) return;
  const int leaf = (pl->dtype >> 8) & 0xff;
  pl->bf_planes = leaf == 3 ? 2 : 1;
  pl->bf_base = (int64_t)round_up((int64_t)pl->ws_bytes, 256);
  pl->ws_bytes = (size_t)pl->bf_base + (size_t)2 * pl->prods.size() * pl->bf_planes * pl->m * pl->m * 2;
  const int32_t np = (int32_t)pl->prods.size();
  std::vector<std::vector<StageOut>> per_set(pl->bf_sets.size());
  for (int32_t z = 0; z < np; ++z) {
    const Blk& a = ops_a[(size_t)z];
    const Blk& b = ops_b[(size_t)z];
    per_set[(size_t)a.stage_set].push_back({z, a.stage_coef});
    per_set[(size_t)b.stage_set].push_back({np + z, b.stage_coef});
  }
  pl->bf_outs.clear();
  for (size_t k = 0; k < per_set.size(); ++k) {
    pl->bf_sets[k].out_beg = (int32_t)pl->bf_outs.size();
    pl->bf_outs.insert(pl->bf_outs.end(), per_set[k].begin(), per_set[k].end());
    pl->bf_sets[k].out_end = (int32_t)pl->bf_outs.size();
  }
}

// BF16 leaves: a staging set over the p^2 quarters q of one block; returns
// its index.
int32_t add_stage_set(Plan* pl, int side, const std::vector<Blk>& q) {
  StageSet ss{};
  ss.in_beg = (int32_t)pl->bf_ins.size();
  ss.side = side;
  for (const Blk& b : q) pl->bf_ins.push_back(as_input(b));
  pl->bf_sets.push_back(ss);
  return (int32_t)pl->bf_sets.size() - 1;
}

mf_status build_classical(const Shape& sh, Plan* pl) {
  pl->P = pl->P_outer = 1;
  pl->R = pl->groups = 1;
  const int64_t g = leaf_granule(pl->dtype);
  pl->m = pl->m_outer = round_up(sh.M, g);
  pl->leaf_n = round_up(sh.N, g);
  pl->leaf_k = round_up(sh.K, g);
  pl->npad = pl->m;
  ProdDesc pd{};
  pd.a_src = SRC_A;
  pd.b_src = SRC_B;
  pd.lda = (int32_t)sh.lda;
  pd.ldb = (int32_t)sh.ldb;
  pd.a_vr = (int32_t)sh.M;
  pd.a_vc = pd.b_vr = (int32_t)sh.K;
  pd.b_vc = (int32_t)sh.N;
  pd.epi_beg = 0;
  pd.epi_end = 1;
  pl->prods.push_back(pd);
  EpiDesc ed{};
  ed.c_src = SRC_C;
  ed.ldc = (int32_t)sh.ldc;
  ed.c_vr = (int32_t)sh.M;
  ed.c_vc = (int32_t)sh.N;
  ed.first = 1;
  ed.coef = 1.0;
  pl->epis.push_back(ed);
  pl->group_beg = {0, 1};
  // Caller rows of A or B that are not 16-byte aligned keep every GEMM tile
  // on the masked K loop (the GEMM takes one alignment flag for both caller
  // operands).  Past a minimum size both operands are then copied once into
  // workspace blocks with rows of a multiple of 16 elements (a pre-addition
  // stage of one-term combinations, zeros past the views), and the product
  // reads the copies.  Blocks of a square product are square, the form
  // batched stages take.
  const bool unaligned = !sh.no_copy && (sh.copy_in || (sh.lda * (int64_t)pl->elem) % 16 != 0 ||
                                         (sh.ldb * (int64_t)pl->elem) % 16 != 0);
  if (!bf16_leaves(pl->dtype) && unaligned && std::min(sh.M, std::min(sh.N, sh.K)) >= kAlignCopyMin) {
    const bool cube = sh.M == sh.N && sh.N == sh.K;
    CombineStage st;
    st.nin = 1;
    int64_t ws = 0;
    for (int side = 0; side < 2; ++side) {
      const int64_t rows = side == 0 ? sh.M : sh.K, cols = side == 0 ? sh.K : sh.N;
      int64_t br = round_up(rows, kLeafStep), bc = round_up(cols, kLeafStep);
      if (cube) br = bc = std::max(br, bc);
      Blk v;
      v.src = side == 0 ? SRC_A : SRC_B;
      v.off = 0;
      v.ld = (int32_t)(side == 0 ? sh.lda : sh.ldb);
      v.vr = (int32_t)rows;
      v.vc = (int32_t)cols;
      v.zero = false;
      CombSet set{};
      set.in_beg = (int32_t)st.ins.size();
      set.out_beg = (int32_t)st.outs.size();
      st.ins.push_back(as_input(v));
      CombOut co{};
      co.off = ws;
      co.dst = SRC_WS;
      co.ld = (int32_t)bc;
      co.vr = (int32_t)br;
      co.vc = (int32_t)bc;
      co.coef_off = (int32_t)st.coef.size();
      st.coef.push_back(1.0);
      st.outs.push_back(co);
      set.out_end = (int32_t)st.outs.size();
      finish_set(&st, set, br, bc);
      ws += round_up(br * bc, 64);
      ProdDesc& q = pl->prods[0];
      // the copy holds zeros past the view, so its padded inner size (and
      // B's padded columns) are valid: whole K steps, and a moved edge tile
      // of B starts on an aligned column
      if (side == 0) {
        q.a_src = SRC_WS;
        q.a_off = co.off;
        q.lda = (int32_t)bc;
        q.a_vc = (int32_t)bc;
      } else {
        q.b_src = SRC_WS;
        q.b_off = co.off;
        q.ldb = (int32_t)bc;
        q.b_vr = (int32_t)br;
        q.b_vc = (int32_t)bc;
      }
    }
    st.m = cube ? st.sets[0].rows : 0;
    pl->pre.push_back(std::move(st));
    pl->ws_bytes = (size_t)ws * pl->elem;
  }
  if (bf16_leaves(pl->dtype)) {  // each operand is a set of one input (square plans only)
    const int64_t n = sh.M;
    Blk ops[2];
    pl->bf_nin = 1;
    for (int side = 0; side < 2; ++side) {
      Blk& b = ops[side];
      b.src = side == 0 ? SRC_A : SRC_B;
      b.ld = (int32_t)n;
      b.vr = b.vc = (int32_t)n;
      b.zero = false;
      b.stage_set = add_stage_set(pl, side, {b});
      b.stage_coef = (int32_t)pl->bf_coef.size();
      pl->bf_coef.push_back(1.0f);
    }
    finish_bf16(pl, {ops[0]}, {ops[1]});
  }
  return MF_OK;
}

// Fused-operand plan of one level of `al` (the schedule bit MF_SCHED_FUSED):
// no pre-addition stage and no workspace.  Product r's operands are the term
// lists of columns r of U and V over the blocks of A and B (the pre-addition
// is done in the GEMM's operand load), and its epilogue adds W[c, r] times
// the product into every block c of C it feeds; products run in index order
// within one group, so each workgroup owns one tile position of every C
// block and its read-modify-writes are ordered (the first product feeding a
// block stores).
mf_status build_fused(const Algo& al, const Shape& sh, Plan* pl) {
  const int m0 = al.m0, k0 = al.k0, n0 = al.n0, R = al.R;
  pl->levels = 1;
  pl->levels_outer = 0;
  pl->groups = 1;
  pl->P = m0;
  pl->P_outer = 1;
  pl->R = R;
  pl->m = round_up((sh.M + m0 - 1) / m0, kLeafTile);
  pl->leaf_n = round_up((sh.N + n0 - 1) / n0, kLeafTile);
  pl->leaf_k = round_up((sh.K + k0 - 1) / k0, kLeafTile);
  pl->npad = pl->m * m0;
  pl->m_outer = pl->m * m0;
  const int64_t m = pl->m, mn = pl->leaf_n, mk = pl->leaf_k;
  Blk top[2];
  for (int side = 0; side < 2; ++side) {
    top[side].src = side == 0 ? SRC_A : SRC_B;
    top[side].ld = (int32_t)(side == 0 ? sh.lda : sh.ldb);
    top[side].vr = (int32_t)(side == 0 ? sh.M : sh.K);
    top[side].vc = (int32_t)(side == 0 ? sh.K : sh.N);
    top[side].zero = false;
  }
  std::vector<Blk> qa(m0 * k0), qb(k0 * n0);
  for (int k = 0; k < m0 * k0; ++k) qa[k] = quarter(top[0], k, k0, m, mk);
  for (int k = 0; k < k0 * n0; ++k) qb[k] = quarter(top[1], k, n0, mk, mn);
  auto terms_of = [&](const std::vector<double>& X, const std::vector<Blk>& q, int r, int32_t* beg) {
    *beg = (int32_t)pl->terms.size();
    int n = 0;
    for (size_t k = 0; k < q.size(); ++k) {
      const double x = X[k * R + r];
      if (x == 0.0 || q[k].zero) continue;
      pl->terms.push_back(TermDesc{q[k].off, x, q[k].vr, q[k].vc});
      ++n;
    }
    return n;
  };
  const int nout = m0 * n0;
  std::vector<char> written(nout, 0);
  auto out_view = [&](int c, EpiDesc* ed) {
    const int64_t r0 = (int64_t)(c / n0) * m, c0 = (int64_t)(c % n0) * mn;
    ed->c_src = SRC_C;
    ed->ldc = (int32_t)sh.ldc;
    ed->c_vr = (int32_t)std::max<int64_t>(0, std::min<int64_t>(m, sh.M - r0));
    ed->c_vc = (int32_t)std::max<int64_t>(0, std::min<int64_t>(mn, sh.N - c0));
    if (ed->c_vr == 0 || ed->c_vc == 0) ed->c_vr = ed->c_vc = 0;
    ed->c_off = ed->c_vr > 0 ? r0 * sh.ldc + c0 : 0;
  };
  pl->group_beg.push_back(0);
  for (int r = 0; r < R; ++r) {
    ProdDesc pd{};
    const size_t terms_before = pl->terms.size();
    pd.a_terms = terms_of(al.U, qa, r, &pd.a_term0);
    pd.b_terms = terms_of(al.V, qb, r, &pd.b_term0);
    if (pd.a_terms == 0 || pd.b_terms == 0) {  // a zero product
      pl->terms.resize(terms_before);
      continue;
    }
    pl->fused_terms = std::max(pl->fused_terms, std::max(pd.a_terms, pd.b_terms));
    const TermDesc& ta = pl->terms[(size_t)pd.a_term0];
    const TermDesc& tb = pl->terms[(size_t)pd.b_term0];
    pd.a_src = SRC_A;
    pd.a_off = ta.off;
    pd.lda = (int32_t)sh.lda;
    pd.a_vr = ta.vr;
    pd.a_vc = ta.vc;
    pd.b_src = SRC_B;
    pd.b_off = tb.off;
    pd.ldb = (int32_t)sh.ldb;
    pd.b_vr = tb.vr;
    pd.b_vc = tb.vc;
    pd.epi_beg = (int32_t)pl->epis.size();
    for (int c = 0; c < nout; ++c) {
      const double w = al.w(c, r);
      if (w == 0.0) continue;
      EpiDesc ed{};
      out_view(c, &ed);
      if (ed.c_vr == 0) continue;
      ed.first = written[c] ? 0 : 1;
      ed.coef = w;
      written[c] = 1;
      pl->epis.push_back(ed);
    }
    pd.epi_end = (int32_t)pl->epis.size();
    pl->prods.push_back(pd);
  }
  if (pl->prods.empty()) return fail(MF_ERR_SHAPE, "plan has no products");
  // C blocks that no product feeds (only through padding) are zero: the first
  // product stores zeros there
  for (int c = 0; c < nout; ++c) {
    if (written[c]) continue;
    EpiDesc ed{};
    out_view(c, &ed);
    if (ed.c_vr == 0) continue;
    ed.first = 2;
    const int at = pl->prods[0].epi_end;
    pl->epis.insert(pl->epis.begin() + at, ed);
    pl->prods[0].epi_end += 1;
    for (size_t qd = 1; qd < pl->prods.size(); ++qd) {
      pl->prods[qd].epi_beg += 1;
      pl->prods[qd].epi_end += 1;
    }
  }
  pl->group_beg.push_back((int32_t)pl->prods.size());
  pl->ws_bytes = 0;
  return MF_OK;
}

// Whether linear-combination kernels exist for one level of an algorithm:
// m0 k0 inputs per A-side pre-addition set, k0 n0 per B-side set and R per
// post-addition set.
bool level_supported(const Algo& a) {
  return combine_supported(a.m0 * a.k0) && combine_supported(a.k0 * a.n0) && combine_supported(a.R);
}

// The algorithm of every recursion level, outermost first.  An algorithm
// runs as one level of its own when linear-combination kernels exist for its
// shape or when it is a three-factor composition of <2,2,2;7> algorithms
// (factor-by-factor kernels).  A Kronecker composition without such kernels
// (for example a 2 x 3 split, <6,6,6;189>) runs as its factors, one level
// each, outer factor first: the same algorithm (the composed coefficients are
// the factors' products), evaluated level by level.  One level of the
// algorithm is taken while levels remain, every dimension it splits exceeds
// the cutoff and the leaf tile, and the leaf count stays within the limit; a
// level taken is taken whole (all of its factors).  Returns false if some
// level has no kernel.
bool level_sequence(const Algo& a, int depth, int cutoff, const Shape& sh, std::vector<const Algo*>* seq) {
  seq->clear();
  std::vector<const Algo*> unit;
  const bool direct = is_kron3(a) || level_supported(a);
  if (direct || a.factors.empty()) {
    unit.push_back(&a);
  } else {
    for (const Algo& f : a.factors) unit.push_back(&f);
  }
  for (const Algo* f : unit)
    if (f != &a || !is_kron3(a))
      if (!level_supported(*f)) return false;
  const int L = levels_for(sh.M, sh.K, sh.N, a.m0, a.k0, a.n0, a.R, depth, cutoff);
  for (int d = 0; d < L; ++d) seq->insert(seq->end(), unit.begin(), unit.end());
  return true;
}

mf_status build(const Algo* algo, int depth, int cutoff, const Shape& sh, int dtype, int64_t min_wg, Plan* pl) {
  pl->shape = sh;
  pl->n = sh.M;
  pl->dtype = dtype;
  pl->elem = (dtype & 0xff) == MF_F64 ? 8 : 4;
  std::vector<const Algo*> seq;
  if (algo && !level_sequence(*algo, depth, cutoff, sh, &seq))
    return fail(MF_ERR_UNSUPPORTED, "no linear-combination kernel for this algorithm shape");
  const int L = (int)seq.size();
  pl->levels = L;
  bool sq_levels = true;
  for (const Algo* f : seq) sq_levels = sq_levels && f->square();
  pl->square = sh.square() && sq_levels;
  if (bf16_leaves(dtype) && !pl->square)
    return fail(MF_ERR_UNSUPPORTED, "BF16 leaves need square operands and a square algorithm");
  if (L == 0) return build_classical(sh, pl);
  if (dtype & MF_SCHED_FUSED) {
    if (bf16_leaves(dtype)) return fail(MF_ERR_UNSUPPORTED, "fused operands take leaves in the storage type");
    if (L != 1 || is_kron3(*seq[0]))
      return fail(MF_ERR_UNSUPPORTED,
                  "fused operands run one level of an algorithm with at most 16 terms per operand "
                  "(compose the algorithm for a deeper split)");
    const mf_status st = build_fused(*seq[0], sh, pl);
    if (st == MF_OK && pl->fused_terms > 16)
      return fail(MF_ERR_UNSUPPORTED, "fused operands take at most 16 terms per operand");
    return st;
  }

  const bool kron3 = is_kron3(*seq[0]);
  // Caller rows of A or B that are not 16-byte aligned keep every GEMM tile
  // reading a view of either caller operand on the masked path (the GEMM
  // takes one alignment flag for both); at the first level such views are
  // then copied into workspace blocks (one-term combinations) instead of
  // aliased, so that every leaf operand has aligned rows.
  const bool unaligned_in = !sh.no_copy && (sh.copy_in || (sh.lda * (int64_t)pl->elem) % 16 != 0 ||
                                            (sh.ldb * (int64_t)pl->elem) % 16 != 0);
  int64_t Pm = 1, Pk = 1, Pn = 1;
  for (const Algo* f : seq) {
    Pm *= f->m0;
    Pk *= f->k0;
    Pn *= f->n0;
  }
  pl->P = (int)Pm;
  if (bf16_leaves(dtype)) {
    const int p2_last = seq.back()->p * seq.back()->p;
    if (!stage_supported(p2_last)) return fail(MF_ERR_UNSUPPORTED, "no BF16 staging kernel for this algorithm shape");
    pl->bf_nin = p2_last;
  }
  // leaf sizes: rows, columns and inner size, each a multiple of the granule
  const int64_t lg = leaf_granule(dtype);
  pl->m = round_up((sh.M + Pm - 1) / Pm, lg);
  pl->leaf_n = round_up((sh.N + Pn - 1) / Pn, lg);
  pl->leaf_k = round_up((sh.K + Pk - 1) / Pk, lg);
  pl->npad = pl->m * Pm;
  const int64_t m = pl->m, mn = pl->leaf_n, mk = pl->leaf_k;
  const int64_t positions = ((m + kLeafTile - 1) / kLeafTile) * ((mn + kLeafTile - 1) / kLeafTile);

  // Outer levels split off as groups (with post-addition stages) until the
  // grouped GEMM has enough workgroups; the inner levels run as one composed
  // algorithm in the GEMM epilogue.
  int Lo = 0;
  int64_t outer_products = 1;
  while (Lo < L && positions * outer_products < min_wg) outer_products *= seq[(size_t)Lo++]->R;
  const int Li = L - Lo;
  pl->levels_outer = Lo;
  Algo Fi;
  if (Li > 0) {
    Fi = *seq[(size_t)L - 1];
    for (int l = L - 2; l >= Lo; --l) Fi = compose(*seq[(size_t)l], Fi);
  }
  // C grid of the levels fused into the epilogue
  const int Pim = Li > 0 ? Fi.m0 : 1, Pin = Li > 0 ? Fi.n0 : 1, Ri = Li > 0 ? Fi.R : 1;
  int64_t P_outer = 1, R_all = 1;
  for (int l = 0; l < Lo; ++l) P_outer *= seq[(size_t)l]->m0;
  for (const Algo* f : seq) R_all *= f->R;
  pl->P_outer = (int)P_outer;
  pl->R = (int)R_all;
  pl->groups = (int)outer_products;
  pl->m_outer = (int64_t)Pim * m;
  const int64_t mo_r = (int64_t)Pim * m, mo_c = (int64_t)Pin * mn;  // a group's output block
  int64_t ws = 0;  // workspace elements allocated so far
  auto alloc = [&](int64_t elems) {
    const int64_t off = ws;
    ws += round_up(elems, 64);
    return off;
  };

  // ---- pre-addition stages, level by level.  Side 0 splits A (rows M,
  // columns K) into m0 x k0 parts, side 1 splits B (K x N) into k0 x n0 parts;
  // both sides go into one launch when their sets have the same number of
  // inputs, else one launch each.  BF16 leaves fuse the last level into the
  // staging kernel: its linear combinations become term lists instead of
  // FP32 workspace blocks.
  std::vector<Blk> leaves[2];
  {
    std::vector<Blk> cur[2];
    for (int side = 0; side < 2; ++side) {
      Blk top;
      top.src = side == 0 ? SRC_A : SRC_B;
      top.off = 0;
      top.ld = (int32_t)(side == 0 ? sh.lda : sh.ldb);
      top.vr = (int32_t)(side == 0 ? sh.M : sh.K);
      top.vc = (int32_t)(side == 0 ? sh.K : sh.N);
      top.scale = 1.0;
      top.zero = false;
      cur[side] = {top};
    }
    // current block sizes of each side: rows, columns
    int64_t size[2][2] = {{m * Pm, mk * Pk}, {mk * Pk, mn * Pn}};
    for (int lev = 1; lev <= L; ++lev) {
      const Algo& al = *seq[(size_t)lev - 1];
      const int R = al.R;
      const int pr[2] = {al.m0, al.k0}, pc[2] = {al.k0, al.n0};
      const bool one_launch = pr[0] * pc[0] == pr[1] * pc[1];
      CombineStage stage[2];
      std::vector<Blk> next[2];
      for (int side = 0; side < 2; ++side) {
        CombineStage& st = stage[one_launch ? 0 : side];
        const int np = pr[side] * pc[side];
        const int64_t sr = size[side][0] / pr[side], sc = size[side][1] / pc[side];
        st.nin = np;
        st.m = sr == sc ? sr : 0;
        st.kron3 = kron3 ? 1 : 0;
        const std::vector<double>& X = side == 0 ? al.U : al.V;
        for (const Blk& b : cur[side]) {
          std::vector<Blk> q(np);
          for (int k = 0; k < np; ++k) q[k] = quarter(b, k, pc[side], sr, sc);
          if (lev == L && bf16_leaves(pl->dtype)) {
            // last level fused with the BF16 staging (square plans): every
            // nonzero child is an output of this block's staging set
            // (aliased ones included)
            const int64_t sz = sr;
            if (b.zero) {
              next[side].resize(next[side].size() + (size_t)R);
              continue;
            }
            const int32_t set_idx = add_stage_set(pl, side, q);
            for (int r = 0; r < R; ++r) {
              Blk child;
              const int32_t coef_off = (int32_t)pl->bf_coef.size();
              bool any = false;
              for (int k = 0; k < np; ++k) {
                const double x = q[k].zero ? 0.0 : X[(size_t)k * R + r] * b.scale;
                any = any || x != 0.0;
                pl->bf_coef.push_back((float)x);
              }
              if (!any) pl->bf_coef.resize((size_t)coef_off);
              if (any) {
                child.src = SRC_WS;
                child.off = 0;
                child.ld = (int32_t)sz;
                child.vr = child.vc = (int32_t)sz;
                child.scale = 1.0;
                child.zero = false;
                child.stage_set = set_idx;
                child.stage_coef = coef_off;
              }
              next[side].push_back(child);
            }
            continue;
          }
          CombSet set{};
          set.in_beg = (int32_t)st.ins.size();
          set.out_beg = (int32_t)st.outs.size();
          // kron3: every product has an output entry (empty unless stored) and
          // the set's coefficients are the factor matrices
          const int32_t kcoef = (int32_t)st.coef.size();
          if (kron3) kron3_coef(al, side == 0 ? 'u' : 'v', b.scale, &st.coef);
          bool stored = false;
          for (int r = 0; r < R; ++r) {
            int nnz = 0, last = -1;
            for (int k = 0; k < np; ++k)
              if (X[(size_t)k * R + r] != 0.0 && !q[k].zero) {
                ++nnz;
                last = k;
              }
            Blk child;
            if (nnz == 0) {
              child.zero = true;
            } else if (nnz == 1 && !(lev == 1 && unaligned_in)) {
              child = q[last];
              child.scale = b.scale * X[(size_t)last * R + r];
            } else {
              CombOut co{};
              co.off = alloc(sr * sc);
              co.dst = SRC_WS;
              co.ld = (int32_t)sc;
              co.vr = (int32_t)sr;
              co.vc = (int32_t)sc;
              if (kron3) {
                co.coef_off = kcoef;
              } else {
                co.coef_off = (int32_t)st.coef.size();
                for (int k = 0; k < np; ++k) st.coef.push_back(q[k].zero ? 0.0 : X[(size_t)k * R + r] * b.scale);
              }
              st.outs.push_back(co);
              stored = true;
              child.src = SRC_WS;
              child.off = co.off;
              child.ld = (int32_t)sc;
              child.vr = (int32_t)sr;
              child.vc = (int32_t)sc;
              child.scale = 1.0;
              child.zero = false;
            }
            if (kron3 && (int32_t)st.outs.size() == set.out_beg + r) {  // not stored: an empty entry
              CombOut co{};
              co.dst = SRC_WS;
              co.coef_off = kcoef;
              st.outs.push_back(co);
            }
            next[side].push_back(child);
          }
          set.out_end = (int32_t)st.outs.size();
          if (kron3 && stored) {
            // then the element offset in the workspace of each product's
            // operand (-1: not stored); every stored one is an sz x sz block
            for (int r = 0; r < R; ++r) {
              const CombOut& co = st.outs[(size_t)set.out_beg + r];
              st.coef.push_back(co.vr > 0 ? (double)co.off : -1.0);
            }
          }
          if (kron3 && !stored) {  // nothing to store: drop the set
            st.outs.resize((size_t)set.out_beg);
            st.coef.resize((size_t)kcoef);
          } else if (set.out_end > set.out_beg) {
            for (int k = 0; k < np; ++k) st.ins.push_back(as_input(q[kron3 ? kron3_block(k) : k]));
            finish_set(&st, set, sr, sc);
          }
        }
        size[side][0] = sr;
        size[side][1] = sc;
      }
      for (int k = 0; k < (one_launch ? 1 : 2); ++k)
        if (!stage[k].sets.empty()) pl->pre.push_back(std::move(stage[k]));
      cur[0].swap(next[0]);
      cur[1].swap(next[1]);
    }
    leaves[0].swap(cur[0]);
    leaves[1].swap(cur[1]);
  }

  // ---- group output buffers (sub-problem results of the outer levels)
  const int G = pl->groups;
  std::vector<int64_t> gbuf(G, 0);
  if (Lo > 0)
    for (int g = 0; g < G; ++g) gbuf[g] = alloc(mo_r * mo_c);

  // ---- grouped leaf products with the inner post-addition in the epilogue
  std::vector<char> group_empty(G, 1);
  std::vector<Blk> ops_a, ops_b;  // BF16 leaves: the leaf blocks in product order
  for (int g = 0; g < G; ++g) {
    pl->group_beg.push_back((int32_t)pl->prods.size());
    const int nout = Pim * Pin;
    std::vector<char> written(nout, 0);
    auto out_view = [&](int c, EpiDesc* ed) {
      const int64_t r0 = (int64_t)(c / Pin) * m, c0 = (int64_t)(c % Pin) * mn;
      if (Lo == 0) {
        ed->c_src = SRC_C;
        ed->ldc = (int32_t)sh.ldc;
        ed->c_vr = (int32_t)std::max<int64_t>(0, std::min<int64_t>(m, sh.M - r0));
        ed->c_vc = (int32_t)std::max<int64_t>(0, std::min<int64_t>(mn, sh.N - c0));
        if (ed->c_vr == 0 || ed->c_vc == 0) ed->c_vr = ed->c_vc = 0;
        ed->c_off = ed->c_vr > 0 ? r0 * sh.ldc + c0 : 0;
      } else {
        ed->c_src = SRC_WS;
        ed->ldc = (int32_t)mo_c;
        ed->c_vr = (int32_t)m;
        ed->c_vc = (int32_t)mn;
        ed->c_off = gbuf[g] + r0 * mo_c + c0;
      }
    };
    const int group_first = (int)pl->prods.size();
    for (int ri = 0; ri < Ri; ++ri) {
      const int r = g * Ri + ri;
      const Blk& a = leaves[0][r];
      const Blk& b = leaves[1][r];
      if (a.zero || b.zero) continue;
      ProdDesc pd{};
      pd.a_src = a.src;
      pd.a_off = a.off;
      pd.lda = a.ld;
      pd.a_vr = a.vr;
      pd.a_vc = a.vc;
      pd.b_src = b.src;
      pd.b_off = b.off;
      pd.ldb = b.ld;
      pd.b_vr = b.vr;
      pd.b_vc = b.vc;
      const double scale = a.scale * b.scale;
      pd.epi_beg = (int32_t)pl->epis.size();
      for (int c = 0; c < nout; ++c) {
        const double w = Li > 0 ? Fi.w(c, ri) : 1.0;
        if (w == 0.0) continue;
        EpiDesc ed{};
        out_view(c, &ed);
        if (ed.c_vr == 0) continue;
        ed.first = written[c] ? 0 : 1;
        ed.coef = w * scale;
        written[c] = 1;
        pl->epis.push_back(ed);
      }
      pd.epi_end = (int32_t)pl->epis.size();
      pl->prods.push_back(pd);
      if (bf16_leaves(pl->dtype)) {
        ops_a.push_back(a);
        ops_b.push_back(b);
      }
      group_empty[g] = 0;
    }
    // Output blocks that no product of the group feeds are zero; the first
    // product of the group stores zeros there.  (An empty group is read as
    // zero by the post-addition instead.)
    for (int c = 0; c < nout && !group_empty[g]; ++c) {
      if (written[c]) continue;
      EpiDesc ed{};
      out_view(c, &ed);
      if (ed.c_vr == 0) continue;
      ed.first = 2;
      ed.coef = 0.0;
      const int at = pl->prods[group_first].epi_end;
      pl->epis.insert(pl->epis.begin() + at, ed);
      pl->prods[group_first].epi_end += 1;
      for (size_t qd = group_first + 1; qd < pl->prods.size(); ++qd) {
        pl->prods[qd].epi_beg += 1;
        pl->prods[qd].epi_end += 1;
      }
      written[c] = 1;
    }
  }
  pl->group_beg.push_back((int32_t)pl->prods.size());
  if (pl->prods.empty()) return fail(MF_ERR_SHAPE, "plan has no products");

  // ---- post-addition stages, innermost outer level first:
  // parent_c = sum_r W[c, r] child_r for each of the m0 x n0 blocks c of a
  // parent.
  if (Lo > 0) {
    std::vector<Blk> child(G);
    for (int g = 0; g < G; ++g) {
      child[g].src = SRC_WS;
      child[g].off = gbuf[g];
      child[g].ld = (int32_t)mo_c;
      child[g].vr = (int32_t)mo_r;
      child[g].vc = (int32_t)mo_c;
      child[g].zero = group_empty[g] != 0;
    }
    int64_t cr = mo_r, cc = mo_c;  // size of a child result
    for (int lev = Lo; lev >= 1; --lev) {
      const Algo& al = *seq[(size_t)lev - 1];
      const int R = al.R, pm = al.m0, pn = al.n0;
      int nparent = 1;
      for (int l = 0; l < lev - 1; ++l) nparent *= seq[(size_t)l]->R;
      const int64_t pr = cr * pm, pcol = cc * pn;
      CombineStage st;
      st.nin = R;
      st.m = cr == cc ? cr : 0;
      st.kron3 = kron3 ? 1 : 0;
      st.kpost = 1;
      std::vector<Blk> parents(nparent);
      for (int q = 0; q < nparent; ++q) {
        Blk par;
        if (lev == 1) {
          par.src = SRC_C;
          par.off = 0;
          par.ld = (int32_t)sh.ldc;
          par.vr = (int32_t)sh.M;
          par.vc = (int32_t)sh.N;
          par.zero = false;
        } else {
          par.src = SRC_WS;
          par.off = alloc(pr * pcol);
          par.ld = (int32_t)pcol;
          par.vr = (int32_t)pr;
          par.vc = (int32_t)pcol;
          par.zero = false;
        }
        parents[q] = par;
        CombSet set{};
        set.in_beg = (int32_t)st.ins.size();
        for (int r = 0; r < R; ++r) st.ins.push_back(as_input(child[(size_t)q * R + r]));
        set.out_beg = (int32_t)st.outs.size();
        const int32_t kcoef = (int32_t)st.coef.size();
        if (kron3) {
          // the factor matrices, then the element offset in the workspace of
          // each product (-1: an empty group, read as zero); every product is
          // a csz x csz block
          kron3_coef(al, 'w', 1.0, &st.coef);
          for (int r = 0; r < R; ++r) {
            const Blk& cb = child[(size_t)q * R + r];
            if (!cb.zero && (cb.src != SRC_WS || cb.ld != cc || cb.vr != cr || cb.vc != cc))
              return fail(MF_ERR_UNSUPPORTED, "Kronecker post-addition needs whole workspace blocks");
            st.coef.push_back(cb.zero ? -1.0 : (double)cb.off);
          }
        }
        for (int t = 0; t < pm * pn; ++t) {
          const int c = kron3 ? kron3_block(t) : t;
          const Blk qb = quarter(par, c, pn, cr, cc);
          CombOut co{};
          if (qb.zero) {
            if (!kron3) continue;
            co.dst = SRC_WS;  // kron3: an entry with an empty extent
            co.coef_off = kcoef;
            st.outs.push_back(co);
            continue;
          }
          co.off = qb.off;
          co.dst = qb.src;
          co.ld = qb.ld;
          co.vr = qb.vr;
          co.vc = qb.vc;
          if (kron3) {
            co.coef_off = kcoef;
          } else {
            co.coef_off = (int32_t)st.coef.size();
            for (int r = 0; r < R; ++r) st.coef.push_back(al.w(c, r));
          }
          st.outs.push_back(co);
        }
        set.out_end = (int32_t)st.outs.size();
        finish_set(&st, set, cr, cc);
      }
      pl->post.push_back(std::move(st));
      child.swap(parents);
      cr = pr;
      cc = pcol;
    }
  }
  pl->ws_bytes = (size_t)ws * pl->elem;
  finish_bf16(pl, ops_a, ops_b);
  return MF_OK;
}

template <class T>
size_t bytes_of(const std::vector<T>& v) {
  return v.size() * sizeof(T);
}

// Lays out every descriptor array of the plan in one image, each at a
// 256-byte aligned offset (an empty array still takes one aligned slot).
void make_image(Plan* pl) {
  auto align = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t total = 0;
  std::vector<std::pair<const void*, size_t>> parts;
  auto place = [&](const void* src, size_t bytes, size_t* off) {
    *off = total;
    parts.push_back({src, bytes});
    total += align(std::max<size_t>(bytes, 1));
  };
  place(pl->prods.data(), bytes_of(pl->prods), &pl->img_prods);
  place(pl->epis.data(), bytes_of(pl->epis), &pl->img_epis);
  place(pl->group_beg.data(), bytes_of(pl->group_beg), &pl->img_group_beg);
  place(pl->terms.data(), bytes_of(pl->terms), &pl->img_terms);
  place(pl->bf_sets.data(), bytes_of(pl->bf_sets), &pl->img_bf_sets);
  place(pl->bf_ins.data(), bytes_of(pl->bf_ins), &pl->img_bf_ins);
  place(pl->bf_outs.data(), bytes_of(pl->bf_outs), &pl->img_bf_outs);
  place(pl->bf_coef.data(), bytes_of(pl->bf_coef), &pl->img_bf_coef);
  for (std::vector<CombineStage>* list : {&pl->pre, &pl->post})
    for (CombineStage& st : *list) {
      place(st.sets.data(), bytes_of(st.sets), &st.img_sets);
      place(st.ins.data(), bytes_of(st.ins), &st.img_ins);
      place(st.outs.data(), bytes_of(st.outs), &st.img_outs);
      place(st.coef.data(), bytes_of(st.coef), &st.img_coef);
    }
  pl->image.assign(total, 0);
  size_t off = 0;
  for (const auto& q : parts) {
    if (q.second) memcpy(pl->image.data() + off, q.first, q.second);
    off += align(std::max<size_t>(q.second, 1));
  }
}

mf_status upload(const Plan* pl) {
  if (hipMalloc(&pl->dev, pl->image.size()) != hipSuccess) {
    (void)hipGetLastError();
    pl->dev = nullptr;
    return MF_ERR_NOMEM;
  }
  if (hipMemcpy(pl->dev, pl->image.data(), pl->image.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return MF_ERR_HIP;
  }
  return MF_OK;
}

// A plan's descriptors live on the device that was current when it was
// first run, so the device is part of the key (-1 where none is visible:
// host-only queries).
struct Key {
  uint64_t algo;
  int levels, dtype, device;
  int64_t M, N, K, lda, ldb, ldc, min_wg;
  bool no_copy, copy_in;
  bool operator<(const Key& o) const {
    return std::tie(algo, levels, dtype, device, M, N, K, lda, ldb, ldc, min_wg, no_copy, copy_in) <
           std::tie(o.algo, o.levels, o.dtype, o.device, o.M, o.N, o.K, o.lda, o.ldb, o.ldc, o.min_wg, o.no_copy,
                    o.copy_in);
  }
};

int current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    dev = -1;
  }
  return dev;
}

// Heap-allocated and never destroyed: plans may hold device memory, which must
// not be released from static destructors after the HIP runtime is gone.
std::mutex g_mu;
std::map<Key, std::shared_ptr<const Plan>>& cache() {
  static auto* c = new std::map<Key, std::shared_ptr<const Plan>>();
  return *c;
}

}  // namespace

// Levels taken for a product: a level is taken while levels remain, every
// dimension the algorithm splits exceeds the cutoff and the leaf tile
// (smaller leaves only add padding on this GEMM), and the leaf count stays
// within the limit (sizes rounded up at each split).
int levels_for(int64_t M, int64_t K, int64_t N, int m0, int k0, int n0, int R, int depth, int cutoff) {
  int d = 0;
  int64_t size[3] = {M, K, N};
  const int split[3] = {m0, k0, n0};
  if (m0 < 1 || k0 < 1 || n0 < 1 || (m0 == 1 && k0 == 1 && n0 == 1)) return 0;
  int64_t leaves = 1;
  auto fits = [&]() {
    for (int x = 0; x < 3; ++x)
      if (split[x] > 1 && (size[x] <= cutoff || size[x] <= kLeafTile)) return false;
    return true;
  };
  while (d < depth && fits() && leaves * R <= kMaxLeafProducts) {
    for (int x = 0; x < 3; ++x) size[x] = (size[x] + split[x] - 1) / split[x];
    leaves *= R;
    ++d;
  }
  return d;
}

mf_status get_plan(const mf_algo* algo, int depth, int cutoff, const Shape& sh, int dtype, int64_t min_wg,
                   std::shared_ptr<const Plan>* out) {
  const int levels =
      algo ? levels_for(sh.M, sh.K, sh.N, algo->a.m0, algo->a.k0, algo->a.n0, algo->a.R, depth, cutoff) : 0;
  const Key key{levels == 0 ? 0 : algo->id, levels, dtype, current_device(), sh.M, sh.N, sh.K, sh.lda, sh.ldb,
                sh.ldc, levels == 0 ? 0 : min_wg, sh.no_copy, sh.copy_in};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = cache().find(key);
    if (it != cache().end()) {
      *out = it->second;
      return MF_OK;
    }
  }
  auto pl = std::make_shared<Plan>();
  const mf_status st = build(levels == 0 ? nullptr : &algo->a, depth, cutoff, sh, dtype, min_wg, pl.get());
  if (st != MF_OK) return st;
  make_image(pl.get());
  std::lock_guard<std::mutex> lk(g_mu);
  auto ins = cache().emplace(key, pl);
  *out = ins.first->second;
  return MF_OK;
}

mf_status ensure_device(const Plan& pl) {
  std::call_once(pl.uploaded, [&]() { pl.upload_status = upload(&pl); });
  if (pl.upload_status != MF_OK) return fail(pl.upload_status, "plan descriptors could not be copied to the device");
  return MF_OK;
}

void drop_plans(uint64_t algo_id) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto it = cache().begin(); it != cache().end();) {
    if (it->first.algo == algo_id)
      it = cache().erase(it);
    else
      ++it;
  }
}

}  // namespace mf
