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

#include "mf_internal.h"

namespace mf {

Plan::~Plan() {
  if (dev) (void)hipFree(dev);
}

namespace {

// Levels taken for an n x n product: a level is taken while levels remain and
// the current size exceeds the cutoff (sizes rounded up at each split).
int levels_for(int64_t n, int p, int depth, int cutoff) {
  int d = 0;
  int64_t size = n;
  while (d < depth && size > cutoff && p > 1) {
    size = (size + p - 1) / p;
    ++d;
  }
  return d;
}

int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }
int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  while (e-- > 0) r *= b;
  return r;
}

struct View {
  int64_t off;
  int32_t vr, vc;
};

// Block k of the P x P partition of an n x n matrix with block size m (the
// padded size P*m >= n), clipped to the true size: entries beyond it are
// virtual zeros.  ld of the view is n.
View block_view(int k, int P, int64_t m, int64_t n) {
  const int64_t bi = k / P, bj = k % P;
  View v;
  const int64_t r0 = bi * m, c0 = bj * m;
  v.vr = (int32_t)std::max<int64_t>(0, std::min<int64_t>(m, n - r0));
  v.vc = (int32_t)std::max<int64_t>(0, std::min<int64_t>(m, n - c0));
  if (v.vr == 0 || v.vc == 0) v.vr = v.vc = 0;
  v.off = (v.vr > 0) ? r0 * n + c0 : 0;
  return v;
}

// Marks the operand sets of a stage whose views all cover a full m x m block
// (no virtual padding), which run on the kernel's branch-free path.
void set_full(CombineStage* cs, int64_t m) {
  for (int y = 0; y < cs->n_sets; ++y) {
    bool full = true;
    for (int k = 0; k < cs->nin; ++k) {
      const CombIn& v = cs->ins[(size_t)y * cs->nin + k];
      full = full && v.vr == m && v.vc == m;
    }
    for (int o = cs->out_beg[y]; o < cs->out_beg[y + 1]; ++o) full = full && cs->outs[o].vr == m && cs->outs[o].vc == m;
    cs->full[y] = full ? 1 : 0;
  }
}

// Workgroups wanted in the grouped GEMM before outer levels are split off.
constexpr int64_t kMinWorkgroups = 1024;

mf_status build_classical(int64_t n, Plan* pl) {
  pl->P = pl->P_outer = 1;
  pl->R = pl->groups = 1;
  pl->m = pl->m_outer = round_up(n, kLeafTile);
  pl->npad = pl->m;
  ProdDesc pd{};
  pd.a_src = SRC_A;
  pd.b_src = SRC_B;
  pd.lda = pd.ldb = (int32_t)n;
  pd.a_vr = pd.a_vc = pd.b_vr = pd.b_vc = (int32_t)n;
  pd.epi_beg = 0;
  pd.epi_end = 1;
  pl->prods.push_back(pd);
  EpiDesc ed{};
  ed.c_src = SRC_C;
  ed.ldc = (int32_t)n;
  ed.c_vr = ed.c_vc = (int32_t)n;
  ed.first = 1;
  ed.coef = 1.0;
  pl->epis.push_back(ed);
  pl->group_beg = {0, 1};
  return MF_OK;
}

mf_status build(const Algo* algo, int depth, int cutoff, int64_t n, int dtype, Plan* pl) {
  pl->n = n;
  pl->dtype = dtype;
  pl->elem = (dtype & 0xff) == MF_F64 ? 8 : 4;
  const int L = algo ? levels_for(n, algo->p, depth, cutoff) : 0;
  pl->levels = L;
  if (L == 0) return build_classical(n, pl);

  const int p = algo->p;
  const int64_t P = ipow(p, L);
  const int64_t P2 = P * P;
  if (!combine_supported((int)P2))
    return fail(MF_ERR_UNSUPPORTED, "fused split factor " + std::to_string(P) + " has no pre-addition kernel");
  pl->P = (int)P;
  pl->m = round_up((n + P - 1) / P, kLeafTile);
  pl->npad = pl->m * P;
  const int64_t m = pl->m, mm = m * m;
  const int64_t positions = (m / kLeafTile) * (m / kLeafTile);

  // Outer levels split off as groups until the grid is large enough.
  int Lo = 0;
  while (Lo < L && Lo < 2 && positions * ipow(algo->R, Lo) < kMinWorkgroups &&
         combine_supported((int)ipow(algo->R, Lo + 1)))
    ++Lo;
  const int Li = L - Lo;
  pl->levels_outer = Lo;
  const Algo Fo = Lo > 0 ? power(*algo, Lo) : Algo{};
  const Algo Fi = Li > 0 ? power(*algo, Li) : Algo{};
  const Algo F = power(*algo, L);
  const int Po = Lo > 0 ? Fo.p : 1, Ro = Lo > 0 ? Fo.R : 1;
  const int Pi = Li > 0 ? Fi.p : 1, Ri = Li > 0 ? Fi.R : 1;
  pl->P_outer = Po;
  pl->R = F.R;
  pl->groups = Ro;
  pl->m_outer = (int64_t)Pi * m;
  const int64_t mo = pl->m_outer;

  // ---- pre-addition stage: inputs are the P^2 blocks of A (set 0) and B (set 1)
  std::vector<View> views(P2);
  for (int k = 0; k < P2; ++k) views[k] = block_view(k, (int)P, m, n);
  CombineStage& pre = pl->pre;
  pre.nin = (int)P2;
  for (int side = 0; side < 2; ++side)
    for (int k = 0; k < P2; ++k)
      pre.ins.push_back(CombIn{views[k].off, side == 0 ? SRC_A : SRC_B, (int32_t)n, views[k].vr, views[k].vc});

  struct Operand {
    bool zero = false, view = false;
    int block = -1, slot = -1;
    double scale = 1.0;
  };
  auto classify = [&](const std::vector<double>& X, int r) {
    Operand o;
    int nnz = 0, last = -1;
    for (int k = 0; k < P2; ++k)
      if (X[(size_t)k * F.R + r] != 0.0 && views[k].vr > 0) {
        ++nnz;
        last = k;
      }
    if (nnz == 0) {
      o.zero = true;
    } else if (nnz == 1) {
      o.view = true;
      o.block = last;
      o.scale = X[(size_t)last * F.R + r];
    }
    return o;
  };
  std::vector<Operand> opa(F.R), opb(F.R);
  for (int r = 0; r < F.R; ++r) {
    opa[r] = classify(F.U, r);
    opb[r] = classify(F.V, r);
  }
  // A product with an all-zero operand (only possible through padding)
  // contributes nothing; it and its pre-additions are skipped.
  int slots = 0;
  for (int side = 0; side < 2; ++side) {
    const std::vector<double>& X = side == 0 ? F.U : F.V;
    std::vector<Operand>& ops = side == 0 ? opa : opb;
    pre.out_beg[side] = (int)pre.outs.size();
    for (int r = 0; r < F.R; ++r) {
      if (opa[r].zero || opb[r].zero || ops[r].view) continue;
      ops[r].slot = slots++;
      CombOut co{};
      co.off = (int64_t)ops[r].slot * mm;
      co.dst = SRC_WS;
      co.ld = (int32_t)m;
      co.vr = co.vc = (int32_t)m;
      co.coef_off = (int32_t)pre.coef.size();
      for (int k = 0; k < P2; ++k) pre.coef.push_back(views[k].vr > 0 ? X[(size_t)k * F.R + r] : 0.0);
      pre.outs.push_back(co);
    }
  }
  pre.out_beg[2] = (int)pre.outs.size();
  pre.n_sets = pre.outs.empty() ? 0 : 2;
  set_full(&pre, m);
  const int64_t pbuf_base = (int64_t)slots * mm;  // group output buffers follow the T/S slots

  // ---- grouped leaf products with epilogue post-addition
  for (int g = 0; g < Ro; ++g) {
    pl->group_beg.push_back((int32_t)pl->prods.size());
    const int nout = Pi * Pi;  // output blocks of the group
    std::vector<char> written(nout, 0);
    // Output block c (inner index) of this group.
    auto out_view = [&](int c, EpiDesc* ed) {
      if (Lo == 0) {
        const View v = block_view(c, (int)P, m, n);
        ed->c_src = SRC_C;
        ed->c_off = v.off;
        ed->ldc = (int32_t)n;
        ed->c_vr = v.vr;
        ed->c_vc = v.vc;
      } else {
        ed->c_src = SRC_WS;
        ed->c_off = pbuf_base + (int64_t)g * mo * mo + (int64_t)(c / Pi) * m * mo + (int64_t)(c % Pi) * m;
        ed->ldc = (int32_t)mo;
        ed->c_vr = ed->c_vc = (int32_t)m;
      }
    };
    const int group_first = (int)pl->prods.size();
    for (int ri = 0; ri < Ri; ++ri) {
      const int r = g * Ri + ri;
      if (opa[r].zero || opb[r].zero) continue;
      ProdDesc pd{};
      const Operand& a = opa[r];
      const Operand& b = opb[r];
      if (a.view) {
        pd.a_src = SRC_A;
        pd.a_off = views[a.block].off;
        pd.lda = (int32_t)n;
        pd.a_vr = views[a.block].vr;
        pd.a_vc = views[a.block].vc;
      } else {
        pd.a_src = SRC_WS;
        pd.a_off = (int64_t)a.slot * mm;
        pd.lda = (int32_t)m;
        pd.a_vr = pd.a_vc = (int32_t)m;
      }
      if (b.view) {
        pd.b_src = SRC_B;
        pd.b_off = views[b.block].off;
        pd.ldb = (int32_t)n;
        pd.b_vr = views[b.block].vr;
        pd.b_vc = views[b.block].vc;
      } else {
        pd.b_src = SRC_WS;
        pd.b_off = (int64_t)b.slot * mm;
        pd.ldb = (int32_t)m;
        pd.b_vr = pd.b_vc = (int32_t)m;
      }
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
    }
    // Output blocks that no product of the group feeds are zero; the first
    // product of the group stores zeros there.
    for (int c = 0; c < nout; ++c) {
      if (written[c]) continue;
      EpiDesc ed{};
      out_view(c, &ed);
      if (ed.c_vr == 0) continue;
      if ((int)pl->prods.size() == group_first) break;  // empty group: the post stage reads it as zero
      ed.first = 2;
      ed.coef = 0.0;
      const int at = pl->prods[group_first].epi_end;
      pl->epis.insert(pl->epis.begin() + at, ed);
      pl->prods[group_first].epi_end += 1;
      for (size_t q = group_first + 1; q < pl->prods.size(); ++q) {
        pl->prods[q].epi_beg += 1;
        pl->prods[q].epi_end += 1;
      }
      written[c] = 1;
    }
  }
  pl->group_beg.push_back((int32_t)pl->prods.size());
  if (pl->prods.empty()) return fail(MF_ERR_SHAPE, "plan has no products");

  // ---- outer post-addition: C_c = sum_g W_outer[c, g] P_g
  size_t ws_elems = (size_t)pbuf_base;
  if (Lo > 0) {
    CombineStage& post = pl->post;
    post.nin = Ro;
    for (int g = 0; g < Ro; ++g) {
      const bool empty = pl->group_beg[g] == pl->group_beg[g + 1];
      post.ins.push_back(CombIn{pbuf_base + (int64_t)g * mo * mo, SRC_WS, (int32_t)mo, empty ? 0 : (int32_t)mo,
                                empty ? 0 : (int32_t)mo});
    }
    post.out_beg[0] = 0;
    for (int c = 0; c < Po * Po; ++c) {
      const View v = block_view(c, Po, mo, n);
      if (v.vr == 0) continue;
      CombOut co{};
      co.off = v.off;
      co.dst = SRC_C;
      co.ld = (int32_t)n;
      co.vr = v.vr;
      co.vc = v.vc;
      co.coef_off = (int32_t)post.coef.size();
      for (int g = 0; g < Ro; ++g) post.coef.push_back(Fo.w(c, g));
      post.outs.push_back(co);
    }
    post.out_beg[1] = post.out_beg[2] = (int)post.outs.size();
    post.n_sets = 1;
    set_full(&post, mo);
    ws_elems += (size_t)Ro * (size_t)mo * (size_t)mo;
  }
  pl->ws_bytes = ws_elems * pl->elem;
  return MF_OK;
}

template <class T>
size_t bytes_of(const std::vector<T>& v) {
  return v.size() * sizeof(T);
}

mf_status upload(const Plan* pl) {
  auto align = [](size_t x) { return (x + 255) / 256 * 256; };
  struct Part {
    const void* src;
    size_t bytes;
    size_t off;
  };
  std::vector<Part> parts = {
      {pl->prods.data(), bytes_of(pl->prods), 0},         {pl->epis.data(), bytes_of(pl->epis), 0},
      {pl->group_beg.data(), bytes_of(pl->group_beg), 0}, {pl->pre.ins.data(), bytes_of(pl->pre.ins), 0},
      {pl->pre.outs.data(), bytes_of(pl->pre.outs), 0},   {pl->pre.coef.data(), bytes_of(pl->pre.coef), 0},
      {pl->post.ins.data(), bytes_of(pl->post.ins), 0},   {pl->post.outs.data(), bytes_of(pl->post.outs), 0},
      {pl->post.coef.data(), bytes_of(pl->post.coef), 0},
  };
  size_t total = 0;
  for (auto& q : parts) {
    q.off = total;
    total += align(q.bytes);
  }
  if (total == 0) return MF_OK;
  std::vector<char> host(total, 0);
  for (auto& q : parts)
    if (q.bytes) memcpy(host.data() + q.off, q.src, q.bytes);
  if (hipMalloc(&pl->dev, total) != hipSuccess) {
    (void)hipGetLastError();
    pl->dev = nullptr;
    return MF_ERR_NOMEM;
  }
  if (hipMemcpy(pl->dev, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return MF_ERR_HIP;
  }
  char* d = static_cast<char*>(pl->dev);
  pl->d_prods = reinterpret_cast<ProdDesc*>(d + parts[0].off);
  pl->d_epis = reinterpret_cast<EpiDesc*>(d + parts[1].off);
  pl->d_group_beg = reinterpret_cast<int32_t*>(d + parts[2].off);
  pl->pre.d_ins = reinterpret_cast<CombIn*>(d + parts[3].off);
  pl->pre.d_outs = reinterpret_cast<CombOut*>(d + parts[4].off);
  pl->pre.d_coef = reinterpret_cast<double*>(d + parts[5].off);
  pl->post.d_ins = reinterpret_cast<CombIn*>(d + parts[6].off);
  pl->post.d_outs = reinterpret_cast<CombOut*>(d + parts[7].off);
  pl->post.d_coef = reinterpret_cast<double*>(d + parts[8].off);
  return MF_OK;
}

struct Key {
  uint64_t algo;
  int levels, dtype;
  int64_t n;
  bool operator<(const Key& o) const {
    return std::tie(algo, levels, dtype, n) < std::tie(o.algo, o.levels, o.dtype, o.n);
  }
};

// Heap-allocated and never destroyed: plans may hold device memory, which must
// not be released from static destructors after the HIP runtime is gone.
std::mutex g_mu;
std::map<Key, std::shared_ptr<const Plan>>& cache() {
  static auto* c = new std::map<Key, std::shared_ptr<const Plan>>();
  return *c;
}

}  // namespace

mf_status get_plan(const mf_algo* algo, int depth, int cutoff, int64_t n, int dtype,
                   std::shared_ptr<const Plan>* out) {
  const int levels = algo ? levels_for(n, algo->a.p, depth, cutoff) : 0;
  const Key key{levels == 0 ? 0 : algo->id, levels, dtype, n};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = cache().find(key);
    if (it != cache().end()) {
      *out = it->second;
      return MF_OK;
    }
  }
  auto pl = std::make_shared<Plan>();
  const mf_status st = build(levels == 0 ? nullptr : &algo->a, depth, cutoff, n, dtype, pl.get());
  if (st != MF_OK) return st;
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
