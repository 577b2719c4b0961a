// Planner: turns (algorithm, depth, cutoff, n, dtype) into the descriptors of
// one fused level - the pre-addition outputs, the leaf products and the
// post-addition terms - plus the workspace size.  Plans are immutable and
// cached; their descriptors live in one device allocation.
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

struct View {
  int64_t off;
  int32_t vr, vc;
};

// Block k of the P x P partition of the padded n x n input (block size m),
// clipped to the true size n: entries beyond it are virtual zeros.
View block_view(int k, int P, int64_t m, int64_t n) {
  const int64_t bi = k / P, bj = k % P;
  View v;
  const int64_t r0 = bi * m, c0 = bj * m;
  v.vr = (int32_t)std::max<int64_t>(0, std::min<int64_t>(m, n - r0));
  v.vc = (int32_t)std::max<int64_t>(0, std::min<int64_t>(m, n - c0));
  v.off = (v.vr > 0 && v.vc > 0) ? r0 * n + c0 : 0;
  if (v.vr == 0 || v.vc == 0) v.vr = v.vc = 0;
  return v;
}

mf_status upload(const Plan* pl) {
  auto align = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t sp = align(pl->prods.size() * sizeof(ProdDesc));
  const size_t se = align(pl->epis.size() * sizeof(EpiDesc));
  const size_t so = align(pl->pre_out.size() * sizeof(PreOut));
  const size_t si = align(pl->pre_in.size() * sizeof(PreIn));
  const size_t sc = align(pl->pre_coef.size() * sizeof(double));
  const size_t total = sp + se + so + si + sc;
  if (total == 0) return MF_OK;
  std::vector<char> host(total, 0);
  char* h = host.data();
  memcpy(h, pl->prods.data(), pl->prods.size() * sizeof(ProdDesc));
  memcpy(h + sp, pl->epis.data(), pl->epis.size() * sizeof(EpiDesc));
  memcpy(h + sp + se, pl->pre_out.data(), pl->pre_out.size() * sizeof(PreOut));
  memcpy(h + sp + se + so, pl->pre_in.data(), pl->pre_in.size() * sizeof(PreIn));
  memcpy(h + sp + se + so + si, pl->pre_coef.data(), pl->pre_coef.size() * sizeof(double));
  if (hipMalloc(&pl->dev, total) != hipSuccess) {
    pl->dev = nullptr;
    return fail(MF_ERR_NOMEM, "hipMalloc of plan descriptors failed");
  }
  if (hipMemcpy(pl->dev, host.data(), total, hipMemcpyHostToDevice) != hipSuccess)
    return fail(MF_ERR_HIP, "copy of plan descriptors failed");
  char* d = static_cast<char*>(pl->dev);
  pl->d_prods = reinterpret_cast<ProdDesc*>(d);
  pl->d_epis = reinterpret_cast<EpiDesc*>(d + sp);
  pl->d_pre_out = reinterpret_cast<PreOut*>(d + sp + se);
  pl->d_pre_in = reinterpret_cast<PreIn*>(d + sp + se + so);
  pl->d_pre_coef = reinterpret_cast<double*>(d + sp + se + so + si);
  return MF_OK;
}

mf_status build(const Algo* algo, int depth, int cutoff, int64_t n, int dtype, Plan* pl) {
  pl->n = n;
  pl->dtype = dtype;
  pl->elem = (dtype & 0xff) == MF_F64 ? 8 : 4;
  const int levels = algo ? levels_for(n, algo->p, depth, cutoff) : 0;
  pl->levels = levels;

  if (levels == 0) {
    // Classical product: one leaf of size round_up(n, tile) with virtual padding.
    pl->P = 1;
    pl->R = 1;
    pl->m = round_up(n, kLeafTile);
    pl->npad = pl->m;
    ProdDesc pd{};
    pd.a_off = 0;
    pd.b_off = 0;
    pd.a_src = SRC_A;
    pd.b_src = SRC_B;
    pd.lda = pd.ldb = (int32_t)n;
    pd.a_vr = pd.a_vc = pd.b_vr = pd.b_vc = (int32_t)n;
    pd.epi_beg = 0;
    pd.epi_end = 1;
    pl->prods.push_back(pd);
    EpiDesc ed{};
    ed.c_off = 0;
    ed.c_vr = ed.c_vc = (int32_t)n;
    ed.first = 1;
    ed.coef = 1.0;
    pl->epis.push_back(ed);
    return MF_OK;
  }

  const Algo F = power(*algo, levels);
  const int P = F.p, P2 = P * P;
  pl->P = P;
  pl->R = F.R;
  pl->m = round_up((n + P - 1) / P, kLeafTile);
  pl->npad = pl->m * P;
  const int64_t m = pl->m;
  const int64_t mm = m * m;

  std::vector<View> views(P2);
  for (int k = 0; k < P2; ++k) views[k] = block_view(k, P, m, n);
  for (int op = 0; op < 2; ++op)
    for (int k = 0; k < P2; ++k) pl->pre_in.push_back(PreIn{views[k].off, views[k].vr, views[k].vc});

  // Operand of product r for one side: a single-coefficient column is a view
  // (scaled by its coefficient in the epilogue); otherwise a workspace block.
  struct Operand {
    bool zero = false;
    bool view = false;
    int block = -1;
    double scale = 1.0;
    int slot = -1;
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
  int slots = 0;
  for (int side = 0; side < 2; ++side) {
    const std::vector<double>& X = side == 0 ? F.U : F.V;
    std::vector<Operand>& ops = side == 0 ? opa : opb;
    for (int r = 0; r < F.R; ++r) ops[r] = classify(X, r);
  }
  // A product with an all-zero operand (only possible through padding)
  // contributes nothing; skip it and its pre-additions.
  for (int side = 0; side < 2; ++side) {
    const std::vector<double>& X = side == 0 ? F.U : F.V;
    std::vector<Operand>& ops = side == 0 ? opa : opb;
    for (int r = 0; r < F.R; ++r) {
      if (opa[r].zero || opb[r].zero) continue;
      Operand& o = ops[r];
      if (o.view) continue;
      o.slot = slots++;
      PreOut po;
      po.out_off = (int64_t)o.slot * mm;
      po.coef_off = (int32_t)pl->pre_coef.size();
      po.nnz = 0;
      for (int k = 0; k < P2; ++k) {
        const double c = views[k].vr > 0 ? X[(size_t)k * F.R + r] : 0.0;
        pl->pre_coef.push_back(c);
        if (c != 0.0) ++po.nnz;
      }
      pl->pre_out.push_back(po);
      if (side == 0)
        ++pl->n_pre_a;
      else
        ++pl->n_pre_b;
    }
  }
  pl->ws_bytes = (size_t)slots * (size_t)mm * pl->elem;

  std::vector<View> cviews(P2);
  for (int c = 0; c < P2; ++c) cviews[c] = block_view(c, P, m, n);
  std::vector<bool> written(P2, false);
  for (int r = 0; r < F.R; ++r) {
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
    for (int c = 0; c < P2; ++c) {
      const double w = F.w(c, r);
      if (w == 0.0 || cviews[c].vr == 0) continue;
      EpiDesc ed{};
      ed.c_off = cviews[c].off;
      ed.c_vr = cviews[c].vr;
      ed.c_vc = cviews[c].vc;
      ed.first = written[c] ? 0 : 1;
      ed.coef = w * scale;
      written[c] = true;
      pl->epis.push_back(ed);
    }
    pd.epi_end = (int32_t)pl->epis.size();
    pl->prods.push_back(pd);
  }
  // A C block that no remaining product feeds is zero (padding only): the
  // first product stores zeros there.
  for (int c = 0; c < P2; ++c) {
    if (written[c] || cviews[c].vr == 0) continue;
    if (pl->prods.empty()) return fail(MF_ERR_SHAPE, "plan has no products");
    EpiDesc ed{};
    ed.c_off = cviews[c].off;
    ed.c_vr = cviews[c].vr;
    ed.c_vc = cviews[c].vc;
    ed.first = 2;
    ed.coef = 0.0;
    // Insert at the end of product 0's range, shifting later ranges.
    const int at = pl->prods[0].epi_end;
    pl->epis.insert(pl->epis.begin() + at, ed);
    pl->prods[0].epi_end += 1;
    for (size_t q = 1; q < pl->prods.size(); ++q) {
      pl->prods[q].epi_beg += 1;
      pl->prods[q].epi_end += 1;
    }
    written[c] = true;
  }
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
