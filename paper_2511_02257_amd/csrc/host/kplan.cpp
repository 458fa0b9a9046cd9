// Launch planning (see kplan.hpp).
#include "kplan.hpp"

#include <algorithm>
#include <climits>
#include <cstring>
#include <set>

#include "../../../include/cdag.h"

namespace cdag {

namespace {
int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

template <class T>
int64_t put(std::vector<uint8_t>& blob, const T& v) {
  int64_t off = (int64_t)blob.size();
  blob.resize(blob.size() + sizeof(T));
  std::memcpy(blob.data() + off, &v, sizeof(T));
  return off;
}
}  // namespace

int64_t elem_bytes_of(int prec) { return prec == CDAG_FP64 ? 16 : 8; }

IndexMap index_map(const Spec& s, int n) {
  IndexMap m{};
  const int rl = s.rank_l, rr = s.rank_r, c = s.n_pairs, ro = rl + rr - 2 * c;
  auto stride = [&](int rank, int axis) {
    int64_t x = 1;
    for (int i = axis + 1; i < rank; ++i) x *= n;
    return x;
  };
  m.n = n;
  m.dk = c;
  int dm = 0, dn = 0;
  for (int a = 0; a < rl; ++a) {
    bool paired = false;
    for (int k = 0; k < c; ++k) paired |= s.pair_l[k] == a;
    if (!paired) m.a_m[dm++] = stride(rl, a);
  }
  for (int b = 0; b < rr; ++b) {
    bool paired = false;
    for (int k = 0; k < c; ++k) paired |= s.pair_r[k] == b;
    if (!paired) m.b_n[dn++] = stride(rr, b);
  }
  for (int k = 0; k < c; ++k) {
    m.a_k[k] = stride(rl, s.pair_l[k]);
    m.b_k[k] = stride(rr, s.pair_r[k]);
  }
  m.dm = dm;
  m.dn = dn;
  // natural output position q (m digits, then n digits) sits at output axis j
  // with perm[j] = q
  int64_t at[8];
  for (int j = 0; j < ro; ++j) at[s.perm[j]] = stride(ro, j);
  for (int d = 0; d < dm; ++d) m.c_m[d] = at[d];
  for (int d = 0; d < dn; ++d) m.c_n[d] = at[dm + d];
  return m;
}

std::map<std::pair<int, int>, TuneShape> tune_shapes(const Dag& d) {
  std::map<std::pair<int, int>, TuneShape> out;
  for (int64_t u = d.n_leaves; u < d.n_nodes(); ++u) {
    if (d.kind[u] == HCA || is_spec(d.kind[u])) continue;   // specs always run the general kernel
    Gemm g;
    d.gemm_shape(u, &g.M, &g.N, &g.K);
    auto it = out.find({d.kind[u], d.nvec[u]});
    if (it == out.end()) {
      out[{d.kind[u], d.nvec[u]}] = {d.nt[u], g};
      continue;
    }
    TuneShape& t = it->second;
    t.nt = std::max(t.nt, (int)d.nt[u]);
    if ((double)g.M * g.N * g.K > (double)t.gemm.M * t.gemm.N * t.gemm.K) t.gemm = g;
  }
  return out;
}

void decompose(const Gemm& g, int nt, int choice, int prec, HecDesc* h, int nt_run) {
  if (choice < 0 || choice >= kNumChoices) throw std::invalid_argument("kernel choice out of range");
  if (g.M > INT32_MAX || g.N > INT32_MAX || g.K > INT32_MAX)
    throw Error(CDAG_E_INVALID, "contraction dimensions exceed 2^31");
  const int variant = choice_variant(choice);
  const int ks = k_step(prec);
  h->map_off = -1;                           // set by the caller for a contraction over index pairs
  h->M = (int32_t)g.M;
  h->N = (int32_t)g.N;
  h->K = (int32_t)g.K;
  const TileShape& ts = kTileShapes[variant_tile(variant)];
  h->nt = nt_run > 0 ? nt_run : nt;
  h->tiles_m = (h->M + ts.bm - 1) / ts.bm;
  h->tiles_n = (h->N + ts.bn - 1) / ts.bn;
  const int64_t base = (int64_t)nt * h->tiles_m * h->tiles_n;
  int64_t splits = std::min<int64_t>((kSplitTarget + base - 1) / base, h->K / kMinKSplit);
  splits = choice_split_k(choice) ? std::max<int64_t>(splits, 1) : 1;
  int64_t kspl = (h->K + splits - 1) / splits;
  kspl = (kspl + ks - 1) / ks * ks;
  splits = (h->K + kspl - 1) / kspl;
  h->splits = (int32_t)splits;
  h->k_split = (int32_t)kspl;
  h->tile_count = (int32_t)((int64_t)h->nt * h->tiles_m * h->tiles_n * splits);
}

int default_tile(int prec, int kind, int n) {
  (void)prec;
  (void)kind;
  int tile = 0;                              // 64 x 64
  if (n % 64 == 0) tile = 0;
  else if (n % 48 == 0) tile = 2;            // 48 x 48
  else if (n % 32 == 0 || n < 32) tile = 1;  // 32 x 32
  return choice_of(variant_of(tile, 1), true);
}

KernelPlan make_kernel_plan(const Dag& d, const Plan& p, int prec, const TileTable& tiles, bool fuse_traces) {
  KernelPlan kp;
  kp.prec = prec;
  const int64_t acc_bytes = prec == CDAG_FP64 ? 8 : 4;   // one real accumulator
  const int64_t S = (int64_t)p.steps.size();

  // tree index of each root, correlator buffers
  std::vector<int64_t> tree_of(d.n_nodes(), -1);
  for (int64_t t = 0; t < (int64_t)d.tree_root.size(); ++t) tree_of[d.tree_root[t]] = t;
  kp.tree_corr_off.resize(d.tree_root.size());
  int64_t co = 0;
  for (size_t t = 0; t < d.tree_root.size(); ++t) {
    kp.tree_corr_off[t] = co;
    co += 16LL * d.nt[d.tree_root[t]];
  }
  kp.corr_bytes = align256(std::max<int64_t>(co, 16));
  int32_t n_corr = 0;
  for (int32_t c : d.corr) n_corr = std::max(n_corr, c + 1);
  kp.sum_nt.assign(n_corr, 0);
  for (size_t g = 0; g < d.corr.size(); ++g) kp.sum_nt[d.corr[g]] = d.nt[d.root_of_graph[g]];
  kp.sum_corr_off.resize(n_corr);
  int64_t so = 0;
  for (int32_t c = 0; c < n_corr; ++c) {
    kp.sum_corr_off[c] = so;
    so += 16LL * kp.sum_nt[c];
  }
  kp.sums_bytes = align256(std::max<int64_t>(so, 16));

  // split-K decision per contraction (independent of batching, so results do
  // not depend on how contractions are grouped into launches)
  auto tile_of = [&](int64_t u) -> int {
    if (is_spec(d.kind[u])) return choice_of(variant_of(kGenTile, 1, 2), false);
    auto it = tiles.find(std::make_tuple(prec, (int)d.kind[u], (int)d.nvec[u]));
    return it != tiles.end() ? it->second : default_tile(prec, d.kind[u], d.nvec[u]);
  };
  for (int64_t u = d.n_leaves; u < d.n_nodes(); ++u)
    if (is_spec(d.kind[u]) && prec >= 2)
      throw Error(CDAG_E_INVALID, "contractions over any index pairs run in FP64 and FP32 only");
  // one index map per (spec, N), laid out after the descriptor tables
  std::map<std::pair<int32_t, int32_t>, int64_t> map_index;
  std::vector<IndexMap> maps;
  // A pass covers nt / t_chunks slices; the split count follows the whole
  // contraction (all nt slices), so it does not change with t_chunks and the
  // results stay bit-identical.
  auto decomp = [&](int64_t u, HecDesc& h) {
    Gemm g;
    d.gemm_shape(u, &g.M, &g.N, &g.K);
    decompose(g, d.nt[u], tile_of(u), prec, &h, (int)(d.nt[u] / p.chunks()));
  };

  // pass 1: workspace size (max over steps) and descriptor counts
  for (int64_t s = 0; s < S; ++s) {
    int64_t ws = 0;
    for (int64_t u : p.steps[s]) {
      if (d.kind[u] == HCA) continue;
      HecDesc h{};
      decomp(u, h);
      if (h.splits > 1) ws += align256((int64_t)h.splits * h.nt * 2 * h.M * h.N * acc_bytes);
    }
    kp.ws_bytes = std::max(kp.ws_bytes, ws);
  }
  // [leaf region][half 0: tensor pool, workspace][half 1 (t_chunks > 1)]...
  const int64_t C = p.chunks();
  kp.chunks = C;
  kp.half_bytes = align256(p.pool_bytes) + kp.ws_bytes;
  kp.ws_off = align256(p.leaf_region_bytes + p.pool_bytes);
  kp.tensors_end = p.leaf_region_bytes + p.halves() * kp.half_bytes;

  // pass 2: descriptors (host blob; arena offset = blob_off + host offset),
  // one set per pass over the time slices: pass k runs in half k % 2 on
  // slices [k nt / C, (k + 1) nt / C) of every tensor.
  kp.launch_off.reserve(C * S + 1);
  for (int64_t k = 0; k < C; ++k) {
    const int64_t shift = (k % 2) * kp.half_bytes;
    // arena offset of operand x of a contraction in pass k: a resident leaf's
    // slices of this pass, else the planned offset in the pass's half
    auto operand_off = [&](int64_t x, int64_t planned) {
      if (p.opts.leaves_resident && d.is_leaf(x)) return p.leaf_off[x] + k * p.tsize(d, x);
      return planned + shift;
    };
    for (int64_t s = 0; s < S; ++s) {
      const size_t step_first = kp.launches.size();
      kp.launch_off.push_back((int64_t)kp.launches.size());
      constexpr int kGroups = kNumVariants + 1;   // the variants, then the general kernel
      std::vector<HecDesc> hec[kGroups];
      int64_t tiles[kGroups] = {0};
      double v_flops[kGroups] = {0}, v_bytes[kGroups] = {0};
      int32_t v_kinds[kGroups] = {0};
      bool v_interior[kGroups];
      std::fill(v_interior, v_interior + kGroups, true);
      double red_bytes = 0, hca_flops = 0, hca_bytes = 0;
      int32_t red_kinds = 0;
      std::vector<RedDesc> red;
      std::vector<HcaDesc> hca;
      int64_t ws = kp.ws_off + shift, items = 0;
      // algorithmic bytes of a launch: each distinct operand read once, each
      // output written once (operands shared by contractions of one launch,
      // e.g. a closing meson traced against many roots, count once)
      std::set<int64_t> v_seen[kGroups], hca_seen;
      auto operand_bytes = [&](std::set<int64_t>& seen, int64_t x) {
        return seen.insert(x).second ? (double)p.tsize(d, x) : 0.0;
      };
      for (int64_t ri = p.rec_off[s]; ri < p.rec_off[s + 1]; ++ri) {
        const PlanRec& r = p.recs[ri];
        if (r.op != OP_EXEC) continue;
        const int64_t u = r.node;
        const double fl = d.flops(u) / (double)C;
        kp.flops += fl;
        const int64_t a_off = operand_off(d.left[u], r.a_off), b_off = operand_off(d.right[u], r.b_off);
        if (d.kind[u] == HCA) {
          HcaDesc h{};
          h.p_off = a_off;
          h.q_off = b_off;
          h.nt = (int32_t)(d.nt[u] / C);
          // relative to the correlator buffer; fixed up below (needs corr_off)
          h.out_off = -1 - (kp.tree_corr_off[tree_of[u]] + 16LL * k * h.nt);
          h.n = d.nvec[u];
          hca.push_back(h);
          hca_flops += fl;
          hca_bytes += operand_bytes(hca_seen, d.left[u]) + operand_bytes(hca_seen, d.right[u]);
          continue;
        }
        HecDesc h{};
        decomp(u, h);
        const bool gen = is_spec(d.kind[u]);
        const int tl = gen ? kGenVariant : choice_variant(tile_of(u));
        h.map_off = -1;
        if (gen) {
          const auto key = std::make_pair(d.kind[u], d.nvec[u]);
          auto it = map_index.find(key);
          if (it == map_index.end()) {
            it = map_index.emplace(key, (int64_t)maps.size()).first;
            maps.push_back(index_map(d.specs[d.kind[u] - kSpecBase], d.nvec[u]));
          }
          h.map_off = -2 - it->second;                   // fixed up below (needs the layout)
        }
        const double ab = operand_bytes(v_seen[tl], d.left[u]) + operand_bytes(v_seen[tl], d.right[u]) +
                          (double)p.tsize(d, u);
        kp.hec_flops += fl;
        kp.hec_bytes += ab;
        v_flops[tl] += fl;
        v_bytes[tl] += ab;
        v_kinds[tl] |= 1 << std::min<int32_t>(d.kind[u], 7);
        h.a_off = a_off;
        h.b_off = b_off;
        h.c_off = r.dev_off + shift;
        h.ws_off = -1;
        h.tile_begin = (int32_t)tiles[tl];
        tiles[tl] += h.tile_count;
        if (gen || !hec_interior(h, kTileShapes[variant_tile(tl)].bm, kTileShapes[variant_tile(tl)].bn, k_step(prec)))
          v_interior[tl] = false;
        kp.hec_items += h.tile_count;
        if (h.splits > 1) {
          h.ws_off = ws;
          RedDesc rd{};
          rd.ws_off = ws;
          rd.c_off = h.c_off;
          rd.mn = h.M * h.N;
          rd.nt = h.nt;
          rd.splits = h.splits;
          rd.item_begin = (int32_t)items;
          items += (2LL * rd.nt * rd.mn + 255) / 256;
          red.push_back(rd);
          red_bytes += 2.0 * rd.nt * (double)rd.mn * ((double)rd.splits * acc_bytes + elem_bytes_of(prec));
          red_kinds |= 1 << d.kind[u];
          ws += align256((int64_t)h.splits * h.nt * 2 * h.M * h.N * acc_bytes);
        }
        hec[tl].push_back(h);
      }
      for (int tl = 0; tl < kGroups; ++tl) {
        if (hec[tl].empty()) continue;
        Launch L{L_HEC, tl, (int32_t)hec[tl].size(), 0, tiles[tl], 0};
        L.flops = v_flops[tl];
        L.bytes = v_bytes[tl];
        L.kinds = v_kinds[tl];
        L.interior = v_interior[tl] ? 1 : 0;
        L.host_desc = (int64_t)kp.blob.size();
        for (auto& h : hec[tl]) put(kp.blob, h);
        kp.launches.push_back(L);
      }
      if (!red.empty()) {
        Launch L{L_RED, 0, (int32_t)red.size(), 0, items, 0};
        L.bytes = red_bytes;
        L.kinds = red_kinds;
        L.host_desc = (int64_t)kp.blob.size();
        for (auto& x : red) put(kp.blob, x);
        kp.launches.push_back(L);
      }
      if (!hca.empty()) {
        int64_t n_titems = 0;
        for (auto& h : hca) { h.item_begin = (int32_t)n_titems; n_titems += h.nt; }
        // the exterior-contraction launch of this step that carries the
        // traces, if fused: the last one of one workgroup per item whose grid
        // stays within kMaxGrid with the trace workgroups added
        Launch* carrier = nullptr;
        for (size_t li = kp.launches.size(); fuse_traces && li-- > step_first;) {
          Launch& L = kp.launches[li];
          if (L.type != L_HEC || L.tile == kGenVariant || variant_grid(L.tile) != 1) continue;
          if (L.n_items + trace_blocks(kTileShapes[variant_tile(L.tile)].nth, n_titems) > kMaxGrid) continue;
          carrier = &L;
          break;
        }
        if (carrier) {
          carrier->tr_n_desc = (int32_t)hca.size();
          carrier->tr_n_items = n_titems;
          carrier->tr_flops = hca_flops;
          carrier->tr_bytes = hca_bytes;
          carrier->kinds |= 1 << HCA;
          carrier->tr_host_desc = (int64_t)kp.blob.size();
          for (auto& h : hca) put(kp.blob, h);
        } else {
          Launch L{L_HCA, 0, (int32_t)hca.size(), 0, n_titems, 0};
          L.flops = hca_flops;
          L.bytes = hca_bytes;
          L.kinds = 1 << HCA;
          L.host_desc = (int64_t)kp.blob.size();
          for (auto& h : hca) put(kp.blob, h);
          kp.launches.push_back(L);
        }
      }
    }
  }
  kp.launch_off.push_back((int64_t)kp.launches.size());

  // cross-diagram sums: per correlator, entries in ascending graph order
  std::vector<std::vector<int64_t>> by_corr(n_corr);
  for (size_t g = 0; g < d.corr.size(); ++g) by_corr[d.corr[g]].push_back((int64_t)g);
  std::vector<XsumDesc> xd;
  std::vector<XsumEntry> xe;
  for (int32_t c = 0; c < n_corr; ++c) {
    XsumDesc x{};
    x.out_off = kp.sum_corr_off[c];   // relative; fixed up below
    x.e_begin = (int32_t)xe.size();
    for (int64_t g : by_corr[c])
      xe.push_back({kp.tree_corr_off[tree_of[d.root_of_graph[g]]], d.w_re[g], d.w_im[g]});
    x.e_end = (int32_t)xe.size();
    x.nt = kp.sum_nt[c];
    xd.push_back(x);
  }
  while (kp.blob.size() % 16) kp.blob.push_back(0);
  kp.xsum = {L_XSUM, 0, (int32_t)xd.size(), 0, (int64_t)xd.size(), (int64_t)kp.blob.size()};
  for (auto& x : xd) put(kp.blob, x);
  const int64_t entries_host = (int64_t)kp.blob.size();
  for (auto& e : xe) put(kp.blob, e);
  while (kp.blob.size() % 16) kp.blob.push_back(0);
  const int64_t maps_host = (int64_t)kp.blob.size();
  for (auto& m : maps) put(kp.blob, m);

  // final layout and fix-ups of buffer-relative offsets
  kp.blob_off = align256(kp.tensors_end);
  kp.corr_off = align256(kp.blob_off + (int64_t)kp.blob.size());
  kp.sums_off = kp.corr_off + kp.corr_bytes;
  kp.total_bytes = align256(kp.sums_off + kp.sums_bytes);
  for (Launch& L : kp.launches) {
    L.desc_off = kp.blob_off + L.host_desc;
    if (L.type == L_HEC && L.tile == kGenVariant) {
      auto* h = reinterpret_cast<HecDesc*>(kp.blob.data() + L.host_desc);
      for (int32_t i = 0; i < L.n_desc; ++i)
        h[i].map_off = kp.blob_off + maps_host + (-2 - h[i].map_off) * (int64_t)sizeof(IndexMap);
    }
    if (L.type == L_HCA) {
      auto* h = reinterpret_cast<HcaDesc*>(kp.blob.data() + L.host_desc);
      for (int32_t i = 0; i < L.n_desc; ++i) h[i].out_off = kp.corr_off + (-1 - h[i].out_off);
    }
    if (L.tr_n_desc > 0) {
      L.tr_desc_off = kp.blob_off + L.tr_host_desc;
      auto* h = reinterpret_cast<HcaDesc*>(kp.blob.data() + L.tr_host_desc);
      for (int32_t i = 0; i < L.tr_n_desc; ++i) h[i].out_off = kp.corr_off + (-1 - h[i].out_off);
    }
  }
  kp.xsum.desc_off = kp.blob_off + kp.xsum.host_desc;
  kp.xsum_entries_off = kp.blob_off + entries_host;
  auto* x = reinterpret_cast<XsumDesc*>(kp.blob.data() + kp.xsum.host_desc);
  for (int32_t i = 0; i < kp.xsum.n_desc; ++i) x[i].out_off += kp.sums_off;
  auto* e = reinterpret_cast<XsumEntry*>(kp.blob.data() + entries_host);
  for (size_t i = 0; i < xe.size(); ++i) e[i].root_off += kp.corr_off;
  return kp;
}

}  // namespace cdag
