// Budgeted execution plan: wave cut, next-use eviction, uploads and releases,
// then physical placement of every allocation in the device arena.
//
// The paper counts evictions, transfers and transfer bytes (Sec. IV-C) but its
// memory manager is not specified; this plan is the engine's own policy:
//   steps     one per contraction, or waves of ready contractions in schedule
//             order (cut_waves); with lookahead 0 the order is kept and a wave
//             closes before c when (a) an operand of c is produced in the wave,
//             (b) the bytes of the wave's distinct operands and outputs with c
//             would exceed the budget, or (c) the wave holds wave_max;
//   eviction  while used + need > budget, evict the resident tensor that is
//             not an operand of the step with the furthest next use (ties:
//             larger size, then smaller id); leaves and already-spilled
//             intermediates are dropped, other intermediates copied to the
//             host once;
//   then      upload missing operands (ascending id), allocate outputs (a
//             root's output is 0 bytes), run, free what nothing later needs.
#include <algorithm>
#include <map>
#include <set>
#include <tuple>

#include "host.hpp"
#include "../../../include/cdag.h"

namespace cdag {

std::vector<std::vector<int64_t>> cut_waves(const Dag& d, const std::vector<int64_t>& order,
                                            const std::vector<int64_t>& size, int64_t budget,
                                            int64_t wave_max, int64_t lookahead) {
  // A contraction is ready when both operands are leaves or outputs of earlier
  // waves.  Scanning unplaced contractions in schedule order, a wave takes each
  // ready one and passes over at most `lookahead` not-ready ones; it closes at
  // the next not-ready one, when the distinct operand and output bytes would
  // exceed the budget, or at wave_max contractions.
  std::vector<std::vector<int64_t>> waves;
  const int64_t n = (int64_t)order.size();
  std::vector<char> placed(n, 0), produced(d.n_nodes(), 0);
  std::vector<int64_t> member(d.n_nodes(), -1);
  int64_t start = 0, wid = 0;
  auto ready = [&](int64_t x) { return d.is_leaf(x) || produced[x]; };
  while (start < n) {
    std::vector<int64_t> wave;
    int64_t bytes = 0, skipped = 0;
    for (int64_t pos = start; pos < n; ++pos) {
      if (placed[pos]) continue;
      const int64_t c = order[pos], l = d.left[c], r = d.right[c];
      if (!ready(l) || !ready(r)) {
        if (++skipped > lookahead) break;
        continue;
      }
      int64_t extra = 0;
      for (int64_t x : {l, r, c})
        if (member[x] != wid) extra += size[x];
      if (!wave.empty() && (bytes + extra > budget || (int64_t)wave.size() >= wave_max)) break;
      for (int64_t x : {l, r, c}) member[x] = wid;
      bytes += extra;
      wave.push_back(c);
      placed[pos] = 1;
    }
    for (int64_t c : wave) produced[c] = 1;
    waves.push_back(std::move(wave));
    ++wid;
    while (start < n && placed[start]) ++start;
  }
  return waves;
}

PlanTotals plan_totals(const Plan& p) {
  const int64_t C = p.chunks();
  return {C * (int64_t)p.steps.size(), p.halves() * p.peak_resident, C * p.n_evict, C * p.n_h2d,
          C * p.h2d_bytes, C * p.n_d2h, C * p.d2h_bytes};
}

Plan make_plan(const Dag& d, const std::vector<int64_t>& order, const PlanOpts& o) {
  const int64_t n = d.n_nodes();
  if (o.t_chunks < 1) throw Error(CDAG_E_INVALID, "t_chunks must be >= 1");
  for (int64_t u = 0; u < n && o.t_chunks > 1; ++u)
    if (d.nt[u] % o.t_chunks != 0)
      throw Error(CDAG_E_INVALID, "t_chunks must divide the number of time slices of every tensor");
  Plan p;
  p.opts = o;
  // one pass: tensors of nt / t_chunks slices in one half of the budget
  const int64_t budget = o.t_chunks > 1 ? o.budget / 2 : o.budget;
  std::vector<int64_t> size(n);
  for (int64_t u = 0; u < n; ++u) size[u] = p.tsize(d, u);
  if (o.leaves_resident)
    for (int64_t u = 0; u < d.n_leaves; ++u) size[u] = 0;
  if (o.batched) {
    p.steps = cut_waves(d, order, size, budget, o.wave_max, o.lookahead);
  } else {
    p.steps.reserve(order.size());
    for (int64_t c : order) p.steps.push_back({c});
  }
  const int64_t S = (int64_t)p.steps.size();
  // uses[x]: ascending distinct steps where x is an operand
  std::vector<int64_t> cnt(n + 1, 0), last(n, -1);
  for (int64_t s = 0; s < S; ++s)
    for (int64_t c : p.steps[s])
      for (int64_t x : {d.left[c], d.right[c]})
        if (last[x] != s) { last[x] = s; cnt[x]++; }
  std::vector<int64_t> use_off(n + 1, 0);
  for (int64_t u = 0; u < n; ++u) use_off[u + 1] = use_off[u] + cnt[u];
  std::vector<int64_t> uses(use_off[n]), fill(use_off.begin(), use_off.end() - 1);
  std::fill(last.begin(), last.end(), -1);
  for (int64_t s = 0; s < S; ++s)
    for (int64_t c : p.steps[s])
      for (int64_t x : {d.left[c], d.right[c]})
        if (last[x] != s) { last[x] = s; uses[fill[x]++] = s; }
  std::vector<int64_t> ptr(use_off.begin(), use_off.end() - 1);
  auto next_use_after = [&](int64_t x, int64_t s) -> int64_t {
    while (ptr[x] < use_off[x + 1] && uses[ptr[x]] <= s) ++ptr[x];
    return ptr[x] < use_off[x + 1] ? uses[ptr[x]] : INT64_MAX;
  };

  std::vector<int64_t> remaining(n);
  for (int64_t u = 0; u < n; ++u) remaining[u] = d.n_parents(u);
  std::vector<char> resident(n, 0), host_copy(n, 0), pinned(n, 0);
  // evictable residents keyed (next use, size, -id); the max is the victim
  using Key = std::tuple<int64_t, int64_t, int64_t>;
  std::set<Key> cand;
  std::vector<int64_t> key_nu(n, -1);
  auto cand_insert = [&](int64_t x, int64_t nu) { key_nu[x] = nu; cand.insert({nu, size[x], -x}); };
  auto cand_erase = [&](int64_t x) { cand.erase({key_nu[x], size[x], -x}); };
  if (o.leaves_resident)
    for (int64_t u = 0; u < d.n_leaves; ++u) resident[u] = 1;   // never candidates

  int64_t used = 0;
  std::vector<int64_t> operands;
  p.rec_off.reserve(S + 1);
  for (int64_t s = 0; s < S; ++s) {
    p.rec_off.push_back((int64_t)p.recs.size());
    const auto& wave = p.steps[s];
    operands.clear();
    for (int64_t c : wave) { operands.push_back(d.left[c]); operands.push_back(d.right[c]); }
    std::sort(operands.begin(), operands.end());
    operands.erase(std::unique(operands.begin(), operands.end()), operands.end());
    int64_t need = 0;
    for (int64_t x : operands) {
      pinned[x] = 1;
      if (!resident[x]) need += size[x];
    }
    for (int64_t c : wave) need += size[c];
    // pinned residents are keyed by next use == s, below every other candidate
    for (int64_t x : operands)
      if (resident[x] && !(o.leaves_resident && d.is_leaf(x))) { cand_erase(x); cand_insert(x, s); }
    while (used + need > budget) {
      if (cand.empty()) throw Error(CDAG_E_BUDGET, "step " + std::to_string(s) + " does not fit in the budget");
      auto it = std::prev(cand.end());
      int64_t v = -std::get<2>(*it);
      if (pinned[v]) throw Error(CDAG_E_BUDGET, "step " + std::to_string(s) + " does not fit in the budget");
      cand.erase(it);
      if (d.is_leaf(v) || host_copy[v]) {
        p.recs.push_back({OP_DROP, v, s});
      } else {
        p.recs.push_back({OP_D2H, v, s});
        p.n_d2h++;
        p.d2h_bytes += size[v];
        host_copy[v] = 1;
      }
      p.n_evict++;
      resident[v] = 0;
      used -= size[v];
    }
    for (int64_t x : operands) {
      if (resident[x]) continue;
      if (!d.is_leaf(x) && !host_copy[x]) throw Error(CDAG_E_STATE, "plan: intermediate lost");
      p.recs.push_back({OP_H2D, x, s});
      p.n_h2d++;
      p.h2d_bytes += size[x];
      resident[x] = 1;
      used += size[x];
      cand_insert(x, s);
    }
    for (int64_t c : wave) {
      if (d.kind[c] == HCA) continue;
      p.recs.push_back({OP_ALLOC, c, s});
      resident[c] = 1;
      used += size[c];
    }
    p.peak_resident = std::max(p.peak_resident, used);
    for (int64_t c : wave) p.recs.push_back({OP_EXEC, c, s});
    for (int64_t c : wave) { remaining[d.left[c]]--; remaining[d.right[c]]--; }
    for (int64_t x : operands) {
      pinned[x] = 0;
      if (o.leaves_resident && d.is_leaf(x)) continue;
      cand_erase(x);
      if (remaining[x] == 0) {
        p.recs.push_back({OP_FREE, x, s});
        resident[x] = 0;
        host_copy[x] = 0;
        used -= size[x];
      } else {
        cand_insert(x, next_use_after(x, s));
      }
    }
    for (int64_t c : wave)
      if (d.kind[c] != HCA) cand_insert(c, next_use_after(c, s));
  }
  p.rec_off.push_back((int64_t)p.recs.size());
  return p;
}

// ---------------------------------------------------------------- placement
namespace {
constexpr int64_t kAlign = 256;
int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Best-fit allocator over [0, inf) that remembers, per free range, the last
// compute step that touched the memory and the last transfer that read it
// (device ranges: a spill; host ranges: an upload).
class Pool {
 public:
  struct Free { int64_t size, comp, copy; };
  int64_t top = 0;
  std::map<int64_t, Free> free_;             // offset -> block
  std::set<std::pair<int64_t, int64_t>> by_size;  // (size, offset)

  // Returns offset; *comp / *copy receive the waits inherited from the block.
  int64_t alloc(int64_t bytes, int64_t* comp, int64_t* copy) {
    bytes = align_up(std::max<int64_t>(bytes, 1));
    auto it = by_size.lower_bound({bytes, -1});
    if (it != by_size.end()) {
      int64_t off = it->second;
      Free f = free_[off];
      by_size.erase(it);
      free_.erase(off);
      if (f.size > bytes) put(off + bytes, {f.size - bytes, f.comp, f.copy});
      *comp = f.comp;
      *copy = f.copy;
      return off;
    }
    // extend from a free block that ends at the top, else from fresh memory
    if (!free_.empty()) {
      auto last = std::prev(free_.end());
      if (last->first + last->second.size == top) {
        int64_t off = last->first;
        Free f = last->second;
        by_size.erase({f.size, off});
        free_.erase(last);
        top = off + bytes;
        *comp = f.comp;
        *copy = f.copy;
        return off;
      }
    }
    int64_t off = top;
    top += bytes;
    *comp = -1;
    *copy = -1;
    return off;
  }
  void release(int64_t off, int64_t bytes, int64_t comp, int64_t copy) {
    put(off, {align_up(std::max<int64_t>(bytes, 1)), comp, copy});
  }

 private:
  void put(int64_t off, Free f) {
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + f.size == nx->first) {   // merge right
      f = {f.size + nx->second.size, std::max(f.comp, nx->second.comp), std::max(f.copy, nx->second.copy)};
      by_size.erase({nx->second.size, nx->first});
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {                               // merge left
      auto pv = std::prev(nx);
      if (pv->first + pv->second.size == off) {
        off = pv->first;
        f = {f.size + pv->second.size, std::max(f.comp, pv->second.comp), std::max(f.copy, pv->second.copy)};
        by_size.erase({pv->second.size, pv->first});
        free_.erase(pv);
      }
    }
    free_[off] = f;
    by_size.insert({f.size, off});
  }
};
}  // namespace

void place(const Dag& d, Plan& p) {
  const int64_t n = d.n_nodes();
  const int eb = p.opts.elem_bytes;
  p.leaf_off.assign(d.n_leaves, -1);
  int64_t base = 0;
  if (p.opts.leaves_resident) {
    // whole leaves: every pass reads its own slices of them
    for (int64_t u = 0; u < d.n_leaves; ++u) {
      p.leaf_off[u] = base;
      base += align_up(d.size(u, eb));
    }
  }
  p.leaf_region_bytes = base;
  Pool dev, host;
  // last_touch: step of the last kernels that read or wrote the tensor;
  // spilled: step of the spill that wrote its host copy; uploaded: step of the
  // last upload that read that host copy
  std::vector<int64_t> off(n, -1), hoff(n, -1), last_touch(n, -1), spilled(n, -1), uploaded(n, -1);
  if (p.opts.leaves_resident)
    for (int64_t u = 0; u < d.n_leaves; ++u) off[u] = p.leaf_off[u];
  for (PlanRec& r : p.recs) {
    const int64_t x = r.node, s = r.step, sz = p.tsize(d, x);
    switch (r.op) {
      case OP_D2H: {
        int64_t c0, up;
        hoff[x] = host.alloc(sz, &c0, &up);
        r.host_off = hoff[x];
        r.dev_off = off[x];
        r.wait_comp = last_touch[x];
        r.wait_h2d = up;             // an upload still reading this host range
        dev.release(off[x] - base, sz, last_touch[x], s);
        spilled[x] = s;
        off[x] = -1;
        break;
      }
      case OP_DROP:
        r.dev_off = off[x];
        dev.release(off[x] - base, sz, last_touch[x], -1);
        off[x] = -1;
        break;
      case OP_H2D: {
        int64_t comp, spill;
        off[x] = base + dev.alloc(sz, &comp, &spill);
        r.dev_off = off[x];
        r.wait_comp = comp;          // kernels that last touched this memory
        if (d.is_leaf(x)) {
          r.host_off = -1;
          r.wait_d2h = spill;        // a spill still reading this memory
        } else {
          r.host_off = hoff[x];
          r.wait_d2h = std::max(spill, spilled[x]);   // ... and the spill that wrote the host copy
          uploaded[x] = s;
        }
        break;
      }
      case OP_ALLOC: {
        int64_t comp, spill;
        off[x] = base + dev.alloc(sz, &comp, &spill);
        r.dev_off = off[x];
        r.wait_d2h = spill;          // a spill that last read this memory
        break;
      }
      case OP_EXEC:
        r.a_off = off[d.left[x]];
        r.b_off = off[d.right[x]];
        r.dev_off = d.kind[x] == HCA ? -1 : off[x];
        last_touch[d.left[x]] = s;
        last_touch[d.right[x]] = s;
        last_touch[x] = s;
        break;
      case OP_FREE:
        dev.release(off[x] - base, sz, s, -1);
        off[x] = -1;
        if (hoff[x] >= 0) {
          host.release(hoff[x], sz, -1, uploaded[x]);
          hoff[x] = -1;
          uploaded[x] = -1;
        }
        break;
    }
  }
  p.pool_bytes = dev.top;
  p.host_spill_bytes = host.top;
}

}  // namespace cdag
