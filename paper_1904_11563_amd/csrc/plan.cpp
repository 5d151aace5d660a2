// Peeling schedule and plan (host, integer only).
//
// The decoder is the BP (peeling) decoder of Sec. I-A.  Releases are taken
// in rounds: at the start of a round every symbol with exactly one unknown
// id is a candidate; an id released in this round takes the candidate with
// the smallest (degree, g) as its releaser; all of the round's ids become
// known together and the round index is their depth.  Each symbol keeps a
// count of its unknown ids and the XOR of those ids, so a count of one names
// the id directly.
#include <algorithm>
#include <functional>
#include <numeric>

#include "host.hpp"

namespace bpx {

PeelResult peel(const bpx_code& code, const std::vector<int32_t>& syms) {
  const int32_t kb = code.kb();
  PeelResult r;
  r.releaser.assign(kb, -1);
  r.depth.assign(kb, 0);
  const size_t ns = syms.size();
  std::vector<int32_t> cnt(ns), xr(ns);
  std::vector<std::vector<int32_t>> adj(kb);
  for (size_t i = 0; i < ns; ++i) {
    const int32_t g = syms[i];
    cnt[i] = code.deg(g);
    int32_t x = 0;
    for (int32_t e = code.sym_ptr[g]; e < code.sym_ptr[g + 1]; ++e) {
      x ^= code.sym_data[e];
      adj[code.sym_data[e]].push_back((int32_t)i);
    }
    xr[i] = x;
  }
  std::vector<int32_t> best(kb, -1);
  std::vector<int32_t> released;
  int32_t round = 0;
  while (r.n_known < kb) {
    ++round;
    released.clear();
    for (size_t i = 0; i < ns; ++i) {
      if (cnt[i] != 1) continue;
      const int32_t s = xr[i];
      if (best[s] < 0) {
        best[s] = (int32_t)i;
        released.push_back(s);
      } else {
        const int32_t gi = syms[i], gb = syms[best[s]];
        const int32_t di = code.deg(gi), db = code.deg(gb);
        if (di < db || (di == db && gi < gb)) best[s] = (int32_t)i;
      }
    }
    if (released.empty()) break;
    for (int32_t s : released) {
      r.releaser[s] = syms[best[s]];
      r.depth[s] = round;
      ++r.n_known;
    }
    for (int32_t s : released) {
      for (int32_t i : adj[s]) {
        --cnt[i];
        xr[i] ^= s;
      }
      best[s] = -1;
    }
    r.rounds = round;
  }
  return r;
}

namespace {

std::vector<int32_t> symbols_of_columns(const bpx_code& code, const int32_t* cols, int32_t m) {
  std::vector<int32_t> out;
  for (int32_t t = 0; t < m; ++t) {
    const int32_t j = cols[t];
    for (int32_t g = code.col_ptr[j]; g < code.col_ptr[j + 1]; ++g)
      if (code.deg(g) > 0) out.push_back(g);
  }
  std::sort(out.begin(), out.end());
  return out;
}

}  // namespace

int make_plan(const bpx_code& code, const int32_t* arrival, int32_t n_arrival, int32_t n_lost,
              int32_t mode, int64_t M, int64_t K, int64_t N, int32_t prec, int32_t grid,
              bpx_plan* plan, std::string* err) {
  const int32_t n = code.n, kb = code.kb();
  if (!arrival || n_arrival != n) {
    *err = "arrival must list every column";
    return BPX_E_INVALID;
  }
  {
    std::vector<char> seen(n, 0);
    for (int32_t t = 0; t < n; ++t) {
      if (arrival[t] < 0 || arrival[t] >= n || seen[arrival[t]]) {
        *err = "arrival is not a permutation of the columns";
        return BPX_E_INVALID;
      }
      seen[arrival[t]] = 1;
    }
  }
  if (mode < BPX_MODE_ERASURE || mode > BPX_MODE_MIN) {
    *err = "unknown mode";
    return BPX_E_INVALID;
  }
  if (mode == BPX_MODE_ERASURE && (n_lost < 0 || n_lost > n)) {
    *err = "n_lost out of range";
    return BPX_E_INVALID;
  }
  if (M < 1 || K < 1 || N < 1 || prec < BPX_PREC_F32 || prec > BPX_PREC_FP8X2) {
    *err = "bad shape or precision";
    return BPX_E_INVALID;
  }
  plan->code = code;
  plan->mode = mode;
  plan->prec = prec;
  plan->M = M;
  plan->K = K;
  plan->N = N;
  if (grid > 1) {
    if ((int64_t)grid * grid != kb) {
      *err = "the two-dimensional form needs k*b = grid^2";
      return BPX_E_INVALID;
    }
    plan->grid = grid;
    plan->Mb = (M + grid - 1) / grid;
    plan->Nb = N / grid;
  } else {
    plan->grid = 1;
    plan->Mb = (M + kb - 1) / kb;
    plan->Nb = N;
  }

  const int32_t n_avail = mode == BPX_MODE_ERASURE ? n - n_lost : n;
  std::vector<int32_t> syms;
  PeelResult pr;
  bool ok = false;
  int32_t m = 0;
  if (mode == BPX_MODE_FULL) {
    m = n;
    syms = symbols_of_columns(code, arrival, m);
    pr = peel(code, syms);
    ok = pr.n_known == kb;
  } else {
    for (m = 1; m <= n_avail; ++m) {
      syms = symbols_of_columns(code, arrival, m);
      pr = peel(code, syms);
      if (pr.n_known == kb) {
        ok = true;
        break;
      }
    }
    if (!ok) {
      m = n_avail;
      syms = symbols_of_columns(code, arrival, m);
      pr = peel(code, syms);
    }
  }
  plan->decodable = ok;
  plan->prefix_m = m;
  plan->releaser = pr.releaser;
  plan->depth = pr.depth;
  plan->depth_max = 0;
  for (int32_t d : pr.depth) plan->depth_max = std::max(plan->depth_max, d);
  plan->sub_ptr.assign(1, 0);
  plan->sub_data.clear();
  plan->unrecovered.clear();
  for (int32_t s = 0; s < kb; ++s) {
    const int32_t g = pr.releaser[s];
    if (g >= 0) {
      for (int32_t e = code.sym_ptr[g]; e < code.sym_ptr[g + 1]; ++e)
        if (code.sym_data[e] != s) plan->sub_data.push_back(code.sym_data[e]);
    } else {
      plan->unrecovered.push_back(s);
    }
    plan->sub_ptr.push_back((int32_t)plan->sub_data.size());
  }
  if (mode == BPX_MODE_MIN && ok) {
    std::vector<int32_t> rel(pr.releaser.begin(), pr.releaser.end());
    std::sort(rel.begin(), rel.end());
    rel.erase(std::unique(rel.begin(), rel.end()), rel.end());
    plan->computed = rel;
  } else {
    plan->computed = syms;
  }

  // Destination of each computed product: degree-1 releasers go straight to
  // their C block, everything else to a Y slot.
  plan->dest.clear();
  plan->n_yslots = 0;
  for (int32_t g : plan->computed) {
    int32_t d;
    if (code.deg(g) == 1 && pr.releaser[code.sym_data[code.sym_ptr[g]]] == g) {
      d = -1 - (int32_t)code.sym_data[code.sym_ptr[g]];
    } else {
      d = plan->n_yslots++;
    }
    plan->dest.push_back(d);
  }

  // GEMM symbol table.  In the two-dimensional form a gray symbol costs one
  // pass over K per member, the others one pass; the table lists the
  // symbols by decreasing passes (stable), so that a launch deals the
  // longest tiles out first.
  plan->gemm_syms.clear();
  plan->gemm_ids.clear();
  std::vector<size_t> gorder(plan->computed.size());
  std::iota(gorder.begin(), gorder.end(), (size_t)0);
  if (plan->grid > 1) {
    const int32_t G = plan->grid;
    std::vector<int32_t> passes(plan->computed.size(), 1);
    for (size_t i = 0; i < plan->computed.size(); ++i) {
      const int32_t g = plan->computed[i];
      const int32_t b = code.sym_ptr[g], e = code.sym_ptr[g + 1];
      bool same_r = true, same_c = true;
      for (int32_t t = b + 1; t < e; ++t) {
        same_r = same_r && code.sym_data[t] / G == code.sym_data[b] / G;
        same_c = same_c && code.sym_data[t] % G == code.sym_data[b] % G;
      }
      if (!same_r && !same_c) passes[i] = e - b;
    }
    std::stable_sort(gorder.begin(), gorder.end(),
                     [&](size_t x, size_t y) { return passes[x] > passes[y]; });
  }
  for (size_t i : gorder) {
    const int32_t g = plan->computed[i];
    plan->gemm_syms.push_back((int32_t)plan->gemm_ids.size());
    plan->gemm_syms.push_back(code.deg(g));
    plan->gemm_syms.push_back(plan->dest[i]);
    plan->gemm_syms.push_back(g);
    for (int32_t e = code.sym_ptr[g]; e < code.sym_ptr[g + 1]; ++e)
      plan->gemm_ids.push_back(code.sym_data[e]);
  }

  // Peel program: recovered ids in (depth, s) order.  Ids used as
  // subtrahends get an LDS slot; copies already in C that nobody subtracts
  // need no step at all.
  plan->steps.clear();
  plan->step_subs.clear();
  plan->n_lds_slots = 0;
  plan->fused_steps.clear();
  plan->fused_subs.clear();
  plan->fused_ytile.clear();
  plan->n_ytiles = 0;
  if (ok) {
    std::vector<int32_t> order(kb);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) {
      return plan->depth[a] != plan->depth[c] ? plan->depth[a] < plan->depth[c] : a < c;
    });
    std::vector<char> used(kb, 0);
    for (uint16_t u : plan->sub_data) used[u] = 1;
    // LDS slots by liveness: a block's slot is taken when it is recovered
    // and freed after the last step that subtracts it (that step reads its
    // subtrahends before it writes its own result, so it may reuse one of
    // their slots); the lowest free slot is taken first.  The peel kernels'
    // LDS, and with it how many workgroups a CU holds, scale with the count.
    std::vector<int32_t> pos(kb, -1), last_use(kb, -1);
    for (size_t i = 0; i < order.size(); ++i) pos[order[i]] = (int32_t)i;
    for (int32_t s = 0; s < kb; ++s)
      for (int32_t e = plan->sub_ptr[s]; e < plan->sub_ptr[s + 1]; ++e)
        last_use[plan->sub_data[e]] = std::max(last_use[plan->sub_data[e]], pos[s]);
    std::vector<int32_t> slot(kb, -1);
    {
      std::vector<int32_t> free_slots;  // kept sorted descending: back() is the lowest
      for (size_t i = 0; i < order.size(); ++i) {
        const int32_t s = order[i];
        for (int32_t e = plan->sub_ptr[s]; e < plan->sub_ptr[s + 1]; ++e) {
          const int32_t u = plan->sub_data[e];
          if (last_use[u] == (int32_t)i && slot[u] >= 0) {
            free_slots.push_back(slot[u]);
            std::sort(free_slots.begin(), free_slots.end(), std::greater<int32_t>());
          }
        }
        if (!used[s]) continue;
        if (!free_slots.empty()) {
          slot[s] = free_slots.back();
          free_slots.pop_back();
        } else {
          slot[s] = plan->n_lds_slots++;
        }
      }
    }
    auto dest_of = [&](int32_t g) {
      auto it = std::lower_bound(plan->computed.begin(), plan->computed.end(), g);
      return plan->dest[it - plan->computed.begin()];
    };
    // Fused form: the releasers' products stay in LDS Y tiles, numbered in
    // GEMM-table order; every recovered block gets a step and is written.
    std::vector<int32_t> ytile_of_g(code.n_sym(), -1);
    plan->fused_ytile.clear();
    plan->n_ytiles = 0;
    {
      std::vector<char> is_rel(code.n_sym(), 0);
      for (int32_t s = 0; s < kb; ++s)
        if (plan->releaser[s] >= 0) is_rel[plan->releaser[s]] = 1;
      for (size_t t = 0; t < plan->gemm_syms.size() / 4; ++t) {
        const int32_t g = plan->gemm_syms[4 * t + 3];
        if (is_rel[g] && ytile_of_g[g] < 0) ytile_of_g[g] = plan->n_ytiles++;
        plan->fused_ytile.push_back(is_rel[g] ? ytile_of_g[g] : -1);
      }
    }
    for (int32_t s : order) {
      PeelStep st{};
      st.s = s;
      st.src = ytile_of_g[plan->releaser[s]];
      st.nsub = plan->sub_ptr[s + 1] - plan->sub_ptr[s];
      st.sub_off = (int32_t)plan->fused_subs.size();
      st.f64 = plan->depth[s] > 4 ? 1 : 0;
      st.slot = slot[s];
      st.write = 1;
      st.brow = s / plan->grid;
      st.bcol = s % plan->grid;
      for (int32_t e = plan->sub_ptr[s]; e < plan->sub_ptr[s + 1]; ++e)
        plan->fused_subs.push_back(slot[plan->sub_data[e]]);
      plan->fused_steps.push_back(st);
    }
    for (int32_t s : order) {
      const int32_t g = plan->releaser[s];
      const int32_t dst = dest_of(g);
      PeelStep st{};
      st.s = s;
      st.src = dst >= 0 ? dst : -1;
      st.nsub = plan->sub_ptr[s + 1] - plan->sub_ptr[s];
      st.sub_off = (int32_t)plan->step_subs.size();
      st.f64 = plan->depth[s] > 4 ? 1 : 0;
      st.slot = slot[s];
      st.write = dst >= 0 ? 1 : 0;
      st.brow = s / plan->grid;
      st.bcol = s % plan->grid;
      if (st.src < 0 && st.slot < 0) continue;  // copy in place, never reused
      for (int32_t e = plan->sub_ptr[s]; e < plan->sub_ptr[s + 1]; ++e)
        plan->step_subs.push_back(slot[plan->sub_data[e]]);
      plan->steps.push_back(st);
    }
  }
  return ok ? BPX_OK : BPX_E_UNDECODABLE;
}

}  // namespace bpx
