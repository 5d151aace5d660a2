// Code construction (host, integer only).
//
// Presets are the paper's worked codes (Table I, Table III of Sec. III-A);
// the Mojette codes follow Eq. (moj1) with the projection sets of
// Constructions A and B (Sec. III-C); array codes at other parameters come
// from a deterministic search, since the paper gives no general construction
// for array BP-XOR codes.
#include <algorithm>
#include <cstdlib>
#include <numeric>

#include "host.hpp"

int32_t bpx_code::max_degree() const {
  int32_t m = 0;
  for (int32_t g = 0; g < n_sym(); ++g) m = std::max(m, deg(g));
  return m;
}

namespace bpx {
namespace {

using Sym = std::vector<uint16_t>;

void from_columns(int32_t kind, int32_t n, int32_t k, int32_t b,
                  const std::vector<std::vector<Sym>>& cols, bpx_code* out) {
  out->kind = kind;
  out->n = n;
  out->k = k;
  out->b = b;
  out->col_ptr.assign(1, 0);
  out->sym_ptr.assign(1, 0);
  out->sym_data.clear();
  for (const auto& col : cols) {
    for (Sym s : col) {
      std::sort(s.begin(), s.end());
      out->sym_data.insert(out->sym_data.end(), s.begin(), s.end());
      out->sym_ptr.push_back((int32_t)out->sym_data.size());
    }
    out->col_ptr.push_back((int32_t)out->sym_ptr.size() - 1);
  }
}

// Table I: nodes 1..5, processors 1..2, v_i -> id i-1.
void table1(bpx_code* out) {
  std::vector<std::vector<Sym>> c = {
      {{0}, {1, 2}}, {{1}, {0, 3}}, {{2}, {1, 3}}, {{3}, {0, 2}}, {{0, 1}, {2, 3}}};
  from_columns(BPX_CODE_TABLE1, 5, 2, 2, c, out);
}

// Table III: nodes 1..5, processors 1..3, v_i -> id i-1.
void table3(bpx_code* out) {
  std::vector<std::vector<Sym>> c = {{{0}, {2, 3}, {5, 6}},
                                     {{0, 1}, {3, 4}, {6, 7}},
                                     {{1, 2}, {4, 5}, {7, 8}},
                                     {{6}, {8, 0}, {3, 7}},
                                     {{2}, {1, 5}, {8, 4}}};
  from_columns(BPX_CODE_TABLE3, 5, 3, 3, c, out);
}

void identity(int32_t k, int32_t b, bpx_code* out) {
  std::vector<std::vector<Sym>> c(k);
  for (int32_t j = 0; j < k; ++j)
    for (int32_t i = 0; i < b; ++i) c[j].push_back(Sym{(uint16_t)(j * b + i)});
  from_columns(BPX_CODE_IDENTITY, k, k, b, c, out);
}

// Mojette projection (p, q) over the k x b grid f(z, l), z < b, l < k:
// cell (z, l) goes to bin index (b-1) q [q>0] + (k-1) p [p>0] - z q - l p,
// and holds data id l*b + z.  The column has |p|(k-1) + |q|(b-1) + 1 bins.
bool mojette_column(int32_t p, int32_t q, int32_t k, int32_t b, std::vector<Sym>* col) {
  const int64_t nb = (int64_t)std::abs(p) * (k - 1) + (int64_t)std::abs(q) * (b - 1) + 1;
  const int64_t off = (int64_t)(b - 1) * q * (q > 0) + (int64_t)(k - 1) * p * (p > 0);
  col->assign((size_t)nb, Sym{});
  for (int32_t l = 0; l < k; ++l)
    for (int32_t z = 0; z < b; ++z) {
      const int64_t idx = off - (int64_t)z * q - (int64_t)l * p;
      if (idx < 0 || idx >= nb) return false;
      (*col)[(size_t)idx].push_back((uint16_t)(l * b + z));
    }
  return true;
}

int64_t gcd64(int64_t a, int64_t b) {
  a = std::llabs(a);
  b = std::llabs(b);
  while (b) {
    int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

int mojette(int32_t n, int32_t k, int32_t b, int32_t qe, bpx_code* out, std::string* err) {
  std::vector<int32_t> ps;
  int32_t q = 1;
  if (qe == 0) {
    // Construction A: -floor((n-1)/2) .. ceil((n-1)/2)
    const int32_t lo = -((n - 1) / 2);
    const int32_t hi = n / 2;  // ceil((n-1)/2)
    for (int32_t p = lo; p <= hi; ++p) ps.push_back(p);
  } else {
    if (qe > 16) {
      *err = "mojette_qe too large";
      return BPX_E_INVALID;
    }
    q = 1 << qe;
    // Construction B: odd p from ceil_odd(1-n) to ceil_odd(n-1)
    int32_t lo = 1 - n;
    if (lo % 2 == 0) lo += 1;
    for (int32_t p = lo, c = 0; c < n; p += 2, ++c) ps.push_back(p);
  }
  std::vector<std::vector<Sym>> cols(n);
  for (int32_t i = 0; i < n; ++i) {
    if (gcd64(ps[i], q) != 1) {
      *err = "projection parameters not coprime";
      return BPX_E_INVALID;
    }
    if (!mojette_column(ps[i], q, k, b, &cols[i])) {
      *err = "mojette bin index out of range";
      return BPX_E_INVALID;
    }
  }
  from_columns(BPX_CODE_MOJETTE, n, k, b, cols, out);
  return BPX_OK;
}

// ---------------------------------------------------------------- search --

// Round-based peel over 64-bit masks: returns the known mask, rounds in *r.
inline uint64_t peel_masks(const uint64_t* m, int32_t cnt, uint64_t full, int32_t* r) {
  uint64_t known = 0;
  int32_t rounds = 0;
  while (known != full) {
    uint64_t rel = 0;
    for (int32_t i = 0; i < cnt; ++i) {
      const uint64_t res = m[i] & ~known;
      if (res && !(res & (res - 1))) rel |= res;
    }
    if (!rel) break;
    known |= rel;
    ++rounds;
  }
  *r = rounds;
  return known;
}

struct Objective {
  int64_t U, F, L, D, S;
  bool operator<=(const Objective& o) const { return !(o < *this); }
  bool operator<(const Objective& o) const {
    if (U != o.U) return U < o.U;
    if (F != o.F) return F < o.F;
    if (L != o.L) return L < o.L;
    if (D != o.D) return D < o.D;
    return S < o.S;
  }
};

Objective evaluate(const std::vector<uint64_t>& masks, const std::vector<int32_t>& degs,
                   int32_t n, int32_t k, int32_t b, uint64_t full) {
  Objective o{0, 0, 0, 0, 0};
  for (int32_t d : degs) o.S += d;
  int32_t r = 0;
  o.F = peel_masks(masks.data(), n * b, full, &r) == full ? 0 : 1;
  // enumerate k-subsets of the n columns
  std::vector<int32_t> idx(k);
  std::iota(idx.begin(), idx.end(), 0);
  std::vector<uint64_t> sel((size_t)k * b);
  while (true) {
    for (int32_t t = 0; t < k; ++t)
      for (int32_t i = 0; i < b; ++i) sel[(size_t)t * b + i] = masks[(size_t)idx[t] * b + i];
    const uint64_t kn = peel_masks(sel.data(), k * b, full, &r);
    if (kn == full) {
      o.D += r;
    } else {
      o.U += 1;
      o.L += __builtin_popcountll(full & ~kn);
    }
    int32_t t = k - 1;
    while (t >= 0 && idx[t] == n - k + t) --t;
    if (t < 0) break;
    ++idx[t];
    for (int32_t u = t + 1; u < k; ++u) idx[u] = idx[u - 1] + 1;
  }
  return o;
}

void draw_symbol(SplitMix64& rng, int32_t kb, int32_t sigma, Sym* s) {
  const int32_t d = 1 + (int32_t)rng.below((uint64_t)sigma);
  s->clear();
  while ((int32_t)s->size() < d) {
    const uint16_t x = (uint16_t)rng.below((uint64_t)kb);
    if (std::find(s->begin(), s->end(), x) == s->end()) s->push_back(x);
  }
  std::sort(s->begin(), s->end());
}

uint64_t mask_of(const Sym& s) {
  uint64_t m = 0;
  for (uint16_t x : s) m |= 1ull << x;
  return m;
}

// walk = 0: hill-climb, a change is kept when the whole objective does not
// get worse.  walk = 1: plateau walk, a change is kept when (U, F) does not
// get worse, so the search moves freely among codes with as few failing
// subsets (the finer terms would otherwise pin it to the first local
// optimum); the best code seen by the whole objective is kept.
int array_search(int32_t n, int32_t k, int32_t b, int32_t sigma, uint64_t seed, int32_t restarts,
                 int32_t iters, int32_t walk, bpx_code* out, std::string* err) {
  const int32_t kb = k * b;
  if (kb > 64 || sigma < 1 || sigma > kb || restarts < 1 || iters < 0 || k > n || walk < 0 ||
      walk > 1) {
    *err = "array search needs k <= n, k*b <= 64, 1 <= sigma <= k*b, restarts >= 1, walk 0 or 1";
    return BPX_E_INVALID;
  }
  const uint64_t full = kb == 64 ? ~0ull : ((1ull << kb) - 1);
  const int32_t G = n * b;
  SplitMix64 rng(seed);
  std::vector<Sym> best;
  Objective best_obj{};
  bool have = false;
  std::vector<Sym> syms(G);
  std::vector<uint64_t> masks(G);
  std::vector<int32_t> degs(G);
  for (int32_t rs = 0; rs < restarts; ++rs) {
    for (int32_t g = 0; g < G; ++g) {
      draw_symbol(rng, kb, sigma, &syms[g]);
      masks[g] = mask_of(syms[g]);
      degs[g] = (int32_t)syms[g].size();
    }
    Objective cur = evaluate(masks, degs, n, k, b, full);
    Objective run_best = cur;
    std::vector<Sym> run_syms = syms;
    Sym cand;
    for (int32_t it = 0; it < iters; ++it) {
      const int32_t g = (int32_t)rng.below((uint64_t)G);
      draw_symbol(rng, kb, sigma, &cand);
      const uint64_t old_m = masks[g];
      const int32_t old_d = degs[g];
      masks[g] = mask_of(cand);
      degs[g] = (int32_t)cand.size();
      const Objective o = evaluate(masks, degs, n, k, b, full);
      const bool keep = walk ? (o.U < cur.U || (o.U == cur.U && o.F <= cur.F)) : o <= cur;
      if (keep) {
        cur = o;
        syms[g] = cand;
        if (walk && o < run_best) {
          run_best = o;
          run_syms = syms;
        }
      } else {
        masks[g] = old_m;
        degs[g] = old_d;
      }
    }
    if (!walk) {
      run_best = cur;
      run_syms = syms;
    }
    if (!have || run_best < best_obj) {
      best_obj = run_best;
      best = run_syms;
      have = true;
    }
  }
  std::vector<std::vector<Sym>> cols(n);
  for (int32_t j = 0; j < n; ++j)
    for (int32_t i = 0; i < b; ++i) cols[j].push_back(best[(size_t)j * b + i]);
  from_columns(BPX_CODE_ARRAY_SEARCH, n, k, b, cols, out);
  return BPX_OK;
}

}  // namespace

int build_code(const bpx_code_params& p, bpx_code* out, std::string* err) {
  if (p.reserved != 0) {
    *err = "reserved field of the code parameters must be 0";
    return BPX_E_INVALID;
  }
  switch (p.kind) {
    case BPX_CODE_TABLE1:
      table1(out);
      return BPX_OK;
    case BPX_CODE_TABLE3:
      table3(out);
      return BPX_OK;
    case BPX_CODE_IDENTITY:
      if (p.k < 1 || p.b < 1 || (int64_t)p.k * p.b > 65535) {
        *err = "identity code needs k, b >= 1 and k*b <= 65535";
        return BPX_E_INVALID;
      }
      identity(p.k, p.b, out);
      return BPX_OK;
    case BPX_CODE_MOJETTE:
      if (p.n < 1 || p.k < 1 || p.b < 1 || (int64_t)p.k * p.b > 65535 || p.n > 4096 ||
          p.mojette_qe < 0) {
        *err = "mojette code needs n, k, b >= 1, k*b <= 65535, n <= 4096, qe >= 0";
        return BPX_E_INVALID;
      }
      return mojette(p.n, p.k, p.b, p.mojette_qe, out, err);
    case BPX_CODE_ARRAY_SEARCH:
      if (p.n < 1 || p.k < 1 || p.b < 1) {
        *err = "array search needs n, k, b >= 1";
        return BPX_E_INVALID;
      }
      return array_search(p.n, p.k, p.b, p.sigma_max, p.seed, p.restarts, p.iters, p.walk, out,
                          err);
    default:
      *err = "unknown code kind";
      return BPX_E_INVALID;
  }
}

}  // namespace bpx
