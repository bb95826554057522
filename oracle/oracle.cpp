// CPU oracle for sparse-sparse tensor contraction.  TEST INFRASTRUCTURE ONLY:
// the tests, the smoke check and the benchmark's CPU-baseline leg are the only
// callers.  It shares no code, header, table or helper with the GPU library.
//
// What it computes is the definition of tensor contraction (paper section
// 2.2, Eq. 1 and Eq. 2):
//
//     z[fX, fY] = sum over c of x[fX, c] * y[c, fY]
//
// with COO operands (section 2.1, Fig. 1).  The contracted mode lists pair up
// position by position, cx[t] with cy[t], and paired modes must have equal
// length (section 2.2).  The output coordinate is the X free coordinates
// (ascending X mode order) followed by the Y free coordinates (ascending Y
// mode order), as in Eq. 4 and the matrix-multiply example of Fig. 2; entries
// with equal output coordinates are summed (section 2.4, accumulation).
//
// Readings where the paper is silent:
//  * Every output coordinate reached by at least one matching pair is
//    emitted, even when its sum is exactly zero (structural semantics).
//  * Repeated input coordinates are independent terms (bilinearity of Eq. 2).
//  * Output entries are returned in ascending lexicographic order of their
//    coordinates; the method itself leaves the order open (section 4.1.3).
//
// Each product is rounded, then added, in double precision (build with
// -ffp-contract=off so no fused multiply-add merges the two roundings).  The
// terms of one output are summed in input order of x, then input order of y;
// the multi-threaded mode partitions outputs by their leading coordinate, so
// every output still sees exactly that order and the result does not depend
// on the thread count.
//
// Alongside each value it returns the sum of |x*y| over its terms and the
// number of terms, which the tests use to bound reordering error.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <random>
#include <set>
#include <thread>
#include <vector>

namespace {

using Tuple = std::vector<int32_t>;

struct Tensor {
  int32_t order;
  const int64_t* dims;
  int64_t nnz;
  const int32_t* idx;  // mode-major [order][nnz]
  const double* val;
  int32_t coord(int32_t mode, int64_t e) const { return idx[(int64_t)mode * nnz + e]; }
};

struct Acc {
  double sum = 0.0;
  double abs = 0.0;
  int64_t terms = 0;
};

struct Result {
  int32_t order = 0;
  std::vector<int32_t> coords;  // entry-major [nnz][order]
  std::vector<double> val, absval;
  std::vector<int64_t> terms;
};

enum { ORACLE_OK = 0, ORACLE_BAD_ARG = 1, ORACLE_DIM_MISMATCH = 2, ORACLE_NO_MEMORY = 3 };

// Modes of a tensor that are not contracted, ascending.
std::vector<int32_t> free_modes(int32_t order, int32_t nc, const int32_t* c) {
  std::vector<int32_t> out;
  for (int32_t m = 0; m < order; ++m) {
    bool contracted = false;
    for (int32_t t = 0; t < nc; ++t) contracted |= (c[t] == m);
    if (!contracted) out.push_back(m);
  }
  return out;
}

int check_tensor(const Tensor& T) {
  if (T.order < 0 || T.nnz < 0) return ORACLE_BAD_ARG;
  if (T.order > 0 && !T.dims) return ORACLE_BAD_ARG;
  for (int32_t m = 0; m < T.order; ++m)
    if (T.dims[m] < 1) return ORACLE_BAD_ARG;
  if (T.nnz > 0 && (!T.val || (T.order > 0 && !T.idx))) return ORACLE_BAD_ARG;
  for (int32_t m = 0; m < T.order; ++m)
    for (int64_t e = 0; e < T.nnz; ++e)
      if (T.coord(m, e) < 0 || T.coord(m, e) >= T.dims[m]) return ORACLE_BAD_ARG;
  return ORACLE_OK;
}

int check_modes(const Tensor& X, const Tensor& Y, int32_t nc, const int32_t* cx, const int32_t* cy) {
  if (nc < 0 || nc > X.order || nc > Y.order) return ORACLE_BAD_ARG;
  if (nc > 0 && (!cx || !cy)) return ORACLE_BAD_ARG;
  for (int32_t t = 0; t < nc; ++t) {
    if (cx[t] < 0 || cx[t] >= X.order || cy[t] < 0 || cy[t] >= Y.order) return ORACLE_BAD_ARG;
    for (int32_t u = 0; u < t; ++u)
      if (cx[u] == cx[t] || cy[u] == cy[t]) return ORACLE_BAD_ARG;
  }
  for (int32_t t = 0; t < nc; ++t)
    if (X.dims[cx[t]] != Y.dims[cy[t]]) return ORACLE_DIM_MISMATCH;
  return ORACLE_OK;
}

Tuple pick(const Tensor& T, int64_t e, const std::vector<int32_t>& modes) {
  Tuple t(modes.size());
  for (size_t k = 0; k < modes.size(); ++k) t[k] = T.coord(modes[k], e);
  return t;
}

struct Problem {
  Tensor X, Y;
  std::vector<int32_t> cx, cy, fx, fy;
};

// The join restricted to one partition of the outputs.  `x_keep` / `y_keep`
// select the entries whose leading output coordinate lies in the partition.
// Small problems use a true nested loop over all pairs; larger ones index Y
// by its contracting tuple (entries kept in input order) and look each x up.
void join_partition(const Problem& p, const std::vector<char>* x_keep, const std::vector<char>* y_keep,
                    bool nested, std::map<Tuple, Acc>& acc) {
  const Tensor& X = p.X;
  const Tensor& Y = p.Y;
  auto emit = [&](int64_t i, int64_t j) {
    Tuple out = pick(X, i, p.fx);
    Tuple yf = pick(Y, j, p.fy);
    out.insert(out.end(), yf.begin(), yf.end());
    double prod = X.val[i] * Y.val[j];
    Acc& a = acc[out];
    a.sum += prod;
    a.abs += std::fabs(prod);
    a.terms += 1;
  };
  if (nested) {
    for (int64_t i = 0; i < X.nnz; ++i) {
      if (x_keep && !(*x_keep)[i]) continue;
      for (int64_t j = 0; j < Y.nnz; ++j) {
        if (y_keep && !(*y_keep)[j]) continue;
        bool match = true;
        for (size_t t = 0; t < p.cx.size(); ++t) match &= X.coord(p.cx[t], i) == Y.coord(p.cy[t], j);
        if (match) emit(i, j);
      }
    }
    return;
  }
  std::map<Tuple, std::vector<int64_t>> ybykey;
  for (int64_t j = 0; j < Y.nnz; ++j) {
    if (y_keep && !(*y_keep)[j]) continue;
    ybykey[pick(Y, j, p.cy)].push_back(j);
  }
  for (int64_t i = 0; i < X.nnz; ++i) {
    if (x_keep && !(*x_keep)[i]) continue;
    auto it = ybykey.find(pick(X, i, p.cx));
    if (it == ybykey.end()) continue;
    for (int64_t j : it->second) emit(i, j);
  }
}

void append(const std::map<Tuple, Acc>& acc, Result& r) {
  for (const auto& kv : acc) {
    r.coords.insert(r.coords.end(), kv.first.begin(), kv.first.end());
    r.val.push_back(kv.second.sum);
    r.absval.push_back(kv.second.abs);
    r.terms.push_back(kv.second.terms);
  }
}

Tensor make(int32_t order, const int64_t* dims, int64_t nnz, const int32_t* idx, const double* val) {
  Tensor t;
  t.order = order;
  t.dims = dims;
  t.nnz = nnz;
  t.idx = idx;
  t.val = val;
  return t;
}

int setup(Problem& p, int32_t xo, const int64_t* xd, int64_t xn, const int32_t* xi, const double* xv, int32_t yo,
          const int64_t* yd, int64_t yn, const int32_t* yi, const double* yv, int32_t nc, const int32_t* cx,
          const int32_t* cy) {
  p.X = make(xo, xd, xn, xi, xv);
  p.Y = make(yo, yd, yn, yi, yv);
  int rc = check_tensor(p.X);
  if (rc == ORACLE_OK) rc = check_tensor(p.Y);
  if (rc == ORACLE_OK) rc = check_modes(p.X, p.Y, nc, cx, cy);
  if (rc != ORACLE_OK) return rc;
  p.cx.assign(cx, cx + nc);
  p.cy.assign(cy, cy + nc);
  p.fx = free_modes(xo, nc, cx);
  p.fy = free_modes(yo, nc, cy);
  return ORACLE_OK;
}

}  // namespace

extern "C" {

// Contract X with Y.  Tensors are host COO arrays, mode-major idx[order][nnz].
// `nthreads` >= 1 splits the outputs by leading coordinate across threads.
// On success *out receives a result handle (free with oracle_result_free).
// Returns 0, or 1 (bad argument / coordinate out of range), 2 (paired modes
// of unequal length), 3 (out of memory).
int oracle_contract(int32_t xo, const int64_t* xd, int64_t xn, const int32_t* xi, const double* xv, int32_t yo,
                    const int64_t* yd, int64_t yn, const int32_t* yi, const double* yv, int32_t nc, const int32_t* cx,
                    const int32_t* cy, int32_t nthreads, void** out) {
  if (!out) return ORACLE_BAD_ARG;
  *out = nullptr;
  Problem p;
  int rc = setup(p, xo, xd, xn, xi, xv, yo, yd, yn, yi, yv, nc, cx, cy);
  if (rc != ORACLE_OK) return rc;
  try {
    Result* r = new Result();
    r->order = (int32_t)(p.fx.size() + p.fy.size());
    const bool nested = (double)xn * (double)yn <= 2.0e6;
    // Leading output coordinate: first X free mode, else first Y free mode.
    const bool split_x = !p.fx.empty();
    const bool split_y = !split_x && !p.fy.empty();
    int32_t parts = std::max<int32_t>(1, nthreads);
    if (!split_x && !split_y) parts = 1;
    const int64_t lead_dim = split_x ? xd[p.fx[0]] : (split_y ? yd[p.fy[0]] : 1);
    parts = (int32_t)std::min<int64_t>(parts, lead_dim);
    if (parts == 1) {
      std::map<Tuple, Acc> acc;
      join_partition(p, nullptr, nullptr, nested, acc);
      append(acc, *r);
    } else {
      std::vector<std::vector<char>> keep(parts);
      const Tensor& T = split_x ? p.X : p.Y;
      const int32_t lead_mode = split_x ? p.fx[0] : p.fy[0];
      for (int32_t k = 0; k < parts; ++k) keep[k].assign(T.nnz, 0);
      for (int64_t e = 0; e < T.nnz; ++e) {
        int64_t c = T.coord(lead_mode, e);
        keep[(size_t)(c * parts / lead_dim)][e] = 1;  // contiguous coordinate ranges
      }
      std::vector<std::map<Tuple, Acc>> accs(parts);
      std::vector<std::thread> pool;
      for (int32_t k = 0; k < parts; ++k)
        pool.emplace_back([&, k] {
          join_partition(p, split_x ? &keep[k] : nullptr, split_y ? &keep[k] : nullptr, nested, accs[k]);
        });
      for (auto& t : pool) t.join();
      for (int32_t k = 0; k < parts; ++k) {
        append(accs[k], *r);
        accs[k].clear();
      }
    }
    *out = r;
  } catch (const std::bad_alloc&) {
    return ORACLE_NO_MEMORY;
  }
  return ORACLE_OK;
}

int64_t oracle_result_nnz(const void* h) { return (int64_t)static_cast<const Result*>(h)->val.size(); }
int32_t oracle_result_order(const void* h) { return static_cast<const Result*>(h)->order; }

// Copy a result out: idx mode-major [order][nnz], values, |term| sums, term counts.
void oracle_result_copy(const void* h, int32_t* idx, double* val, double* absval, int64_t* terms) {
  const Result* r = static_cast<const Result*>(h);
  const int64_t n = (int64_t)r->val.size();
  for (int64_t e = 0; e < n; ++e)
    for (int32_t m = 0; m < r->order; ++m) idx[(int64_t)m * n + e] = r->coords[(size_t)(e * r->order + m)];
  if (n) {
    std::memcpy(val, r->val.data(), sizeof(double) * n);
    std::memcpy(absval, r->absval.data(), sizeof(double) * n);
    std::memcpy(terms, r->terms.data(), sizeof(int64_t) * n);
  }
}

void oracle_result_free(void* h) { delete static_cast<Result*>(h); }

// Group Y by its contracting tuple (cy order): the distinct tuples in
// ascending order with how many Y entries carry each one.  `tuples` is
// mode-major [nc][cap]; *ngroups receives the number of distinct tuples (when
// it exceeds cap, nothing is copied and 1 is returned).
int oracle_group_counts(int32_t yo, const int64_t* yd, int64_t yn, const int32_t* yi, int32_t nc, const int32_t* cy,
                        int64_t cap, int32_t* tuples, int64_t* counts, int64_t* ngroups) {
  Tensor Y = make(yo, yd, yn, yi, nullptr);
  if (yo < 0 || yn < 0 || (yn > 0 && yo > 0 && !yi) || nc < 0 || nc > yo || !ngroups) return ORACLE_BAD_ARG;
  std::vector<int32_t> modes(cy, cy + nc);
  std::map<Tuple, int64_t> g;
  for (int64_t j = 0; j < yn; ++j) g[pick(Y, j, modes)] += 1;
  *ngroups = (int64_t)g.size();
  if ((int64_t)g.size() > cap) return ORACLE_BAD_ARG;
  int64_t k = 0;
  for (const auto& kv : g) {
    for (int32_t t = 0; t < nc; ++t) tuples[(int64_t)t * cap + k] = kv.first[t];
    counts[k++] = kv.second;
  }
  return ORACLE_OK;
}

// For every X entry, the number of Y entries whose contracting tuple equals
// its own (the number of products it takes part in), and the total number of
// matching pairs.
int oracle_match_counts(int32_t xo, const int64_t* xd, int64_t xn, const int32_t* xi, const double* xv, int32_t yo,
                        const int64_t* yd, int64_t yn, const int32_t* yi, const double* yv, int32_t nc,
                        const int32_t* cx, const int32_t* cy, int64_t* per_x, int64_t* total) {
  Problem p;
  int rc = setup(p, xo, xd, xn, xi, xv, yo, yd, yn, yi, yv, nc, cx, cy);
  if (rc != ORACLE_OK) return rc;
  std::map<Tuple, int64_t> ycount;
  for (int64_t j = 0; j < yn; ++j) ycount[pick(p.Y, j, p.cy)] += 1;
  int64_t sum = 0;
  for (int64_t i = 0; i < xn; ++i) {
    auto it = ycount.find(pick(p.X, i, p.cx));
    int64_t c = it == ycount.end() ? 0 : it->second;
    if (per_x) per_x[i] = c;
    sum += c;
  }
  if (total) *total = sum;
  return ORACLE_OK;
}

// Draw `n` output coordinates of the contraction: each draw picks a uniformly
// random X entry among those with at least one matching Y entry, then one of
// its matching Y entries uniformly (std::mt19937_64 seeded with `seed`).
// `coords` is mode-major [out_order][n].  Returns 1 when nothing matches.
int oracle_sample_outputs(int32_t xo, const int64_t* xd, int64_t xn, const int32_t* xi, const double* xv, int32_t yo,
                          const int64_t* yd, int64_t yn, const int32_t* yi, const double* yv, int32_t nc,
                          const int32_t* cx, const int32_t* cy, int64_t n, uint64_t seed, int32_t* coords) {
  Problem p;
  int rc = setup(p, xo, xd, xn, xi, xv, yo, yd, yn, yi, yv, nc, cx, cy);
  if (rc != ORACLE_OK) return rc;
  std::map<Tuple, std::vector<int64_t>> ybykey;
  for (int64_t j = 0; j < yn; ++j) ybykey[pick(p.Y, j, p.cy)].push_back(j);
  std::vector<int64_t> xs;
  std::vector<const std::vector<int64_t>*> groups;
  for (int64_t i = 0; i < xn; ++i) {
    auto it = ybykey.find(pick(p.X, i, p.cx));
    if (it != ybykey.end()) {
      xs.push_back(i);
      groups.push_back(&it->second);
    }
  }
  if (xs.empty()) return ORACLE_BAD_ARG;
  std::mt19937_64 rng(seed);
  const int32_t order = (int32_t)(p.fx.size() + p.fy.size());
  for (int64_t s = 0; s < n; ++s) {
    size_t a = (size_t)(rng() % xs.size());
    const std::vector<int64_t>& g = *groups[a];
    int64_t j = g[(size_t)(rng() % g.size())];
    int32_t m = 0;
    for (int32_t mode : p.fx) coords[(int64_t)(m++) * n + s] = p.X.coord(mode, xs[a]);
    for (int32_t mode : p.fy) coords[(int64_t)(m++) * n + s] = p.Y.coord(mode, j);
    (void)order;
  }
  return ORACLE_OK;
}

// Evaluate the contraction at `n` given output coordinates, one by one:
// z = sum over x with those X free coordinates (input order) and y with those
// Y free coordinates and the same contracting tuple (input order) of x*y.
// Writes value, sum of |x*y| and term count per query (0 terms: no entry).
int oracle_values_at(int32_t xo, const int64_t* xd, int64_t xn, const int32_t* xi, const double* xv, int32_t yo,
                     const int64_t* yd, int64_t yn, const int32_t* yi, const double* yv, int32_t nc,
                     const int32_t* cx, const int32_t* cy, int64_t n, const int32_t* coords, double* val,
                     double* absval, int64_t* terms) {
  Problem p;
  int rc = setup(p, xo, xd, xn, xi, xv, yo, yd, yn, yi, yv, nc, cx, cy);
  if (rc != ORACLE_OK) return rc;
  const size_t nfx = p.fx.size(), nfy = p.fy.size();
  std::map<Tuple, std::vector<int64_t>> queries_by_xfree;
  for (int64_t s = 0; s < n; ++s) {
    Tuple q(nfx);
    for (size_t k = 0; k < nfx; ++k) q[k] = coords[(int64_t)k * n + s];
    queries_by_xfree[q].push_back(s);
    val[s] = 0.0;
    absval[s] = 0.0;
    terms[s] = 0;
  }
  std::map<Tuple, std::vector<int64_t>> ybykey;
  for (int64_t j = 0; j < yn; ++j) ybykey[pick(p.Y, j, p.cy)].push_back(j);
  for (int64_t i = 0; i < xn; ++i) {
    auto qs = queries_by_xfree.find(pick(p.X, i, p.fx));
    if (qs == queries_by_xfree.end()) continue;
    auto g = ybykey.find(pick(p.X, i, p.cx));
    if (g == ybykey.end()) continue;
    for (int64_t s : qs->second) {
      for (int64_t j : g->second) {
        bool same = true;
        for (size_t k = 0; k < nfy; ++k) same &= p.Y.coord(p.fy[k], j) == coords[(int64_t)(nfx + k) * n + s];
        if (!same) continue;
        double prod = p.X.val[i] * p.Y.val[j];
        val[s] += prod;
        absval[s] += std::fabs(prod);
        terms[s] += 1;
      }
    }
  }
  return ORACLE_OK;
}


// The number of distinct output coordinates, nnz(Z), by the definition of
// the output coordinate set (section 2.2, Eq. 2; structural zeros kept):
//
//     S = { (x.c[fX], y.c[fY]) : x in X, y in Y, x.c[cx] = y.c[cy] }
//
// X entries are grouped by their free tuple; a group reaches the union, over
// the contracting tuples its entries carry, of the Y free tuples that carry
// the same contracting tuple.  |S| is the sum of the sizes of those unions.
// No value is read.  `nthreads` >= 1 splits the X groups by leading free
// coordinate (the count does not depend on it).
int oracle_count_outputs(int32_t xo, const int64_t* xd, int64_t xn, const int32_t* xi, const double* xv, int32_t yo,
                         const int64_t* yd, int64_t yn, const int32_t* yi, const double* yv, int32_t nc,
                         const int32_t* cx, const int32_t* cy, int32_t nthreads, int64_t* count) {
  if (!count) return ORACLE_BAD_ARG;
  Problem p;
  int rc = setup(p, xo, xd, xn, xi, xv, yo, yd, yn, yi, yv, nc, cx, cy);
  if (rc != ORACLE_OK) return rc;
  try {
    // Y: contracting tuple -> its distinct free tuples
    std::map<Tuple, std::set<Tuple>> yfree;
    for (int64_t j = 0; j < yn; ++j) yfree[pick(p.Y, j, p.cy)].insert(pick(p.Y, j, p.fy));
    // X: free tuple -> the distinct contracting tuples of its entries that Y has
    int32_t parts = std::max<int32_t>(1, nthreads);
    const int64_t lead_dim = p.fx.empty() ? 1 : xd[p.fx[0]];
    parts = (int32_t)std::min<int64_t>(parts, lead_dim);
    std::vector<int64_t> partial(parts, 0);
    auto run = [&](int32_t k) {
      std::map<Tuple, std::set<const std::set<Tuple>*>> groups;
      for (int64_t i = 0; i < xn; ++i) {
        if (parts > 1 && (int64_t)p.X.coord(p.fx[0], i) * parts / lead_dim != k) continue;
        auto it = yfree.find(pick(p.X, i, p.cx));
        if (it != yfree.end()) groups[pick(p.X, i, p.fx)].insert(&it->second);
      }
      int64_t n = 0;
      for (const auto& g : groups) {
        if (g.second.size() == 1) {
          n += (int64_t)(*g.second.begin())->size();
          continue;
        }
        std::set<Tuple> reach;
        for (const std::set<Tuple>* s : g.second) reach.insert(s->begin(), s->end());
        n += (int64_t)reach.size();
      }
      partial[k] = n;
    };
    if (parts == 1) {
      run(0);
    } else {
      std::vector<std::thread> pool;
      for (int32_t k = 0; k < parts; ++k) pool.emplace_back(run, k);
      for (auto& t : pool) t.join();
    }
    int64_t total = 0;
    for (int64_t n : partial) total += n;
    *count = total;
  } catch (const std::bad_alloc&) {
    return ORACLE_NO_MEMORY;
  }
  return ORACLE_OK;
}

}  // extern "C"
