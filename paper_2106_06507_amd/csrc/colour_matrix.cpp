// Colour matrix C(n) of the adjoint decomposition, exact integers
// (Section 2.2, eqs. color_decomposition_adjoint and color_coefficient_adjoint).
//
// With Tr(T^a T^b) = delta^ab and F^a_bc = Tr([T^a, T^b] T^c) (the reading of
// i f^abc under which the projection identity of Section 2.3 holds), repeated
// use of completeness turns the chain (F^{x_1} .. F^{x_k})_{a_1 a_n} into
// +- Tr(T^{a_1} [T^{x_1}, [T^{x_2}, .. [T^{x_k}, T^{a_n}] ..]]) with a sign
// common to all orderings.  Expanding the nested commutator gives 2^k signed
// trace words; C_{s t} = sum over word pairs of sign * N^{loops}, where the
// loops are the index cycles left by contracting sum_a T^a_ij T^a_kl =
// d_il d_jk between a word and the reverse of the other word (complex
// conjugation of a trace reverses it).  The U(1) part of U(N) drops out since
// every gluon sits in a commutator or against a traceless one.
//
// For n >= 7 only the first row is evaluated: renaming the summed colour
// labels of gluons 2..n-1 gives C_{s t} = C_{id, pi(t)} where pi maps s to
// the identity ordering.
#include <stdint.h>

#include <algorithm>
#include <vector>

namespace bg {
namespace {

struct Word {
  int sign;
  uint8_t g[16];
};

void nested_commutator_words(int n, const int* sigma, std::vector<Word>& out) {
  // innermost [x_k, a_n] .. outermost [x_1, .]; words carry gluon labels; the
  // leading gluon 0 is prepended at the end.
  const int k = n - 2;
  std::vector<Word> cur(1);
  cur[0].sign = 1;
  int len = 1;
  cur[0].g[0] = (uint8_t)(n - 1);
  for (int idx = k - 1; idx >= 0; --idx) {
    const uint8_t x = (uint8_t)sigma[idx];
    std::vector<Word> nxt;
    nxt.reserve(cur.size() * 2);
    for (const Word& w : cur) {
      Word left;  // x w
      left.sign = w.sign;
      left.g[0] = x;
      for (int i = 0; i < len; ++i) left.g[i + 1] = w.g[i];
      Word right;  // - w x
      right.sign = -w.sign;
      for (int i = 0; i < len; ++i) right.g[i] = w.g[i];
      right.g[len] = x;
      nxt.push_back(left);
      nxt.push_back(right);
    }
    cur.swap(nxt);
    ++len;
  }
  out.clear();
  for (const Word& w : cur) {
    Word full;
    full.sign = w.sign;
    full.g[0] = 0;
    for (int i = 0; i < len; ++i) full.g[i + 1] = w.g[i];
    out.push_back(full);
  }
}

int find_root(int* parent, int x) {
  while (parent[x] != x) {
    parent[x] = parent[parent[x]];
    x = parent[x];
  }
  return x;
}

// index cycles of sum_a Tr(w) Tr(v) under d_il d_jk contraction
int count_loops(int n, const uint8_t* w, const uint8_t* v) {
  int parent[32];
  for (int i = 0; i < 2 * n; ++i) parent[i] = i;
  int pos_v[16];
  for (int q = 0; q < n; ++q) pos_v[v[q]] = q;
  int comps = 2 * n;
  auto unite = [&](int a, int b) {
    const int ra = find_root(parent, a), rb = find_root(parent, b);
    if (ra != rb) {
      parent[ra] = rb;
      --comps;
    }
  };
  for (int p = 0; p < n; ++p) {
    const int q = pos_v[w[p]];
    unite(p, n + (q + 1) % n);
    unite((p + 1) % n, n + q);
  }
  return comps;
}

int64_t entry(int n, const std::vector<Word>& ws, const std::vector<Word>& vs) {
  int64_t pw[40];
  pw[0] = 1;
  for (int i = 1; i < 40; ++i) pw[i] = pw[i - 1] * 3;
  int64_t tot = 0;
  uint8_t rev[16];
  for (const Word& v : vs) {
    for (int i = 0; i < n; ++i) rev[i] = v.g[n - 1 - i];
    for (const Word& w : ws) tot += (int64_t)(w.sign * v.sign) * pw[count_loops(n, w.g, rev)];
  }
  return tot;
}

void all_perms(int k, std::vector<std::vector<int>>& perms) {
  std::vector<int> p(k);
  for (int i = 0; i < k; ++i) p[i] = i + 1;
  perms.clear();
  do {
    perms.push_back(p);
  } while (std::next_permutation(p.begin(), p.end()));  // lexicographic
}

int64_t perm_rank(const std::vector<int>& p) {
  // lexicographic rank of a permutation of 1..k (Lehmer code)
  const int k = (int)p.size();
  int64_t rank = 0;
  for (int i = 0; i < k; ++i) {
    int smaller = 0;
    for (int j = i + 1; j < k; ++j) smaller += p[j] < p[i];
    int64_t f = 1;
    for (int t = 2; t <= k - 1 - i; ++t) f *= t;
    rank += smaller * f;
  }
  return rank;
}

}  // namespace

// Fills row 0 of C(n) (K entries): the entries C_{id, t} for every ordering t
// in lexicographic order.  Returns K.
int64_t colour_matrix_row0(int n, double* row) {
  const int k = n - 2;
  std::vector<std::vector<int>> perms;
  all_perms(k, perms);
  const int64_t K = (int64_t)perms.size();
  std::vector<Word> w0, wj;
  nested_commutator_words(n, perms[0].data(), w0);
  for (int64_t j = 0; j < K; ++j) {
    nested_commutator_words(n, perms[j].data(), wj);
    row[j] = (double)entry(n, w0, wj);
  }
  return K;
}

// Fills C (K x K row-major) for n in [4, 8].  Returns K.
int64_t colour_matrix(int n, double* C) {
  const int k = n - 2;
  std::vector<std::vector<int>> perms;
  all_perms(k, perms);
  const int64_t K = (int64_t)perms.size();
  std::vector<std::vector<Word>> words(K);
  if (n <= 6) {
    for (int64_t i = 0; i < K; ++i) nested_commutator_words(n, perms[i].data(), words[i]);
    for (int64_t i = 0; i < K; ++i)
      for (int64_t j = i; j < K; ++j) {
        const double v = (double)entry(n, words[i], words[j]);
        C[i * K + j] = v;
        C[j * K + i] = v;
      }
    return K;
  }
  std::vector<Word> w0;
  nested_commutator_words(n, perms[0].data(), w0);
  std::vector<double> row(K);
  std::vector<Word> wj;
  for (int64_t j = 0; j < K; ++j) {
    nested_commutator_words(n, perms[j].data(), wj);
    row[j] = (double)entry(n, w0, wj);
  }
  std::vector<int> pi(k + 1), img(k);
  for (int64_t i = 0; i < K; ++i) {
    for (int pos = 0; pos < k; ++pos) pi[perms[i][pos]] = pos + 1;
    for (int64_t j = 0; j < K; ++j) {
      for (int pos = 0; pos < k; ++pos) img[pos] = pi[perms[j][pos]];
      C[i * K + j] = row[perm_rank(img)];
    }
  }
  return K;
}

}  // namespace bg
