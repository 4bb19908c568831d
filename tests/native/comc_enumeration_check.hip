// Host check of the colour-sampled colour-ordered enumeration (comc.hip):
// for random colour-flow assignments (uniform, chain-constructed, two-colour
// loops only, one colour only) the closed-form count of closing orderings,
// the per-prefix counts and the order of the split enumeration must equal a
// plain depth-first walk over all orderings (1, sigma) with the delta-chain
// condition.  The device functions are __host__ __device__; nothing runs on
// a GPU.  Exit status 0 on success.
#include "comc.hip"

#include <cstdio>
#include <random>
#include <vector>

namespace {

template <int N>
void plain_walk(const int8_t* col, int prev, unsigned used, int depth, std::vector<int>& seq,
                std::vector<std::vector<int>>& out) {
  if (depth == N) {
    if (col[prev] == col[N + 0]) out.push_back(seq);  // i_last == j_1
    return;
  }
  for (int g = 1; g < N; ++g) {
    if ((used >> g) & 1u) continue;
    if (col[N + g] != col[prev]) continue;  // j_g == i_prev
    seq.push_back(g);
    plain_walk<N>(col, g, used | (1u << g), depth + 1, seq, out);
    seq.pop_back();
  }
}

std::vector<int> decode(uint32_t code, int n) {
  std::vector<int> s;
  for (int d = 1; d < n; ++d) s.push_back((int)((code >> (4 * (d - 1))) & 15u));
  return s;
}

template <int N>
int run(std::mt19937_64& rng, int trials) {
  int bad = 0;
  std::vector<int8_t> col(2 * N);
  for (int t = 0; t < trials; ++t) {
    for (int k = 0; k < 2 * N; ++k) col[k] = (int8_t)(rng() % 3);
    if (t % 3 == 0) {
      std::vector<int> perm(N);
      for (int k = 0; k < N; ++k) perm[k] = k;
      for (int k = N - 1; k > 0; --k) std::swap(perm[k], perm[rng() % (k + 1)]);
      for (int k = 0; k < N; ++k) {
        const int c = (int)(rng() % 3);
        col[perm[k]] = (int8_t)c;
        col[N + perm[(k + 1) % N]] = (int8_t)c;
      }
    }
    if (t % 7 == 0)
      for (int k = 0; k < N; ++k) col[k] = col[N + k] = (int8_t)(rng() % 2);
    if (t % 11 == 0)
      for (int k = 0; k < N; ++k) col[k] = col[N + k] = 1;
    std::vector<std::vector<int>> ref;
    std::vector<int> seq;
    plain_walk<N>(col.data(), 0, 1u, 1, seq, ref);
    bool in_range;
    const auto f = bg::comck::load_flow<N>(1, col.data(), 0, in_range);
    const unsigned c = bg::comck::closing_count<N>(f);
    std::vector<std::vector<int>> split;
    unsigned psum = 0;
    bool prefix_ok = true;
    for (int l = 0; l < (N - 1) * (N - 2); ++l) {
      int a, b;
      bg::comck::prefix_of<N>(l, a, b);
      const unsigned pc = bg::comck::prefix_count<N>(f, a, b);
      psum += pc;
      const size_t before = split.size();
      auto visit = [&](uint32_t code) { split.push_back(decode(code, N)); };
      if (pc) bg::comck::orderings<N, 3>(f, 1u | (1u << a) | (1u << b), b, (uint32_t)a | ((uint32_t)b << 4), visit);
      prefix_ok = prefix_ok && split.size() - before == pc;
    }
    if (!in_range || c != ref.size() || psum != c || !prefix_ok || split != ref) {
      if (bad < 5) std::printf("n=%d trial %d: count %u prefix sum %u walk %zu\n", N, t, c, psum, ref.size());
      ++bad;
    }
  }
  std::printf("n=%d: %d flows, %d mismatches\n", N, trials, bad);
  return bad;
}

}  // namespace

int main() {
  std::mt19937_64 rng(20210612);
  int bad = run<4>(rng, 20000) + run<5>(rng, 20000) + run<6>(rng, 10000) + run<7>(rng, 4000) +
            run<8>(rng, 1500) + run<9>(rng, 400);
  return bad != 0;
}
