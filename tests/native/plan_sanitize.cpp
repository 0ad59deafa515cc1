// Host-side driver of the symbolic plan (step 1 of Fig. 2) for an
// AddressSanitizer / UndefinedBehaviorSanitizer build: valid patterns of
// several shapes (a pattern file written by the test, and generated chains
// with ragged block sizes), every padding and chunk budget, every storage
// code, and each malformed pattern the plan must refuse.  Touches no device.
// Exit status 0 when every check holds; prints the first failure otherwise.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "smsign.h"

namespace {

struct Pattern {
  std::vector<int32_t> bs, row_idx;
  std::vector<int64_t> col_ptr, panel_off;
  sm_bsr_pattern view() const {
    return sm_bsr_pattern{(int32_t)bs.size(), bs.data(), col_ptr.data(), row_idx.data(), panel_off.data()};
  }
};

int fails = 0;
#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++fails;                                                        \
    }                                                                 \
  } while (0)

void finish_panels(Pattern& p) {
  const int n = (int)p.bs.size();
  p.panel_off.assign(n + 1, 0);
  for (int c = 0; c < n; ++c) {
    int64_t h = 0;
    for (int64_t k = p.col_ptr[c]; k < p.col_ptr[c + 1]; ++k) h += p.bs[p.row_idx[k]];
    p.panel_off[c + 1] = p.panel_off[c] + h * p.bs[c];
  }
}

// periodic chain of n atoms, atom i coupled to i +- 1 .. radius, block sizes 1 .. 7
Pattern chain(int n, int radius, uint32_t seed) {
  Pattern p;
  uint32_t x = seed * 2654435761u + 12345u;
  for (int i = 0; i < n; ++i) {
    x = x * 1664525u + 1013904223u;
    p.bs.push_back(1 + (int)((x >> 16) % 7));
  }
  p.col_ptr.push_back(0);
  for (int c = 0; c < n; ++c) {
    std::vector<int> rows;
    for (int r = 0; r < n; ++r) {
      int d = r > c ? r - c : c - r;
      d = d < n - d ? d : n - d;
      if (d <= radius) rows.push_back(r);
    }
    for (int r : rows) p.row_idx.push_back(r);
    p.col_ptr.push_back((int64_t)p.row_idx.size());
  }
  finish_panels(p);
  return p;
}

bool read_pattern(const char* path, Pattern& p) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return false;
  int32_t n = 0;
  int64_t nnzb = 0;
  bool ok = std::fread(&n, 4, 1, f) == 1 && std::fread(&nnzb, 8, 1, f) == 1 && n > 0 && nnzb > 0;
  if (ok) {
    p.bs.resize(n);
    p.col_ptr.resize(n + 1);
    p.row_idx.resize(nnzb);
    p.panel_off.resize(n + 1);
    ok = std::fread(p.bs.data(), 4, n, f) == (size_t)n && std::fread(p.col_ptr.data(), 8, n + 1, f) == (size_t)n + 1 &&
         std::fread(p.row_idx.data(), 4, nnzb, f) == (size_t)nnzb &&
         std::fread(p.panel_off.data(), 8, n + 1, f) == (size_t)n + 1;
  }
  std::fclose(f);
  return ok;
}

// every pad and budget, in index order and in the order of positions (size
// buckets, Morton order): sizes, the per-atom tables and their invariants
void exercise(const Pattern& p) {
  const int n = (int)p.bs.size();
  const sm_bsr_pattern v = p.view();
  std::vector<double> xyz(3 * (size_t)n);
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) xyz[3 * i + d] = std::sin(1.7 * i + 2.3 * d) * (d + 1);
  for (int pad : {32, 64, 128})
  for (int bucket : {-1, 0, 64})
  {
    for (int64_t budget : {(int64_t)0, (int64_t)3 * 64 * 64, (int64_t)1 << 22}) {
      sm_plan* plan = nullptr;
      CHECK(sm_plan_create(&v, pad, budget, &plan) == SM_OK && plan);
      if (!plan) continue;
      if (bucket >= 0) CHECK(sm_plan_set_positions(plan, xyz.data(), bucket) == SM_OK);
      std::vector<int32_t> nn(n), npad(n), loc(n), chunk(n), order(n);
      CHECK(sm_plan_info(plan, nn.data(), npad.data(), loc.data(), chunk.data(), order.data()) == SM_OK);
      int64_t n_sub = 0, n_chunks = 0, ws = 0, nvals = 0;
      for (int st = SM_F64; st <= SM_BF16X3; ++st) {
        CHECK(sm_plan_sizes(plan, st, &n_sub, &n_chunks, &ws, &nvals) == SM_OK);
        CHECK(n_sub == n && n_chunks >= 1 && ws > 0 && nvals == p.panel_off[n]);
      }
      CHECK(sm_plan_sizes(plan, 99, &n_sub, &n_chunks, &ws, &nvals) == SM_ERR_ARG);
      std::vector<int> seen(n, 0);
      for (int i = 0; i < n; ++i) {
        int64_t h = 0;
        for (int64_t k = p.col_ptr[i]; k < p.col_ptr[i + 1]; ++k) h += p.bs[p.row_idx[k]];
        CHECK(nn[i] == h && npad[i] % pad == 0 && npad[i] >= nn[i] && npad[i] < nn[i] + pad);
        CHECK(loc[i] >= 0 && loc[i] + p.bs[i] <= nn[i]);
        CHECK(chunk[i] >= 0 && chunk[i] < n_chunks);
        CHECK(order[i] >= 0 && order[i] < n);
        if (order[i] >= 0 && order[i] < n) ++seen[order[i]];
      }
      for (int i = 0; i < n; ++i) CHECK(seen[i] == 1);
      if (budget == 0) CHECK(n_chunks == 1);
      // chunks are contiguous ranges of the processing order
      for (int g = 1; g < n; ++g) CHECK(chunk[order[g]] == chunk[order[g - 1]] || chunk[order[g]] == chunk[order[g - 1]] + 1);
      if (bucket > 0)   // larger buckets first
        for (int g = 1; g < n; ++g) CHECK(npad[order[g]] / bucket <= npad[order[g - 1]] / bucket);
      if (bucket >= 0) {
        std::vector<double> bad(xyz);
        bad[0] = NAN;
        CHECK(sm_plan_set_positions(plan, bad.data(), bucket) == SM_ERR_ARG);
      }
      sm_plan_destroy(plan);
    }
  }
}

void refuse(Pattern p, const char* what, void (*spoil)(Pattern&)) {
  spoil(p);
  const sm_bsr_pattern v = p.view();
  sm_plan* plan = (sm_plan*)0x1;
  const int rc = sm_plan_create(&v, 64, 0, &plan);
  if (rc != SM_ERR_ARG || plan != nullptr) {
    std::fprintf(stderr, "malformed pattern accepted (%s): rc %d\n", what, rc);
    ++fails;
  }
  CHECK(std::strlen(sm_last_error()) > 0);
}

}  // namespace

int main(int argc, char** argv) {
  for (int prec = SM_F64; prec <= SM_BF16X3; ++prec) {
    sm_sign_opts o;
    CHECK(sm_default_opts(prec, &o) == SM_OK);
    CHECK(sm_ws_storage(&o) >= SM_F64);
  }
  sm_sign_opts o;
  CHECK(sm_default_opts(42, &o) == SM_ERR_ARG);
  if (argc > 1) {
    Pattern f;
    CHECK(read_pattern(argv[1], f));
    if (!f.bs.empty()) exercise(f);
  }
  for (int n : {1, 2, 9, 40}) exercise(chain(n, 2, (uint32_t)n));
  const Pattern base = chain(12, 2, 7);
  {   // pad 48 and a null pattern
    const sm_bsr_pattern v = base.view();
    sm_plan* plan = nullptr;
    CHECK(sm_plan_create(&v, 48, 0, &plan) == SM_ERR_ARG && plan == nullptr);
    CHECK(sm_plan_create(nullptr, 64, 0, &plan) == SM_ERR_ARG);
  }
  refuse(base, "diagonal missing", [](Pattern& p) {
    // drop block (0, 0) and its mirror-free counterpart: column 0 loses its diagonal
    p.row_idx.erase(p.row_idx.begin());
    for (size_t c = 1; c < p.col_ptr.size(); ++c) --p.col_ptr[c];
    finish_panels(p);
  });
  refuse(base, "rows unsorted", [](Pattern& p) { std::swap(p.row_idx[0], p.row_idx[1]); });
  refuse(base, "row out of range", [](Pattern& p) { p.row_idx.back() = 1000; });
  refuse(base, "asymmetric", [](Pattern& p) {
    // column 0 keeps rows {0, 1, 2, 10, 11}; remove row 2 from it only
    p.row_idx.erase(p.row_idx.begin() + 2);
    for (size_t c = 1; c < p.col_ptr.size(); ++c) --p.col_ptr[c];
    finish_panels(p);
  });
  refuse(base, "panel mismatch", [](Pattern& p) { p.panel_off.back() += 1; });
  refuse(base, "zero block size", [](Pattern& p) { p.bs[3] = 0; });
  refuse(base, "empty column", [](Pattern& p) { p.col_ptr[5] = p.col_ptr[4]; });
  refuse(chain(2, 1, 3), "panel taller than 32767 rows", [](Pattern& p) {
    p.bs[0] = p.bs[1] = 20000;
    finish_panels(p);
  });
  refuse(base, "no atoms", [](Pattern& p) {
    p.bs.clear();
    p.col_ptr.assign(1, 0);
    p.panel_off.assign(1, 0);
  });
  if (fails) {
    std::fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  std::printf("plan checks passed\n");
  return 0;
}
