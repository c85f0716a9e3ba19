// Checks of the host planning tables (paper_2011_01850_amd/csrc/host_plan.cpp)
// against brute-force recomputation on seeded random CSR structures.  Built by
// tests/test_host_plan.py with the address and undefined-behaviour sanitizers
// and bounds-checked standard containers, so an out-of-range read or write in
// the planner fails the run as well as a wrong table.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "host_plan.hpp"

using namespace gm;

namespace {

int g_checks = 0;

#define CHECK(cond, ...)                                      \
  do {                                                        \
    ++g_checks;                                               \
    if (!(cond)) {                                            \
      std::fprintf(stderr, "FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond); \
      std::fprintf(stderr, __VA_ARGS__);                      \
      std::fprintf(stderr, "\n");                             \
      std::exit(1);                                           \
    }                                                         \
  } while (0)

// splitmix64 (Steele, Lea and Flood, 2014)
struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed) {}
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  int64_t uniform(int64_t lo, int64_t hi) { return lo + (int64_t)(next() % (uint64_t)(hi - lo + 1)); }
};

// Row lengths with the mix the solver meets: empty rows, short stencil-like
// rows, and now and then a long row.
std::vector<int32_t> random_row_ptr(Rng& g, int64_t n, int max_long) {
  std::vector<int32_t> rp(n + 1, 0);
  for (int64_t r = 0; r < n; ++r) {
    const int64_t u = g.uniform(0, 99);
    int64_t len = u < 10 ? 0 : u < 90 ? g.uniform(1, 9) : u < 98 ? g.uniform(10, 200) : g.uniform(200, max_long);
    rp[r + 1] = rp[r] + (int32_t)len;
  }
  return rp;
}

int lanes_brute(int len) {
  int best = 1;
  for (int p = 1; p <= kRowLaneMax; p *= 2)
    if (p * kRowLanePer <= len) best = p;
  return best;
}

void check_row_lanes() {
  for (int len = 0; len <= 4096; ++len) {
    const int t = row_lanes(len);
    CHECK(t == lanes_brute(len), "len %d: %d vs %d", len, t, lanes_brute(len));
  }
  CHECK(row_lanes(INT_MAX) == kRowLaneMax, "longest row");
}

void check_row_blocks(Rng& g) {
  const int budgets[] = {1, 7, 64, 1024, 2048, 4096, 8192};
  for (int trial = 0; trial < 40; ++trial) {
    const int64_t n = g.uniform(0, 3000);
    const std::vector<int32_t> rp = random_row_ptr(g, n, trial % 4 == 0 ? 20000 : 600);
    const int64_t b0 = n ? g.uniform(0, n) : 0, b1 = n ? g.uniform(b0, n) : 0;
    for (int budget : budgets) {
      std::vector<int32_t> rb, lanes;
      rb.push_back(-7);  // blocks are appended after what the vector holds
      plan::build_row_blocks(rp.data(), b0, b1, budget, rb, &lanes);
      CHECK(rb[0] == -7, "prefix kept");
      rb.erase(rb.begin());
      CHECK(rb.size() == lanes.size(), "one lane width per block");
      CHECK(rb.empty() == (b0 == b1), "blocks iff rows");
      const int64_t max_rows = budget >= 4096 ? 2 * kBlock : kBlock;
      for (size_t i = 0; i < rb.size(); ++i) {
        const int64_t s = rb[i], e = i + 1 < rb.size() ? rb[i + 1] : b1;
        CHECK(i > 0 || s == b0, "first block starts the range");
        CHECK(e > s && e - s <= max_rows, "block %zu: %lld rows", i, (long long)(e - s));
        const int64_t nz = (int64_t)rp[e] - rp[s];
        CHECK(nz <= budget || e - s == 1, "block %zu over budget with %lld rows", i, (long long)(e - s));
        if (e < b1 && e - s < max_rows && nz <= budget)
          CHECK(nz + (rp[e + 1] - rp[e]) > budget, "block %zu could take row %lld", i, (long long)e);
        int64_t maxlen = 0;
        for (int64_t r = s; r < e; ++r) maxlen = std::max<int64_t>(maxlen, rp[r + 1] - rp[r]);
        CHECK(lanes[i] == row_lanes((int)maxlen), "block %zu lanes", i);
      }
    }
  }
}

void check_row_ptr_pieces(Rng& g) {
  for (int trial = 0; trial < 60; ++trial) {
    const int64_t n = g.uniform(1, 5000);
    std::vector<int32_t> rp = random_row_ptr(g, n, 300);
    const int32_t nnz = rp[n];
    const int64_t piece = g.uniform(1, 700);
    for (int64_t i0 = 0; i0 < n; i0 += piece)
      CHECK(plan::row_ptr_piece_ok(rp.data(), n, nnz, i0, std::min(n, i0 + piece)), "valid row pointer refused");
    // one decrease at j (v[j] < v[j - 1]) or past the end (v[n - 1] > nnz)
    const int64_t j = g.uniform(1, n);
    if (j < n) {
      if (rp[j - 1] == 0) continue;
      rp[j] = rp[j - 1] - 1;
    } else {
      rp[n - 1] = nnz + 1;
    }
    const int64_t bad = j - 1;  // the entry whose successor is smaller
    for (int64_t i0 = 0; i0 < n; i0 += piece) {
      const int64_t i1 = std::min(n, i0 + piece);
      const bool ok = plan::row_ptr_piece_ok(rp.data(), n, nnz, i0, i1);
      const bool holds = bad >= i0 && bad < i1;
      CHECK(ok == !holds, "piece [%lld, %lld) with a decrease after %lld", (long long)i0, (long long)i1,
            (long long)bad);
    }
  }
}

void check_split(Rng& g) {
  const int grids[] = {1, 2, 3, 7, 64, 256, 2048, 4096};
  for (int trial = 0; trial < 50; ++trial) {
    const int32_t nsys = (int32_t)g.uniform(1, trial % 5 == 0 ? 600 : 12);
    std::vector<int32_t> t0(nsys), nt(nsys);
    int32_t t = 0;
    for (int k = 0; k < nsys; ++k) {
      t0[k] = t;
      nt[k] = (int32_t)(g.uniform(0, 9) == 0 ? 0 : g.uniform(1, trial % 3 == 0 ? 4000 : 40));
      t += nt[k];
    }
    const int64_t T = t;
    for (int G : grids) {
      const plan::TileSplit sp = plan::split_tiles(t0.data(), nt.data(), nsys, G);
      const size_t nseg = sp.seg_t0.size();
      CHECK(sp.bseg0.size() == (size_t)G + 1 && sp.bseg0[0] == 0 && sp.bseg0[G] == (int32_t)nseg, "bseg0");
      CHECK(sp.seg_nt.size() == nseg && sp.seg_sys.size() == nseg, "segment table sizes");
      CHECK(sp.sys_sg0.size() == (size_t)nsys && sp.sys_nsg.size() == (size_t)nsys, "system table sizes");
      std::vector<int> seen(T, 0);
      for (int b = 0; b < G; ++b) {
        CHECK(sp.bseg0[b] <= sp.bseg0[b + 1], "bseg0 order");
        int64_t at = (int64_t)b * T / G;
        for (int32_t q = sp.bseg0[b]; q < sp.bseg0[b + 1]; ++q) {
          CHECK(sp.seg_t0[q] == at && sp.seg_nt[q] > 0, "workgroup %d segment %d", b, q);
          const int32_t k = sp.seg_sys[q];
          CHECK(k >= 0 && k < nsys, "segment system");
          CHECK(sp.seg_t0[q] >= t0[k] && sp.seg_t0[q] + sp.seg_nt[q] <= t0[k] + nt[k], "segment inside its system");
          for (int32_t x = 0; x < sp.seg_nt[q]; ++x) ++seen[sp.seg_t0[q] + x];
          at += sp.seg_nt[q];
        }
        CHECK(at == (int64_t)(b + 1) * T / G, "workgroup %d covers its tiles", b);
      }
      for (int64_t x = 0; x < T; ++x) CHECK(seen[x] == 1, "tile %lld covered %d times", (long long)x, seen[x]);
      for (int k = 0; k < nsys; ++k) {
        int32_t first = -1, cnt = 0;
        for (size_t q = 0; q < nseg; ++q)
          if (sp.seg_sys[q] == k) {
            if (first < 0) first = (int32_t)q;
            CHECK((int32_t)q == first + cnt, "system %d segments contiguous", k);
            ++cnt;
          }
        CHECK(sp.sys_sg0[k] == first && sp.sys_nsg[k] == cnt, "system %d: %d %d vs %d %d", k, sp.sys_sg0[k],
              sp.sys_nsg[k], first, cnt);
      }
    }
  }
}

// Random sparse structure with sorted unique columns and the diagonal in
// every stored row, then empty padding rows up to ld.
void random_ilu_structure(Rng& g, int64_t n, int64_t ld, std::vector<int32_t>& rp, std::vector<int32_t>& ci) {
  rp.assign(ld + 1, 0);
  ci.clear();
  const int64_t band = g.uniform(1, 40);
  for (int64_t r = 0; r < ld; ++r) {
    if (r < n) {
      std::vector<int32_t> cols{(int32_t)r};
      const int64_t extra = g.uniform(0, 6);
      for (int64_t e = 0; e < extra; ++e) {
        const int64_t c = g.uniform(0, 3) == 0 ? g.uniform(0, n - 1)
                                               : std::min<int64_t>(n - 1, std::max<int64_t>(0, r + g.uniform(-band, band)));
        cols.push_back((int32_t)c);
      }
      std::sort(cols.begin(), cols.end());
      cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
      ci.insert(ci.end(), cols.begin(), cols.end());
    }
    rp[r + 1] = (int32_t)ci.size();
  }
}

void check_ilu(Rng& g) {
  for (int trial = 0; trial < 40; ++trial) {
    const int64_t n = g.uniform(1, 1500), ld = (n + 255) / 256 * 256;
    std::vector<int32_t> rp, ci;
    random_ilu_structure(g, n, ld, rp, ci);
    plan::IluPlan ip;
    CHECK(plan::ilu_plan(rp.data(), ci.data(), ld, ip) == plan::ILU_OK, "valid structure refused");
    CHECK(ip.diag.size() == (size_t)ld && ip.order.size() == (size_t)ld, "table sizes");
    CHECK(ip.count.size() == (size_t)ip.depth_l + 1 && ip.count[0] == 0 && ip.count[ip.depth_l] == ld, "count");
    for (int64_t r = 0; r < ld; ++r) {
      if (rp[r] == rp[r + 1]) {
        CHECK(ip.diag[r] == rp[r], "padding row %lld", (long long)r);
      } else {
        CHECK(ip.diag[r] >= rp[r] && ip.diag[r] < rp[r + 1] && ci[ip.diag[r]] == r, "diag of row %lld", (long long)r);
      }
    }
    // levels read back from the order, against a fixed point of
    // level(r) = 1 + max level of the rows r's strictly lower entries name
    std::vector<int32_t> lvl(ld, -1), want(ld, 0), seen(ld, 0);
    for (int32_t l = 0; l < ip.depth_l; ++l) {
      CHECK(ip.count[l] < ip.count[l + 1], "level %d empty", l);
      for (int32_t q = ip.count[l]; q < ip.count[l + 1]; ++q) {
        const int32_t r = ip.order[q];
        CHECK(r >= 0 && r < ld && !seen[r], "order is a permutation");
        CHECK(q == ip.count[l] || ip.order[q - 1] < r, "ascending rows within level %d", l);
        seen[r] = 1;
        lvl[r] = l;
      }
    }
    auto fixpoint = [&](bool lower) {
      std::vector<int32_t> v(ld, 0);
      for (bool changed = true; changed;) {
        changed = false;
        for (int64_t r = 0; r < ld; ++r)
          for (int32_t p = rp[r]; p < rp[r + 1]; ++p) {
            if (lower ? ci[p] >= r : ci[p] <= r) continue;
            if (v[ci[p]] + 1 > v[r]) {
              v[r] = v[ci[p]] + 1;
              changed = true;
            }
          }
      }
      return v;
    };
    want = fixpoint(true);
    for (int64_t r = 0; r < ld; ++r) CHECK(lvl[r] == want[r], "row %lld level %d vs %d", (long long)r, lvl[r], want[r]);
    const std::vector<int32_t> up = fixpoint(false);
    CHECK(ip.depth_u == *std::max_element(up.begin(), up.end()) + 1, "upper depth");

    // refusals: a stored row without its diagonal; columns out of order; a duplicate
    const int64_t r = g.uniform(0, n - 1);
    if (rp[r + 1] - rp[r] >= 2) {
      std::vector<int32_t> c2 = ci;
      std::swap(c2[rp[r]], c2[rp[r] + 1]);
      CHECK(plan::ilu_plan(rp.data(), c2.data(), ld, ip) == plan::ILU_UNSORTED, "swapped columns accepted");
      c2 = ci;
      c2[rp[r] + 1] = c2[rp[r]];
      CHECK(plan::ilu_plan(rp.data(), c2.data(), ld, ip) == plan::ILU_UNSORTED, "duplicate column accepted");
    }
    {
      std::vector<int32_t> c2 = ci;
      const int32_t d = [&] {
        for (int32_t p = rp[r]; p < rp[r + 1]; ++p)
          if (ci[p] == r) return p;
        return -1;
      }();
      CHECK(d >= 0, "generator stores the diagonal");
      // move the diagonal's column to a free column that keeps the order
      const int32_t lo = d > rp[r] ? c2[d - 1] : -1, hi = d + 1 < rp[r + 1] ? c2[d + 1] : (int32_t)n;
      int32_t c = -1;
      for (int32_t x = lo + 1; x < hi; ++x)
        if (x != r) c = x;
      if (c >= 0) {
        c2[d] = c;
        CHECK(plan::ilu_plan(rp.data(), c2.data(), ld, ip) == plan::ILU_NO_DIAGONAL, "row without diagonal accepted");
      }
    }
  }
}

void check_sell(Rng& g) {
  for (int trial = 0; trial < 40; ++trial) {
    const int64_t ld = 64 * g.uniform(0, 80);
    std::vector<int32_t> rp(ld + 1, 0);
    for (int64_t r = 0; r < ld; ++r) rp[r + 1] = rp[r] + (int32_t)g.uniform(0, 2 * kRowLanePer - 1);
    std::vector<int32_t> off;
    std::vector<uint8_t> len;
    CHECK(plan::sell_layout(rp.data(), ld, off, len), "short rows refused");
    CHECK(off.size() == (size_t)ld / 64 + 1 && off[0] == 0 && len.size() == (size_t)ld, "sizes");
    for (int64_t s = 0; s < ld / 64; ++s) {
      int w = 0;
      for (int64_t r = 64 * s; r < 64 * s + 64; ++r) {
        w = std::max(w, rp[r + 1] - rp[r]);
        CHECK(len[r] == rp[r + 1] - rp[r], "row %lld length", (long long)r);
      }
      CHECK(off[s + 1] - off[s] == 64 * w, "slice %lld width", (long long)s);
    }
    // the two-step form over random pieces of slices gives the same offsets
    {
      const int64_t nslice = ld / 64;
      std::vector<int32_t> wid(nslice, -1), off2;
      for (int64_t s0 = 0; s0 < nslice;) {
        const int64_t s1 = std::min<int64_t>(nslice, s0 + g.uniform(1, 9));
        plan::sell_widths(rp.data(), s0, s1, wid.data());
        s0 = s1;
      }
      CHECK(plan::sell_offsets(wid.data(), nslice, off2) && off2 == off, "piecewise offsets");
    }
    if (ld > 0) {
      const int64_t r = g.uniform(0, ld - 1);
      for (int64_t q = r + 1; q <= ld; ++q) rp[q] += 2 * kRowLanePer - (rp[r + 1] - rp[r]) + (int32_t)g.uniform(0, 3);
      CHECK(!plan::sell_layout(rp.data(), ld, off, len), "a row of %d entries accepted", rp[r + 1] - rp[r]);
    }
  }
}

void check_sizes() {
  const int64_t big = (int64_t)1 << 21;  // 128^3 rows
  int64_t n = big, nnz = 14581760;
  CHECK(plan::sizes_fit(1, &n, &nnz, 50, 4), "the 128^3 float32 basis");
  CHECK(plan::sizes_fit(1, &n, &nnz, 255, 8) == false, "256 float64 columns of 2^21 rows reach 2^32 bytes");
  CHECK(plan::sizes_fit(1, &n, &nnz, 254, 8), "255 float64 columns of 2^21 rows stay below 2^32 bytes");
  n = (int64_t)INT32_MAX + 1;
  CHECK(!plan::sizes_fit(1, &n, &nnz, 10, 2), "n beyond 32 bits");
  n = -1;
  CHECK(!plan::sizes_fit(1, &n, &nnz, 10, 2), "negative n");
  n = 1000;
  nnz = (int64_t)INT32_MAX - 4 * kBlock - 4;
  CHECK(plan::sizes_fit(1, &n, &nnz, 10, 2), "largest non-zero count");
  nnz += 1;
  CHECK(!plan::sizes_fit(1, &n, &nnz, 10, 2), "non-zero count past the pad");
  int64_t ns[3] = {100, 0, 300}, nz[3] = {500, 0, 900};
  CHECK(plan::sizes_fit(3, ns, nz, 30, 4), "a small batch");
  // m + 1 < 4 still reserves 4 columns
  n = (int64_t)1 << 26;  // 4 columns of 2^26 float64 rows: 2^31 bytes
  nnz = 0;
  CHECK(plan::sizes_fit(1, &n, &nnz, 1, 8), "4 reserved columns fit");
  n = (int64_t)1 << 27;  // exactly 2^32 bytes with 4 columns
  CHECK(!plan::sizes_fit(1, &n, &nnz, 1, 8), "4 reserved columns of 2^27 float64 rows reach 2^32 bytes");
}

void check_persistent_tier() {
  for (int64_t n = 1; n <= 1024 * 64 + 5000; n += 97) {
    const int64_t rows = (n + 1023) / 1024;
    const int want = rows <= 1 ? 1 : rows <= 2 ? 2 : rows <= 4 ? 4 : rows <= 8 ? 8 : rows <= 16 ? 16 : rows <= 32 ? 32 : 64;
    CHECK(plan::persistent_rows_per_thread(n, 64) == want, "n %lld", (long long)n);
  }
}

}  // namespace

int main() {
  Rng g(20110185);
  check_row_lanes();
  check_row_blocks(g);
  check_row_ptr_pieces(g);
  check_split(g);
  check_ilu(g);
  check_sell(g);
  check_sizes();
  check_persistent_tier();
  std::printf("host plan checks: %d passed\n", g_checks);
  return 0;
}
