// Host-side planning tables of libgmres (declarations and contracts in
// host_plan.hpp).  No HIP calls: the engine uploads what these return.
#include "host_plan.hpp"

#include <algorithm>
#include <climits>

namespace gm {
namespace plan {

bool sizes_fit(int32_t nsys, const int64_t* n, const int64_t* nnz, int m, int64_t elem_bytes) {
  int64_t ld = 0, nz = 0;
  for (int k = 0; k < nsys; ++k) {
    if (n[k] < 0 || nnz[k] < 0) return false;
    if (n[k] > (int64_t)INT32_MAX || nnz[k] > (int64_t)INT32_MAX) return false;
    ld += (n[k] + kTile - 1) / kTile * kTile;
    nz += nnz[k];
    if (ld >= (int64_t)INT32_MAX || nz > (int64_t)INT32_MAX - 4 * kBlock - 4) return false;
  }
  return (int64_t)std::max(m + 1, 4) * ld * elem_bytes < ((int64_t)1 << 32);
}

bool row_ptr_piece_ok(const int32_t* v, int64_t n, int32_t nnz, int64_t i0, int64_t i1) {
  for (int64_t i = i0; i < i1; ++i)
    if ((i + 1 < n ? v[i + 1] : nnz) < v[i]) return false;
  return true;
}

void build_row_blocks(const int32_t* rp, int64_t r_begin, int64_t r_end, int budget, std::vector<int32_t>& rb,
                      std::vector<int32_t>* lanes) {
  int64_t r = r_begin;
  const int64_t max_rows = budget >= 4096 ? 2 * kBlock : kBlock;
  while (r < r_end) {
    rb.push_back((int32_t)r);
    int64_t nz = 0, rows = 0, maxlen = 0;
    while (r < r_end && rows < max_rows) {
      const int64_t len = (int64_t)rp[r + 1] - rp[r];
      if (rows > 0 && nz + len > budget) break;
      nz += len;
      maxlen = std::max(maxlen, len);
      ++rows;
      ++r;
      if (nz > budget) break;
    }
    if (lanes) lanes->push_back(row_lanes((int)std::min<int64_t>(maxlen, INT32_MAX)));
  }
}

TileSplit split_tiles(const int32_t* t0, const int32_t* nt, int32_t nsys, int G) {
  TileSplit sp;
  sp.sys_sg0.assign(nsys, -1);
  sp.sys_nsg.assign(nsys, 0);
  const int64_t T = nsys > 0 ? (int64_t)t0[nsys - 1] + nt[nsys - 1] : 0;
  int32_t k = 0;
  for (int b = 0; b < G; ++b) {
    sp.bseg0.push_back((int32_t)sp.seg_t0.size());
    int64_t t = (int64_t)b * T / G;
    const int64_t t1 = (int64_t)(b + 1) * T / G;
    while (t < t1) {
      while ((int64_t)t0[k] + nt[k] <= t) ++k;  // t < T: some system k holds tile t
      const int64_t e = std::min<int64_t>(t1, (int64_t)t0[k] + nt[k]);
      if (sp.sys_sg0[k] < 0) sp.sys_sg0[k] = (int32_t)sp.seg_t0.size();
      sp.sys_nsg[k] += 1;
      sp.seg_t0.push_back((int32_t)t);
      sp.seg_nt.push_back((int32_t)(e - t));
      sp.seg_sys.push_back(k);
      t = e;
    }
  }
  sp.bseg0.push_back((int32_t)sp.seg_t0.size());
  return sp;
}

int ilu_plan(const int32_t* rp, const int32_t* ci, int64_t ld, IluPlan& out) {
  out.diag.assign(ld, -1);
  for (int64_t r = 0; r < ld; ++r) {
    for (int p = rp[r]; p < rp[r + 1]; ++p) {
      if (p > rp[r] && ci[p] <= ci[p - 1]) return ILU_UNSORTED;
      if (ci[p] == r) out.diag[r] = p;
    }
    if (out.diag[r] < 0) {
      if (rp[r] != rp[r + 1]) return ILU_NO_DIAGONAL;  // a stored row without its diagonal
      out.diag[r] = rp[r];                             // padding row: empty ranges
    }
  }
  // sorted columns: the entries before the diagonal are the strictly lower
  // ones and name earlier rows, whose levels are already known
  std::vector<int32_t> lvl(ld, 0), ulv(ld, 0);
  out.depth_l = 0;
  out.depth_u = 0;
  for (int64_t r = 0; r < ld; ++r) {
    int32_t v = 0;
    for (int p = rp[r]; p < out.diag[r]; ++p) v = std::max(v, lvl[ci[p]] + 1);
    lvl[r] = v;
    out.depth_l = std::max(out.depth_l, v + 1);
  }
  for (int64_t r = ld - 1; r >= 0; --r) {
    int32_t v = 0;
    for (int p = out.diag[r] + 1; p < rp[r + 1]; ++p) v = std::max(v, ulv[ci[p]] + 1);
    ulv[r] = v;
    out.depth_u = std::max(out.depth_u, v + 1);
  }
  out.count.assign(out.depth_l + 1, 0);
  out.order.assign(ld, 0);
  for (int64_t r = 0; r < ld; ++r) ++out.count[lvl[r] + 1];
  for (int l = 0; l < out.depth_l; ++l) out.count[l + 1] += out.count[l];
  std::vector<int32_t> fill(out.count.begin(), out.count.end() - 1);
  for (int64_t r = 0; r < ld; ++r) out.order[fill[lvl[r]]++] = (int32_t)r;
  return ILU_OK;
}

void sell_widths(const int32_t* rp, int64_t s0, int64_t s1, int32_t* w) {
  for (int64_t sl = s0; sl < s1; ++sl) {
    int m = 0;
    for (int64_t r = sl * 64; r < sl * 64 + 64; ++r) m = std::max(m, rp[r + 1] - rp[r]);
    w[sl] = m;
  }
}

bool sell_offsets(const int32_t* w, int64_t nslice, std::vector<int32_t>& off) {
  off.assign(nslice + 1, 0);
  int64_t total = 0;
  for (int64_t sl = 0; sl < nslice; ++sl) {
    if (w[sl] >= 2 * kRowLanePer) return false;
    off[sl] = (int32_t)total;
    total += (int64_t)w[sl] * 64;
    if (total >= (int64_t)INT32_MAX) return false;
  }
  off[nslice] = (int32_t)total;
  return true;
}

bool sell_layout(const int32_t* rp, int64_t ld, std::vector<int32_t>& off, std::vector<uint8_t>& len) {
  const int64_t nslice = ld / 64;
  std::vector<int32_t> w(nslice);
  sell_widths(rp, 0, nslice, w.data());
  if (!sell_offsets(w.data(), nslice, off)) return false;
  len.resize(ld);
  for (int64_t r = 0; r < ld; ++r) len[r] = (uint8_t)(rp[r + 1] - rp[r]);
  return true;
}

int persistent_rows_per_thread(int64_t n, int max_rows) {
  const int64_t rows = (n + 1023) / 1024;
  int t = 1;
  while (t < rows && t < max_rows) t *= 2;
  return t;
}

}  // namespace plan
}  // namespace gm
