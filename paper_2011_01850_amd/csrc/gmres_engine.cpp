// Host engine and C-ABI of libgmres: setup (matrix copies, row blocks,
// autotuner, workspace), the restart-cycle schedule (direct launches or one
// captured hipGraph per cycle) and the entry points declared in gmres.h.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <memory>
#include <new>
#include <thread>
#include <vector>

#include "gmres.h"
#include "spai.h"
#include "gmres_internal.hpp"

using namespace gm;

namespace {

constexpr uint32_t kMagic = 0x474d5253u;  // "GMRS"

struct Fail {
  int code;
};

inline void hip_check(hipError_t e) {
  if (e == hipErrorOutOfMemory) throw Fail{GMRES_ENOMEM};
  if (e != hipSuccess) throw Fail{GMRES_EHIP};
}

struct System {
  int64_t n = 0, nnz = 0;
  int64_t row0 = 0;  // first global row
  int64_t nz0 = 0;   // first global non-zero
  int32_t nt = 0, t0 = 0;  // tiles, first tile
};

// non-zero budgets per SpMV row block that the autotuner times
constexpr int kTuneBudgets[] = {1024, 2048, 4096};

// SpMV row blocks for one non-zero budget: host tables, uploaded on first use.
struct RowBlocks {
  int budget = 0;
  std::vector<int32_t> rb;     // first row of each block, then the sentinel ld
  std::vector<int32_t> sys;    // system of each block
  std::vector<int32_t> lanes;  // max row_lanes over the block's rows
  std::vector<int32_t> rb0, nrb;  // per system: first block, block count
  std::vector<int32_t> p;         // row pointer at each block start, then nnz
  const int32_t *d_rb = nullptr, *d_sys = nullptr, *d_lanes = nullptr, *d_rb0 = nullptr, *d_nrb = nullptr,
                *d_p = nullptr;
};

}  // namespace

struct gmres_ctx {
  uint32_t magic = kMagic;
  hipStream_t stream = nullptr;  // library-owned, default priority
  gmres_options opt{};
  std::vector<System> sys;
  int64_t ld = 0, nnz = 0, nrows = 0;
  int32_t ntile = 0, nrb = 0;
  std::vector<int32_t> rp_host;  // global row pointer (ld + 1)
  std::vector<std::unique_ptr<RowBlocks>> rbt;  // row-block tables built so far
  std::vector<void*> allocs;
  std::vector<hipEvent_t> tune_ev;  // the SpMV autotuner's event pairs
  size_t bytes = 0;
  KArgs a{};
  // host mirror of per-system state
  SysState* st_host = nullptr;  // pinned
  hipGraphExec_t gexec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipStream_t user = nullptr;    // the caller's stream: work it enqueued comes first
  hipEvent_t evu = nullptr;
  bool spai_set = false;
  spai_handle spai = nullptr;    // network instance on this handle's pattern (gmres_spai_infer)
  // persistent schedule: one workgroup per system, one launch per solve
  bool persistent = false;
  bool near_cols = false;  // every column within 32767 of its row (16-bit sliced ELL offsets)
  int64_t part_rows = 0;   // rows of the partial tables a.part, a.part2
  std::vector<gmres_tune_class> tune;  // size classes and their probe systems
  double tune_probe_us[3] = {-1.0, -1.0, -1.0};  // probe time per SpMV variant
  int pv = 0;                          // the persistent kernel's SpMV variant
  int32_t* order = nullptr;      // systems, largest first
  int32_t* counter = nullptr;    // queue position
  hipGraphExec_t pexec = nullptr;
  // batch gather/scatter pointer tables (device)
  const double** bptrs = nullptr;
  double** xptrs = nullptr;
  // staging for the plain SpMV / residual entry points (ld rows each)
  double* xs = nullptr;
  double* ys = nullptr;
  // SPLIT storage: the float64 values reassembled for the network inputs
  // (allocated on the first inference)
  double* a64_merged = nullptr;
  // sums of squares: kSumsqBlocks partials (allocated on first use); ||A||_F
  // once computed (negative until then)
  double* sq_part = nullptr;
  double afro = -1.0;

  template <typename T>
  T* alloc(size_t count) {
    size_t nb = 0;
    void* p = cache_alloc(count * sizeof(T), &nb);
    if (!p) throw Fail{GMRES_ENOMEM};
    allocs.push_back(p);
    bytes += nb;
    return static_cast<T*>(p);
  }

  // the stream is drained first, so no kernel still reads a block that goes
  // back to the cache (also on a create that failed part way)
  ~gmres_ctx() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (spai) (void)spai_destroy(spai);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (pexec) (void)hipGraphExecDestroy(pexec);
    for (void* p : allocs) cache_free(p);
    if (st_host) (void)hipHostFree(st_host);
    for (hipEvent_t e : tune_ev) (void)hipEventDestroy(e);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (evu) (void)hipEventDestroy(evu);
    if (stream) (void)hipStreamDestroy(stream);
    magic = 0;
  }
};

namespace {

// ROCTx ranges around the timed launches of the kernel timing harness, so a
// profiler that renames kernels by range reports exactly those launches on
// a row of their own.  Resolved at run time; absent library = no markers.
struct Roctx {
  int (*push)(const char*) = nullptr;
  int (*pop)() = nullptr;
};
const Roctx& roctx() {
  static const Roctx r = [] {
    Roctx x;
    void* lib = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (lib) {
      x.push = reinterpret_cast<int (*)(const char*)>(dlsym(lib, "roctxRangePushA"));
      x.pop = reinterpret_cast<int (*)()>(dlsym(lib, "roctxRangePop"));
      if (!x.push || !x.pop) x = Roctx{};
    }
    if (x.push) {  // the first range call sets the marker library up: not inside a timing
      x.push("gmres:marker-setup");
      x.pop();
    }
    return x;
  }();
  return r;
}

// Orders the handle's stream after everything the caller has enqueued on its
// own stream so far (inputs it produced there are complete before use).
void after_caller(gmres_ctx* h) {
  hip_check(hipEventRecord(h->evu, h->user));
  hip_check(hipStreamWaitEvent(h->stream, h->evu, 0));
}

bool valid_options(const gmres_options* o) {
  if (!o) return false;
  if (o->m < 1 || o->m > kMaxM) return false;
  if (!(o->tol >= 0.0)) return false;
  if (o->max_iters < 0) return false;
  if (o->ortho != GMRES_MGS && o->ortho != GMRES_CGSR) return false;
  if (o->precision < GMRES_FP64 || o->precision > GMRES_MIXED_LIMITED) return false;
  if (o->precond < GMRES_PRECOND_NONE || o->precond > GMRES_PRECOND_ILU0) return false;
  if (o->ilu_sweeps < 0 || o->ilu_sweeps > 4096) return false;
  if (o->arnoldi_a < GMRES_ARNOLDI_A_DEFAULT || o->arnoldi_a > GMRES_ARNOLDI_A_FP32) return false;
  if (o->precond_precision != GMRES_PRECOND_NATIVE && o->precond_precision != GMRES_PRECOND_FP32) return false;
  if (o->persistent_spmv < 0 || o->persistent_spmv > PV_COUNT) return false;
  if (o->precond_side != GMRES_PRECOND_RIGHT && o->precond_side != GMRES_PRECOND_LEFT) return false;
  if (o->spmv_format < GMRES_SPMV_AUTO || o->spmv_format > GMRES_SPMV_SELL16) return false;
  if (!(o->restart_improve >= 0.0)) return false;
  if (o->stall_cycles < 1) return false;
  if (o->batch_schedule < GMRES_SCHEDULE_AUTO || o->batch_schedule > GMRES_SCHEDULE_PERSISTENT) return false;
  if (o->spmv_block_nnz != 0 && (o->spmv_block_nnz < 64 || o->spmv_block_nnz > 8192 || o->spmv_block_nnz % 64))
    return false;
  if (o->a_storage != GMRES_A_COPY && o->a_storage != GMRES_A_SPLIT) return false;
  if (o->restart_repeat != 0 && o->restart_repeat != 1) return false;
  if (o->restart_on_stall != 0 && o->restart_on_stall != 1) return false;
  if (!(o->orth_restart >= 0.0) || !std::isfinite(o->orth_restart)) return false;
  if (o->orth_norm != GMRES_ORTH_SPECTRAL && o->orth_norm != GMRES_ORTH_FROBENIUS) return false;
  if (o->orth_restart > 0.0 && o->m > kMaxOrthM) return false;  // U and S of the monitor sit in LDS
  return true;
}

// Sizes the kernels can address, checked before any device work: row
// pointers and column indices are int32 (padded rows and non-zeros, with the
// 4-entry pad and a workgroup's worth of index slack, stay below 2^31), and
// the basis is read through buffer resources whose byte ranges and offsets
// are 32-bit, so (m + 1) padded columns of the basis, and the 4 columns of
// the half of the smallest register tile, must stay below 4 GiB.
int64_t basis_elem_bytes(int precision) {
  return precision == GMRES_FP64 ? 8 : (precision == GMRES_MIXED_BF16 || precision == GMRES_MIXED_FP16) ? 2 : 4;
}

bool sizes_ok(int32_t nsys, const int64_t* n, const int64_t* nnz, const gmres_options* o) {
  return plan::sizes_fit(nsys, n, nnz, o->m, basis_elem_bytes(o->precision));
}

// Conditions of the persistent schedule (one workgroup of 1024 threads per
// system, up to kMaxPR rows per thread, H in LDS, 32-bit buffer offsets).
bool persistent_ok(const gmres_options* o, const int64_t* n, int32_t nsys, int64_t nnz_total, int64_t ld) {
  if (o->precision != GMRES_MIXED_FP32 || o->precond != GMRES_PRECOND_NONE || o->ortho != GMRES_MGS) return false;
  if (o->a_storage != GMRES_A_COPY || o->orth_restart > 0.0) return false;
  if (o->arnoldi_a == GMRES_ARNOLDI_A_FP64) return false;
  if (o->m > kMaxPM) return false;
  for (int k = 0; k < nsys; ++k)
    if (n[k] > (int64_t)1024 * kMaxPR) return false;
  return nnz_total * 8 < ((int64_t)1 << 32) && ld * 8 < ((int64_t)1 << 32);
}

// Host staging for one download, freed when it goes out of scope: pinned
// memory (a faster copy), or ordinary memory when pinning that much fails.
struct PinnedBuffer {
  void* p = nullptr;
  bool pinned = false;
  std::vector<uint8_t> fallback;
  explicit PinnedBuffer(size_t bytes) {
    bytes = std::max<size_t>(bytes, 4);
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) == hipSuccess) {
      pinned = true;
      return;
    }
    (void)hipGetLastError();
    fallback.resize(bytes);  // std::bad_alloc here is reported as out of memory by the caller
    p = fallback.data();
  }
  ~PinnedBuffer() {
    if (pinned) (void)hipHostFree(p);
  }
  PinnedBuffer(const PinnedBuffer&) = delete;
  PinnedBuffer& operator=(const PinnedBuffer&) = delete;
};

// Runs f(i) for i in [0, count) on up to `workers` host threads (plain loop
// for small counts); an exception in any call fails the whole run.
template <typename F>
void parallel_for(int64_t count, int workers, F&& f) {
  if (count <= 1 || workers <= 1) {
    for (int64_t i = 0; i < count; ++i) f(i);
    return;
  }
  const int nt = (int)std::min<int64_t>(workers, count);
  std::vector<std::thread> th;
  std::vector<char> failed(nt, 0);
  for (int w = 0; w < nt; ++w)
    th.emplace_back([&, w] {
      try {
        for (int64_t i = w; i < count; i += nt) f(i);
      } catch (...) {
        failed[w] = 1;
      }
    });
  for (auto& t : th) t.join();
  for (char c : failed)
    if (c) throw Fail{GMRES_EINVAL};
}

int32_t* upload32(gmres_ctx* h, const std::vector<int32_t>& v) {
  int32_t* d = h->alloc<int32_t>(std::max<size_t>(v.size(), 1));
  if (!v.empty()) hip_check(hipMemcpy(d, v.data(), v.size() * 4, hipMemcpyHostToDevice));
  return d;
}

// Several small tables in one allocation and one copy; out[i] points at
// table i (each starts on a 64-entry boundary).
void upload_pack(gmres_ctx* h, std::initializer_list<const std::vector<int32_t>*> tables,
                 std::initializer_list<const int32_t**> out) {
  std::vector<size_t> off;
  size_t total = 0;
  for (const auto* v : tables) {
    off.push_back(total);
    total += (std::max<size_t>(v->size(), 1) + 63) / 64 * 64;
  }
  std::vector<int32_t> host(total, 0);
  size_t i = 0;
  for (const auto* v : tables) std::copy(v->begin(), v->end(), host.begin() + (ptrdiff_t)off[i++]);
  int32_t* d = h->alloc<int32_t>(total);
  hip_check(hipMemcpy(d, host.data(), total * 4, hipMemcpyHostToDevice));
  i = 0;
  for (const int32_t** o : out) *o = d + off[i++];
}

// Host part only (reads h->rp_host and h->sys): safe to run for several
// budgets at once.
void fill_row_blocks(const gmres_ctx* h, RowBlocks& t) {
  t.rb.clear();
  for (size_t k = 0; k < h->sys.size(); ++k) {
    const System& s = h->sys[k];
    const size_t before = t.rb.size();
    constexpr int64_t kChunk = 1 << 18;
    if (s.n <= kChunk) {
      plan::build_row_blocks(h->rp_host.data(), s.row0, s.row0 + s.n, t.budget, t.rb, &t.lanes);
    } else {
      // a large system in row chunks built in parallel (a block never spans
      // two chunks; any blocking gives the same sums)
      const int64_t nc = (s.n + kChunk - 1) / kChunk;
      std::vector<std::vector<int32_t>> rbs(nc), lns(nc);
      parallel_for(nc, 8, [&](int64_t c) {
        plan::build_row_blocks(h->rp_host.data(), s.row0 + c * kChunk,
                               s.row0 + std::min<int64_t>(s.n, (c + 1) * kChunk), t.budget, rbs[c], &lns[c]);
      });
      for (int64_t c = 0; c < nc; ++c) {
        t.rb.insert(t.rb.end(), rbs[c].begin(), rbs[c].end());
        t.lanes.insert(t.lanes.end(), lns[c].begin(), lns[c].end());
      }
    }
    t.rb0.push_back((int32_t)before);
    t.nrb.push_back((int32_t)(t.rb.size() - before));
    t.sys.insert(t.sys.end(), t.rb.size() - before, (int32_t)k);
  }
  // sentinel; no block starts in the padding.  The last block of each system
  // ends at the next block start (or ld): pad rows are empty, so that is exact.
  t.rb.push_back((int32_t)h->ld);
  t.p.resize(t.rb.size());
  for (size_t i = 0; i < t.rb.size(); ++i) t.p[i] = h->rp_host[t.rb[i]];
}

// Builds the tables of every budget in `budgets` not built yet, in parallel.
void prepare_row_blocks(gmres_ctx* h, const std::vector<int>& budgets) {
  std::vector<RowBlocks*> todo;
  for (int b : budgets) {
    bool have = false;
    for (const auto& t : h->rbt) have = have || t->budget == b;
    for (const RowBlocks* t : todo) have = have || t->budget == b;
    if (have) continue;
    h->rbt.push_back(std::make_unique<RowBlocks>());
    h->rbt.back()->budget = b;
    todo.push_back(h->rbt.back().get());
  }
  std::vector<std::thread> th;
  std::vector<char> failed(todo.size(), 0);
  for (size_t i = 1; i < todo.size(); ++i)
    th.emplace_back([h, &todo, &failed, i] {
      try {
        fill_row_blocks(h, *todo[i]);
      } catch (...) {
        failed[i] = 1;
      }
    });
  if (!todo.empty()) {
    try {
      fill_row_blocks(h, *todo[0]);
    } catch (...) {
      failed[0] = 1;
    }
  }
  for (auto& t : th) t.join();
  for (char f : failed)
    if (f) throw Fail{GMRES_ENOMEM};
}

const RowBlocks& row_blocks(gmres_ctx* h, int budget) {
  prepare_row_blocks(h, {budget});
  for (const auto& t : h->rbt)
    if (t->budget == budget) return *t;
  throw Fail{GMRES_EINVAL};
}

void set_row_blocks(gmres_ctx* h, int budget) {
  prepare_row_blocks(h, {budget});
  RowBlocks* t = nullptr;
  for (const auto& p : h->rbt)
    if (p->budget == budget) t = p.get();
  if (!t->d_rb)
    upload_pack(h, {&t->rb, &t->sys, &t->lanes, &t->rb0, &t->nrb, &t->p},
                {&t->d_rb, &t->d_sys, &t->d_lanes, &t->d_rb0, &t->d_nrb, &t->d_p});
  h->nrb = (int32_t)t->sys.size();
  h->a.rb = t->d_rb;
  h->a.rb_p = t->d_p;
  h->a.rb_sys = t->d_sys;
  h->a.rb_lanes = t->d_lanes;
  h->a.sys_rb0 = t->d_rb0;
  h->a.sys_nrb = t->d_nrb;
  h->a.nrb = h->nrb;
  h->a.spmv_budget = budget;
}

// Work split of the persistent basis passes for G workgroups: workgroup b
// owns tiles [b T / G, (b+1) T / G), cut at system boundaries into segments.
SegTab make_split(gmres_ctx* h, int G) {
  std::vector<int32_t> t0, nt;
  for (const System& s : h->sys) {
    t0.push_back(s.t0);
    nt.push_back(s.nt);
  }
  const plan::TileSplit sp = plan::split_tiles(t0.data(), nt.data(), (int32_t)h->sys.size(), G);
  SegTab sg{};
  sg.G = G;
  sg.nseg = (int32_t)sp.seg_t0.size();
  upload_pack(h, {&sp.bseg0, &sp.seg_t0, &sp.seg_nt, &sp.seg_sys, &sp.sys_sg0, &sp.sys_nsg},
              {&sg.bseg0, &sg.seg_t0, &sg.seg_nt, &sg.seg_sys, &sg.sys_sg0, &sg.sys_nsg});
  return sg;
}

int64_t vbytes(int prec) { return prec == P64 ? 8 : ((prec == P32 || prec == PL32) ? 4 : 2); }
int64_t wbytes(int prec) { return wide_w(prec) ? 8 : 4; }

// Enqueue one restart cycle: residual and stop test, m Arnoldi steps,
// back-solve and update.  Every kernel is gated on the device.
hipError_t enqueue_cycle(gmres_ctx* h, hipStream_t st) {
  const KArgs& a = h->a;
  const bool two = a.prec == PBF16 || a.prec == PF16;
  hipError_t e = launch_residual(a, st);
  if (e == hipSuccess) e = launch_left_start(a, st);  // left preconditioning: r = M^-1 z, beta = ||r||
  if (e == hipSuccess) e = launch_encode(a, 0, st);
  const bool ride = a.wsc_defer != 0;  // step j's finaliser launched with product j + 1
  for (int j = 0; j < a.m && e == hipSuccess; ++j) {
    if (a.precond != 0 && !a.left) e = launch_precond(a, j, st);
    if (e == hipSuccess && !(ride && j > 0)) e = launch_spmv_arnoldi(a, j, st);
    if (e == hipSuccess) e = launch_left_apply(a, st);  // w = M^-1 A v_j
    if (e != hipSuccess) break;
    if (h->opt.ortho == GMRES_CGSR) {
      e = launch_cgs_pass1(a, j, st);
      if (e == hipSuccess) e = launch_cgs_pass2(a, j, st);
      if (e == hipSuccess) e = launch_final_pass(a, j, st, !ride);
    } else {
      for (int i = 0; i <= j && e == hipSuccess; ++i) e = launch_mgs_dot(a, j, i, st);
      if (e == hipSuccess) e = launch_final_pass(a, j, st, !ride);
    }
    if (e == hipSuccess && ride) e = j + 1 < a.m ? launch_spmv_fin(a, j, st) : launch_finalize_final(a, j, st);
    if (e == hipSuccess && two && j + 1 <= a.m) e = launch_encode(a, j + 1, st);
    if (e == hipSuccess && a.orth_restart > 0.0) e = launch_orth_check(a, j, st);
  }
  if (e == hipSuccess) e = launch_backsolve(a, st);
  if (e == hipSuccess) e = launch_update(a, st);
  return e;
}

// In-solve kernel profile: the launches of one cycle in the order
// enqueue_cycle issues them, each group between two HIP events on the
// handle's stream.  A group records its family, its Arnoldi column (-1 for
// the launches of the cycle's start and end) and the algorithmic bytes it
// moves when it does work; whether it did work is only known once the cycle
// has ended (steps j >= k of a cycle that ended early are gated off on the
// device).
struct ProfRec {
  int kind;
  int j;        // Arnoldi column, -1: residual / encode of v_1, -2: back-solve / update
  double bytes;
  hipEvent_t e0, e1;
};

struct ProfPool {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  hipEvent_t get() {
    if (used == ev.size()) {
      hipEvent_t e = nullptr;
      // timing only: no system-scope release (its cache write-back and
      // invalidation would both inflate the bracketed time and evict what the
      // next kernel of the solve reuses)
      hip_check(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      ev.push_back(e);
    }
    return ev[used++];
  }
  ~ProfPool() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

void enqueue_cycle_profiled(gmres_ctx* h, hipStream_t st, ProfPool& pool, std::vector<ProfRec>& recs) {
  const KArgs& a = h->a;
  const bool two = a.prec == PBF16 || a.prec == PF16;
  const double n = (double)h->nrows, nnz = (double)h->nnz;
  const double sv = (double)vbytes(a.prec), sw = (double)wbytes(a.prec), sa = a.arn64 ? 8.0 : 4.0;
  const bool ride = a.wsc_defer != 0;
  auto timed = [&](int kind, int j, double bytes, auto&& launch) {
    ProfRec r{kind, j, bytes, pool.get(), pool.get()};
    hip_check(hipEventRecord(r.e0, st));
    hip_check(launch());
    hip_check(hipEventRecord(r.e1, st));
    recs.push_back(r);
  };
  timed(GMRES_PK_RESIDUAL, -1, nnz * 12.0 + 4.0 * (n + 1) + 16.0 * n + n * sw,
        [&] { return launch_residual(a, st, false); });
  timed(GMRES_PK_REDUCE, -1, 0.0, [&] { return launch_residual_finish(a, st); });
  if (a.left && a.precond != 0) timed(GMRES_PK_PRECOND, -1, 0.0, [&] { return launch_left_start(a, st); });
  timed(GMRES_PK_ENCODE, -1, n * sw + n * sv, [&] { return launch_encode(a, 0, st); });
  for (int j = 0; j < a.m; ++j) {
    const double ncol = j + 1;
    if (a.precond != 0 && !a.left) {
      const double sz = a.z64 ? 8.0 : 4.0, sd = a.pc64 ? 8.0 : 4.0;
      const double pb = a.precond == 1 ? n * sv + n * sd + n * sz
                      : a.precond == 2 ? nnz * 8.0 + 4.0 * (n + 1) + n * sv + n * sz : 0.0;
      timed(GMRES_PK_PRECOND, j, pb, [&] { return launch_precond(a, j, st); });
    }
    const double sx = a.precond != 0 && !a.left ? (a.z64 ? 8.0 : 4.0) : sv;
    const double spmv_bytes = nnz * (sa + 4.0) + 4.0 * (n + 1) + n * sx + n * sw;
    if (!(ride && j > 0)) timed(GMRES_PK_SPMV, j, spmv_bytes, [&] { return launch_spmv_arnoldi(a, j, st); });
    if (a.left && a.precond != 0) timed(GMRES_PK_PRECOND, j, 0.0, [&] { return launch_left_apply(a, st); });
    if (h->opt.ortho == GMRES_CGSR) {
      const double win = std::ceil(ncol / 64.0);
      timed(GMRES_PK_PASS1, j, ncol * n * sv + win * n * sw, [&] { return launch_cgs_pass1(a, j, st, false); });
      timed(GMRES_PK_REDUCE, j, 0.0, [&] { return launch_finalize_pass1(a, j, st); });
      const double p2 = ncol <= 64 ? ncol * n * sv + 2.0 * n * sw : 2.0 * ncol * n * sv + 3.0 * win * n * sw;
      timed(GMRES_PK_PASS2, j, p2, [&] { return launch_cgs_pass2(a, j, st, false); });
      timed(GMRES_PK_REDUCE, j, 0.0, [&] { return launch_finalize_pass2(a, j, st); });
    } else {
      for (int i = 0; i <= j; ++i)
        timed(GMRES_PK_MGS, j, i > 0 ? 2.0 * n * sv + 2.0 * n * sw : n * sv + n * sw,
              [&] { return launch_mgs_dot(a, j, i, st); });
    }
    timed(GMRES_PK_FINAL, j,
          (h->opt.ortho == GMRES_CGSR ? ncol * n * sv : n * sv) + n * sw + n * (two ? sw : sv),
          [&] { return launch_final_pass(a, j, st, false); });
    if (ride && j + 1 < a.m)  // this finaliser runs beside product j + 1 (counted as that product)
      timed(GMRES_PK_SPMV, j + 1, spmv_bytes, [&] { return launch_spmv_fin(a, j, st); });
    else
      timed(GMRES_PK_REDUCE, j, 0.0, [&] { return launch_finalize_final(a, j, st); });
    if (two && j + 1 <= a.m) timed(GMRES_PK_ENCODE, j, n * sw + n * sv, [&] { return launch_encode(a, j + 1, st); });
    if (a.orth_restart > 0.0) timed(GMRES_PK_ENCODE, j, 0.0, [&] { return launch_orth_check(a, j, st); });
  }
  timed(GMRES_PK_REDUCE, -2, 0.0, [&] { return launch_backsolve(a, st); });
  // the update reads k basis (or preconditioned) columns: its bytes are set once k is known
  timed(GMRES_PK_UPDATE, -2, 16.0 * n, [&] { return launch_update(a, st); });
}

void build_graph(gmres_ctx* h) {
  if (h->gexec) return;
  hipGraph_t g = nullptr;
  hip_check(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue_cycle(h, h->stream);
  hipError_t e2 = hipStreamEndCapture(h->stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    throw Fail{GMRES_EHIP};
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  hip_check(e);
  h->gexec = ex;
}

// Arnoldi SpMV of the persistent batch schedule, one kernel per variant: the
// one forced by persistent_spmv, else (autotune) the fastest of CSR8, CSR4
// and (when every system allows an ELL copy: n <= 65,536, rows of at most 255
// entries) ELL16 on a probe of the real kernel: the largest system of each
// size class (rows per thread), four Arnoldi steps from b = const, x = 0, one
// untimed launch, then one timed launch per variant between HIP events; else
// CSR8.
// Every variant gives bitwise the same results.
void setup_persistent_spmv(gmres_ctx* h, const gmres_options* opt) {
  KArgs& a = h->a;
  const int S = a.S;
  auto tier = [](int64_t n) { return plan::persistent_rows_per_thread(n, kMaxPR); };
  std::vector<int32_t> width(S, 0);
  std::vector<int64_t> off(S, 0);
  int64_t total = 0;
  bool all_ell = true;
  for (int k = 0; k < S; ++k) {
    const System& sy = h->sys[k];
    int wmax = 0;
    for (int64_t r = sy.row0; r < sy.row0 + sy.n; ++r)
      wmax = std::max(wmax, h->rp_host[r + 1] - h->rp_host[r]);
    if (sy.n <= 65536 && wmax <= 255 && wmax > 0) {
      width[k] = wmax;
      off[k] = total;
      total += (int64_t)wmax * sy.nt * kTile;
    } else {
      all_ell = false;
    }
  }
  const int forced = opt->persistent_spmv;  // 0: tuned, else 1 + PersistentSpmv
  const bool tune = forced == 0 && opt->autotune;
  const bool build_ell = all_ell && (forced == 1 + PV_ELL16 || tune);
  if (build_ell) {
    float* val = h->alloc<float>((size_t)total);
    uint16_t* col = h->alloc<uint16_t>((size_t)total);
    uint8_t* len = h->alloc<uint8_t>((size_t)h->ld);
    hip_check(hipMemsetAsync(len, 0, (size_t)h->ld, h->stream));
    for (int k = 0; k < S; ++k)
      hip_check(launch_build_ell(a, k, h->sys[k].row0, (int)h->sys[k].n, width[k], off[k], h->sys[k].nt * kTile,
                                 val, col, len, h->stream));
    a.ell_val = val;
    a.ell_col = col;
    a.ell_len = len;
    int64_t* d_off = h->alloc<int64_t>(S);
    hip_check(hipMemcpyAsync(d_off, off.data(), S * 8, hipMemcpyHostToDevice, h->stream));
    a.ell_off = d_off;
    a.ell_w = upload32(h, width);
  }
  // size classes and the probe systems (the largest of each class)
  std::vector<int> classes;
  for (int k = 0; k < S; ++k)
    if (std::find(classes.begin(), classes.end(), tier(h->sys[k].n)) == classes.end())
      classes.push_back(tier(h->sys[k].n));
  std::sort(classes.begin(), classes.end());
  h->tune.clear();
  std::vector<int32_t> probe;
  for (int c : classes) {
    gmres_tune_class tc{};
    tc.rows_per_thread = c;
    int big = -1;
    for (int k = 0; k < S; ++k)
      if (tier(h->sys[k].n) == c) {
        tc.systems += 1;
        if (big < 0 || h->sys[k].n > h->sys[big].n) big = k;
      }
    tc.largest_n = (int32_t)h->sys[big].n;
    tc.probe_system = big;
    probe.push_back(big);
    h->tune.push_back(tc);
  }
  for (double& t : h->tune_probe_us) t = -1.0;
  h->pv = PV_CSR8;
  if (forced > 0) {
    h->pv = forced - 1;
    if (h->pv == PV_ELL16 && !all_ell) h->pv = PV_CSR8;  // a system has no ELL copy
  } else if (tune) {
    // largest systems first, as in the solve's queue
    std::sort(probe.begin(), probe.end(), [&](int x, int y) { return h->sys[x].n > h->sys[y].n; });
    int32_t* d_probe = upload32(h, probe);
    KArgs t = a;
    t.S = (int32_t)probe.size();
    t.max_iters = std::min<int64_t>(a.m, 4);
    for (int k : probe) {  // b = a constant (a non-zero byte pattern), x = 0
      hip_check(hipMemsetAsync(a.b + h->sys[k].row0, 0x3f, (size_t)h->sys[k].n * 8, h->stream));
      hip_check(hipMemsetAsync(a.x + h->sys[k].row0, 0, (size_t)h->sys[k].n * 8, h->stream));
    }
    // one untimed launch brings the probe systems' data on chip for every variant alike
    hip_check(launch_batch_persistent(t, d_probe, h->counter, PV_CSR8, h->stream));
    float best = 1e30f;
    for (int v = 0; v < PV_COUNT; ++v) {
      if (v == PV_ELL16 && !all_ell) continue;
      for (int k : probe)
        hip_check(hipMemsetAsync(a.x + h->sys[k].row0, 0, (size_t)h->sys[k].n * 8, h->stream));
      hip_check(hipEventRecord(h->ev0, h->stream));
      hip_check(launch_batch_persistent(t, d_probe, h->counter, v, h->stream));
      hip_check(hipEventRecord(h->ev1, h->stream));
      hip_check(hipEventSynchronize(h->ev1));
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, h->ev0, h->ev1));
      h->tune_probe_us[v] = 1000.0 * ms;
      if (ms < best) {
        best = ms;
        h->pv = v;
      }
    }
    for (int k : probe) hip_check(hipMemsetAsync(a.x + h->sys[k].row0, 0, (size_t)h->sys[k].n * 8, h->stream));
    for (int k : probe) hip_check(hipMemsetAsync(a.b + h->sys[k].row0, 0, (size_t)h->sys[k].n * 8, h->stream));
    hip_check(launch_init_state(a, h->stream));
  }
  hip_check(hipStreamSynchronize(h->stream));
}

// Sliced ELL copy of the Arnoldi product's values, when every row has fewer
// than 2 kRowLanePer entries (each row's canonical sum is then its plain sum
// in storage order, which the sliced kernel keeps) and the padded copy fits
// 32-bit offsets; its columns as 16-bit offsets from the row when d16.
// Returns false (nothing built) otherwise.
bool build_sell(gmres_ctx* h, bool d16) {
  KArgs& a = h->a;
  if (a.asplit || h->persistent) return false;
  // slice widths on host threads, the offsets from them; the row lengths are
  // written on the device by the build kernel
  const int64_t nslice = h->ld / 64;
  std::vector<int32_t> wid(nslice), off;
  constexpr int64_t kPiece = 1 << 12;  // slices per task
  parallel_for((nslice + kPiece - 1) / kPiece, nslice >= 8 * kPiece ? 8 : 1, [&](int64_t p) {
    plan::sell_widths(h->rp_host.data(), p * kPiece, std::min<int64_t>(nslice, (p + 1) * kPiece), wid.data());
  });
  if (!plan::sell_offsets(wid.data(), nslice, off)) return false;
  const int64_t total = off.back();
  a.sell_off = upload32(h, off);
  uint8_t* d_len = h->alloc<uint8_t>((size_t)h->ld);
  a.sell_len = d_len;
  int32_t* col = d16 ? nullptr : h->alloc<int32_t>((size_t)total + 1);
  int16_t* dcol = d16 ? h->alloc<int16_t>((size_t)total + 1) : nullptr;
  void* val = a.arn64 ? (void*)h->alloc<double>((size_t)total + 1) : (void*)h->alloc<float>((size_t)total + 1);
  hip_check(launch_build_sell(a, a.arn64 ? (const void*)a.a64 : (const void*)a.a32, a.arn64 ? 0 : 1, val, col,
                              dcol, d_len, h->stream));
  a.sell_val = val;
  a.sell_col = col;
  a.sell_dcol = dcol;
  hip_check(hipStreamSynchronize(h->stream));  // the host tables are freed on return
  return true;
}

// Partial tables (two, for the passes that alternate) with a row for every
// segment of any persistent split and every row block of any budget built so
// far; reallocated (before any graph is captured) when a new budget needs
// more rows.
void ensure_partials(gmres_ctx* h) {
  KArgs& a = h->a;
  int64_t rows = h->ntile;
  for (const auto& t : h->rbt) rows = std::max<int64_t>(rows, (int64_t)t->sys.size());
  for (int k = 1; k <= kMaxOcc; ++k) rows = std::max<int64_t>(rows, a.seg[k - 1].nseg);
  if (rows <= h->part_rows) return;
  a.part = h->alloc<double>((size_t)rows * a.ps);
  a.part2 = h->alloc<double>((size_t)rows * a.ps);
  h->part_rows = rows;
}

// Times the Arnoldi SpMV for a few row-block budgets, each with and without
// the XCD block mapping (and the sliced ELL copy when there is one), and
// keeps the fastest (of the sliced ELL candidates only, when that format was
// asked for).  Every candidate runs between its own pair of events and the
// host waits once per round.  With a sliced copy the first round times it
// against the middle budget only; the other budgets are built and timed only
// if the copy is not clearly faster (kSellMargin).  The row blocks stay set
// to the fastest budget timed for the other products (residual,
// preconditioner) either way.
constexpr float kSellMargin = 0.85f;

void autotune_spmv(gmres_ctx* h, bool sell, bool sell_only) {
  struct Cand {
    int budget, remap, sell;
    float ms;
  };
  std::vector<Cand> cands;
  auto time_round = [&](size_t first) {
    for (size_t i = first; i < cands.size(); ++i) set_row_blocks(h, cands[i].budget);  // tables uploaded first
    while (h->tune_ev.size() < 2 * cands.size()) {
      hipEvent_t e;
      hip_check(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      h->tune_ev.push_back(e);
    }
    // exercise with a column of the zero-initialised basis; force the kernel on
    hip_check(launch_set_force(h->a, 1, h->stream));
    constexpr int reps = 3;
    for (size_t i = first; i < cands.size(); ++i) {
      const Cand& c = cands[i];
      set_row_blocks(h, c.budget);
      h->a.xcd_remap = c.remap;
      h->a.use_sell = c.sell;
      hip_check(launch_spmv_arnoldi(h->a, 0, h->stream));  // warm
      hip_check(hipEventRecord(h->tune_ev[2 * i], h->stream));
      for (int r = 0; r < reps; ++r) hip_check(launch_spmv_arnoldi(h->a, 0, h->stream));
      hip_check(hipEventRecord(h->tune_ev[2 * i + 1], h->stream));
    }
    hip_check(launch_set_force(h->a, 0, h->stream));
    hip_check(hipEventSynchronize(h->tune_ev[2 * cands.size() - 1]));
    for (size_t i = first; i < cands.size(); ++i)
      hip_check(hipEventElapsedTime(&cands[i].ms, h->tune_ev[2 * i], h->tune_ev[2 * i + 1]));
  };
  auto best_of = [&](int want_sell) {  // -1: any
    size_t bi = cands.size();
    for (size_t i = 0; i < cands.size(); ++i)
      if ((want_sell < 0 || cands[i].sell == want_sell) && (bi == cands.size() || cands[i].ms < cands[bi].ms))
        bi = i;
    return bi;
  };
  constexpr int kMid = 2048;
  for (int budget : kTuneBudgets)
    if (!sell || budget == kMid)
      for (int remap = 0; remap <= 1; ++remap) cands.push_back({budget, remap, 0, 0.f});
  if (sell)
    for (int remap = 0; remap <= 1; ++remap) cands.push_back({kMid, remap, 1, 0.f});
  time_round(0);
  if (sell && !(cands[best_of(1)].ms < kSellMargin * cands[best_of(0)].ms)) {
    // the copy does not win clearly: the other budgets too
    const size_t first = cands.size();
    std::vector<int> more;
    for (int budget : kTuneBudgets)
      if (budget != kMid) {
        more.push_back(budget);
        for (int remap = 0; remap <= 1; ++remap) cands.push_back({budget, remap, 0, 0.f});
      }
    prepare_row_blocks(h, more);
    ensure_partials(h);
    time_round(first);
  }
  const Cand& bc = cands[best_of(0)];
  const Cand& bi = cands[best_of(sell_only ? 1 : -1)];
  set_row_blocks(h, bc.budget);
  h->a.xcd_remap = bi.remap;
  h->a.use_sell = bi.sell;
  hip_check(hipStreamSynchronize(h->stream));
}

void setup_ilu0(gmres_ctx* h, int32_t sweeps);

void setup(gmres_ctx* h, int32_t nsys, const int64_t* n, const int64_t* nnz, const int32_t* const* rp,
           const int32_t* const* ci, const double* const* vals, const gmres_options* opt, void* user_stream) {
  h->opt = *opt;
  h->user = (hipStream_t)user_stream;
  hip_check(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
  // timing events (kernel harness, autotuners): no system-scope fence
  hip_check(hipEventCreateWithFlags(&h->ev0, hipEventDisableSystemFence));
  hip_check(hipEventCreateWithFlags(&h->ev1, hipEventDisableSystemFence));
  hip_check(hipEventCreateWithFlags(&h->evu, hipEventDisableTiming));
  after_caller(h);
  const int m = opt->m;
  const int prec = opt->precision;
  h->sys.resize(nsys);
  int64_t row = 0, nz = 0, tl = 0;
  for (int k = 0; k < nsys; ++k) {
    System& s = h->sys[k];
    s.n = n[k];
    s.nnz = nnz[k];
    s.row0 = row;
    s.nz0 = nz;
    s.t0 = (int32_t)tl;
    s.nt = (int32_t)((s.n + kTile - 1) / kTile);
    row += (int64_t)s.nt * kTile;
    nz += s.nnz;
    tl += s.nt;
    h->nrows += s.n;
  }
  if (row >= (int64_t)INT32_MAX || nz >= (int64_t)INT32_MAX) throw Fail{GMRES_EINVAL};  // (sizes_ok)
  h->ld = row;
  h->nnz = nz;
  h->ntile = (int32_t)tl;
  {
    const bool ok = persistent_ok(opt, n, nsys, nz, row);
    if (opt->batch_schedule == GMRES_SCHEDULE_PERSISTENT && !ok) throw Fail{GMRES_EINVAL};
    h->persistent = ok && (opt->batch_schedule == GMRES_SCHEDULE_PERSISTENT ||
                           (opt->batch_schedule == GMRES_SCHEDULE_AUTO && nsys >= 2));
  }

  // ---- global CSR (rows of padding are empty; columns shifted per system).
  // Each system's row pointer is downloaded into place in a pinned staging
  // buffer, checked (in parallel chunks, read-only), then shifted by its
  // first non-zero and padded (disjoint ranges) into the host copy.
  PinnedBuffer stage((size_t)(h->ld + 1 + nsys) * 4);
  int32_t* const st = static_cast<int32_t*>(stage.p);
  int32_t* const ends = st + h->ld + 1;  // each system's last row-pointer entry
  h->rp_host.resize(h->ld + 1);
  // every system's download is queued on the handle's stream, then one wait
  // (pinned staging: the copies run asynchronously).  Copies land in system
  // order; a system whose row count is a multiple of the tile shares its end
  // entry with the next system's first, so each end entry is also copied on
  // its own.
  for (int k = 0; k < nsys; ++k) {
    const System& s = h->sys[k];
    hip_check(hipMemcpyAsync(st + s.row0, rp[k], (s.n + 1) * 4, hipMemcpyDeviceToHost, h->stream));
    hip_check(hipMemcpyAsync(&ends[k], rp[k] + s.n, 4, hipMemcpyDeviceToHost, h->stream));
  }
  hip_check(hipStreamSynchronize(h->stream));
  for (int k = 0; k < nsys; ++k) {
    const System& s = h->sys[k];
    if (st[s.row0] != 0 || ends[k] != s.nnz) throw Fail{GMRES_EINVAL};
  }
  {
    constexpr int64_t kChunk = 1 << 18;
    struct Piece {
      int k;
      int64_t i0, i1;
    };
    std::vector<Piece> pieces;
    for (int k = 0; k < nsys; ++k)
      for (int64_t i0 = 0; i0 < h->sys[k].n; i0 += kChunk)
        pieces.push_back({k, i0, std::min<int64_t>(h->sys[k].n, i0 + kChunk)});
    const int workers = h->ld >= 4 * kChunk ? 8 : 1;
    parallel_for((int64_t)pieces.size(), workers, [&](int64_t p) {
      const System& s = h->sys[pieces[p].k];
      const int32_t* v = st + s.row0;
      // the entry after the last row may already hold the next system's first
      // entry (n a multiple of the tile): its own value, nnz, was checked above
      if (!plan::row_ptr_piece_ok(v, s.n, (int32_t)s.nnz, pieces[p].i0, pieces[p].i1)) throw Fail{GMRES_EINVAL};
    });
    parallel_for((int64_t)pieces.size(), workers, [&](int64_t p) {
      const System& s = h->sys[pieces[p].k];
      const int32_t* v = st + s.row0;
      int32_t* g = h->rp_host.data() + s.row0;
      const int32_t z0 = (int32_t)s.nz0;
      for (int64_t i = pieces[p].i0; i < pieces[p].i1; ++i) g[i] = v[i] + z0;
      if (pieces[p].i1 == s.n) {  // the system's last piece: its end and its padding rows
        const int64_t end = pieces[p].k + 1 < nsys ? h->sys[pieces[p].k + 1].row0 : h->ld + 1;
        for (int64_t i = s.row0 + s.n; i < end; ++i) h->rp_host[i] = (int32_t)(s.nz0 + s.nnz);
      }
    });
  }
  KArgs& a = h->a;
  a.S = nsys;
  a.m = m;
  a.ld = h->ld;
  a.ntile = h->ntile;
  {
    int dev = 0, ncu = 0;
    hip_check(hipGetDevice(&dev));
    hip_check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    a.ncu = std::max(1, ncu);
  }
  a.ps = m + 3;
  a.prec = prec;
  a.precond = opt->precond;
  a.ortho = opt->ortho;
  a.arn64 = opt->arnoldi_a == GMRES_ARNOLDI_A_FP64 || (opt->arnoldi_a == GMRES_ARNOLDI_A_DEFAULT && prec == P64) ? 1 : 0;
  a.xcd_remap = 1;
  // the device copy of the global row pointer is built on the device from
  // the caller's arrays (shifted by each system's first non-zero, padding
  // rows empty), the same values as the host copy
  int32_t* d_rp = h->alloc<int32_t>(h->ld + 1);
  for (int k = 0; k < nsys; ++k) {
    const System& s = h->sys[k];
    hip_check(launch_shift_cols(rp[k], d_rp + s.row0, s.n, (int32_t)s.nz0, h->stream));
    const int64_t end = k + 1 < nsys ? h->sys[k + 1].row0 : h->ld + 1;
    hip_check(hipMemsetD32Async((hipDeviceptr_t)(d_rp + s.row0 + s.n), (int)(s.nz0 + s.nnz),
                                (size_t)(end - s.row0 - s.n), h->stream));
  }
  // index and value arrays carry a zero pad of 4 entries (SpMV reads aligned groups of 4)
  int32_t* d_ci = h->alloc<int32_t>(h->nnz + 4);
  hip_check(hipMemsetAsync(d_ci + h->nnz, 0, 16, h->stream));
  for (int k = 0; k < nsys; ++k) {
    const System& s = h->sys[k];
    if (s.nnz == 0) continue;
    hip_check(launch_shift_cols(ci[k], d_ci + s.nz0, s.nnz, (int32_t)s.row0, h->stream));
  }
  a.rp = d_rp;
  a.ci = d_ci;
  if (opt->a_storage == GMRES_A_SPLIT) {
    // high and low 32-bit words of the float64 values, in two arrays
    uint32_t* d_hi = h->alloc<uint32_t>(h->nnz + 4);
    uint32_t* d_lo = h->alloc<uint32_t>(h->nnz + 4);
    hip_check(hipMemsetAsync(d_hi + h->nnz, 0, 16, h->stream));
    hip_check(hipMemsetAsync(d_lo + h->nnz, 0, 16, h->stream));
    for (int k = 0; k < nsys; ++k) {
      const System& s = h->sys[k];
      if (s.nnz == 0) continue;
      hip_check(launch_split_words(vals[k], d_hi + s.nz0, d_lo + s.nz0, s.nnz, h->stream));
    }
    a.ahi = d_hi;
    a.alo = d_lo;
    a.asplit = 1;
  } else {
    double* d_a64 = h->alloc<double>(h->nnz + 4);
    hip_check(hipMemsetAsync(d_a64 + h->nnz, 0, 32, h->stream));
    for (int k = 0; k < nsys; ++k) {
      const System& s = h->sys[k];
      if (s.nnz == 0) continue;
      hip_check(hipMemcpyAsync(d_a64 + s.nz0, vals[k], s.nnz * 8, hipMemcpyDeviceToDevice, h->stream));
    }
    a.a64 = d_a64;
    if (!a.arn64) {
      float* d_a32 = h->alloc<float>(h->nnz + 4);
      hip_check(launch_convert_f32(d_a64, d_a32, h->nnz + 4, h->stream));
      a.a32 = d_a32;
    }
  }
  // ---- per-system tables
  std::vector<int32_t> tile_sys(h->ntile), t0(nsys), nt(nsys), sn(nsys);
  std::vector<int64_t> row0(nsys);
  for (int k = 0; k < nsys; ++k) {
    const System& s = h->sys[k];
    for (int c = 0; c < s.nt; ++c) tile_sys[s.t0 + c] = k;
    t0[k] = s.t0;
    nt[k] = s.nt;
    sn[k] = (int32_t)s.n;
    row0[k] = s.row0;
  }
  auto up32 = [&](const std::vector<int32_t>& v) {
    int32_t* d = h->alloc<int32_t>(v.size());
    hip_check(hipMemcpy(d, v.data(), v.size() * 4, hipMemcpyHostToDevice));
    return d;
  };
  a.tile_sys = up32(tile_sys);
  a.sys_t0 = up32(t0);
  a.sys_nt = up32(nt);
  a.sys_n = up32(sn);
  {
    int64_t* d = h->alloc<int64_t>(nsys);
    hip_check(hipMemcpy(d, row0.data(), nsys * 8, hipMemcpyHostToDevice));
    a.sys_row0 = d;
  }
  // ---- workspace
  const int64_t M1 = m + 1, M2 = m + 2;
  // the basis is addressed through 32-bit buffer offsets (checked by sizes_ok)
  if (M1 * h->ld * vbytes(prec) >= (int64_t)1 << 32) throw Fail{GMRES_EINVAL};
  a.V = h->alloc<uint8_t>((size_t)(M1 * h->ld * vbytes(prec)));
  hip_check(hipMemsetAsync(a.V, 0, (size_t)(M1 * h->ld * vbytes(prec)), h->stream));
  a.w = h->alloc<uint8_t>((size_t)(h->ld * wbytes(prec)));
  hip_check(hipMemsetAsync(a.w, 0, (size_t)(h->ld * wbytes(prec)), h->stream));
  // the preconditioner's output Z is float64 in the float64 solver, and so is
  // its arithmetic unless a float32 preconditioner was asked for
  a.z64 = (opt->precond != GMRES_PRECOND_NONE && prec == P64) ? 1 : 0;
  a.pc64 = (a.z64 && opt->precond_precision == GMRES_PRECOND_NATIVE) ? 1 : 0;
  a.left = (opt->precond != GMRES_PRECOND_NONE && opt->precond_side == GMRES_PRECOND_LEFT) ? 1 : 0;
  if (opt->precond != GMRES_PRECOND_NONE && !a.left) {
    const size_t zb = a.z64 ? 8 : 4;
    a.Z = h->alloc<uint8_t>((size_t)(m * h->ld) * zb);
    hip_check(hipMemsetAsync(a.Z, 0, (size_t)(m * h->ld) * zb, h->stream));
  }
  if (a.left && opt->precond == GMRES_PRECOND_SPAI) {
    a.ptmp = h->alloc<uint8_t>((size_t)h->ld * wbytes(prec));
    hip_check(hipMemsetAsync(a.ptmp, 0, (size_t)h->ld * wbytes(prec), h->stream));
  }
  a.x = h->alloc<double>(h->ld);
  a.b = h->alloc<double>(h->ld);
  a.zres = h->alloc<double>(h->ld);  // padding rows stay zero
  hip_check(hipMemsetAsync(a.x, 0, h->ld * 8, h->stream));
  hip_check(hipMemsetAsync(a.b, 0, h->ld * 8, h->stream));
  hip_check(hipMemsetAsync(a.zres, 0, h->ld * 8, h->stream));
  a.st = h->alloc<SysState>(nsys);
  a.H = h->alloc<double>(nsys * M1 * m);
  a.Hbar = h->alloc<double>(nsys * M1 * m);
  hip_check(hipMemsetAsync(a.Hbar, 0, nsys * M1 * m * 8, h->stream));
  a.cs = h->alloc<double>(nsys * m);
  a.sn = h->alloc<double>(nsys * m);
  a.s = h->alloc<double>(nsys * M1);
  a.y = h->alloc<double>(nsys * m);
  a.sc = h->alloc<double>(nsys * M1);
  hip_check(hipMemsetAsync(a.sc, 0, nsys * M1 * 8, h->stream));
  a.hacc = h->alloc<double>(nsys * M2);
  if (opt->orth_restart > 0.0) {
    a.ou = h->alloc<double>((size_t)nsys * M1 * M1);
    a.os = h->alloc<double>((size_t)nsys * M1 * M1);
    a.ocol = h->alloc<double>((size_t)nsys * M1);
  }
  a.h1 = h->alloc<double>(nsys * M2);
  a.coef = h->alloc<double>(nsys * M2);
  a.ares = h->alloc<double>(nsys * M1);
  a.hist = h->alloc<double>((size_t)nsys * kHistCap);
  a.tol = opt->tol;
  a.restart_improve = opt->restart_improve;
  a.restart_repeat = opt->restart_repeat;
  a.restart_on_stall = opt->restart_on_stall;
  a.orth_restart = opt->orth_restart;
  a.orth_norm = opt->orth_norm;
  a.max_iters = opt->max_iters;
  a.stall_cycles = opt->stall_cycles;
  a.stall_win = std::max(1, (int)std::ceil(0.05 * m));
  hip_check(hipHostMalloc((void**)&h->st_host, sizeof(SysState) * nsys, hipHostMallocDefault));
  if (opt->precond == GMRES_PRECOND_JACOBI) {
    if (a.pc64) {
      double* d = h->alloc<double>(h->ld);
      hip_check(launch_jacobi_setup(a, nullptr, d, h->stream));
      a.dinv64 = d;
    } else {
      float* d = h->alloc<float>(h->ld);
      hip_check(launch_jacobi_setup(a, d, nullptr, h->stream));
      a.dinv = d;
    }
  }
  if (opt->precond == GMRES_PRECOND_SPAI) {
    float* d = h->alloc<float>(h->nnz + 4);
    hip_check(hipMemsetAsync(d, 0, (h->nnz + 4) * 4, h->stream));
    a.mval = d;
  }
  if (opt->precond == GMRES_PRECOND_ILU0) setup_ilu0(h, opt->ilu_sweeps);
  {
    int32_t* bad = h->alloc<int32_t>(1);
    hip_check(hipMemsetAsync(bad, 0, 4, h->stream));
    hip_check(launch_check_cols(a, bad, h->stream));
    int32_t hb = 0;
    hip_check(hipMemcpyAsync(&hb, bad, 4, hipMemcpyDeviceToHost, h->stream));
    hip_check(hipStreamSynchronize(h->stream));
    if (hb & 1) throw Fail{GMRES_EINVAL};
    h->near_cols = (hb & 2) == 0;
  }
  const bool tune = !h->persistent && opt->autotune && opt->spmv_block_nnz == 0;
  const int fixed_budget = opt->spmv_block_nnz > 0 ? opt->spmv_block_nnz : 2048;
  // the sliced ELL copy (16-bit column offsets when every column is near its
  // row, unless 32-bit columns were asked for): tuned against the row
  // blocks, or forced
  const int fmt = opt->spmv_format;
  const bool forced_sell = fmt == GMRES_SPMV_SELL || fmt == GMRES_SPMV_SELL16;
  const bool sell = !h->persistent && fmt != GMRES_SPMV_CSR && (tune || forced_sell) &&
                    build_sell(h, h->near_cols && fmt != GMRES_SPMV_SELL);
  // ---- SpMV row blocks, built in parallel on the host: the fixed budget;
  // for the autotuner every candidate budget, or only the middle one first
  // when a sliced copy competes (the others are built if it does not win)
  std::vector<int> budgets{fixed_budget};
  if (tune && !sell) budgets.assign(std::begin(kTuneBudgets), std::end(kTuneBudgets));
  prepare_row_blocks(h, budgets);
  for (int k = 1; k <= kMaxOcc; ++k) a.seg[k - 1] = make_split(h, (int)std::min<int64_t>((int64_t)k * a.ncu, h->ntile));
  ensure_partials(h);
  set_row_blocks(h, fixed_budget);
  hip_check(prepare_occupancy(prec));
  hip_check(launch_init_state(a, h->stream));
  if (h->persistent) {
    a.vsys = 1;
    std::vector<int32_t> ord(nsys);
    for (int k = 0; k < nsys; ++k) ord[k] = k;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return h->sys[x].n > h->sys[y].n; });
    h->order = h->alloc<int32_t>(nsys);
    hip_check(hipMemcpy(h->order, ord.data(), nsys * 4, hipMemcpyHostToDevice));
    h->counter = h->alloc<int32_t>(1);
    setup_persistent_spmv(h, opt);
  } else if (tune) {
    autotune_spmv(h, sell, sell && forced_sell);
  } else {
    a.use_sell = sell ? 1 : 0;
  }
  // the finaliser of each step rides on the next step's sliced product
  // (CGSR over register tiles or MGS, no preconditioner, a 4- or 8-byte
  // basis, no orthogonality monitor); the product then leaves v_j's scale
  // to the first passes that read w, which round the scaled w exactly as
  // the product would have (not so for a float64 product into a float32 w:
  // left out)
  a.wsc_defer = !h->persistent && a.use_sell && (opt->ortho == GMRES_MGS || m <= 64) &&
                opt->precond == GMRES_PRECOND_NONE && (prec == P32 || prec == P64 || prec == PL32) &&
                !(prec == P32 && a.arn64) && opt->orth_restart <= 0.0;
  h->xs = h->alloc<double>(h->ld);
  h->ys = h->alloc<double>(h->ld);
  hip_check(hipStreamSynchronize(h->stream));
}

int finish(gmres_ctx* h, gmres_result* res, int32_t nres, double seconds) {
  for (int k = 0; k < nres; ++k) {
    const SysState& S = h->st_host[k];
    gmres_result r{};
    r.status = S.status;
    r.iters = S.iters;
    r.restarts = S.restarts;
    r.rel_residual = S.rel;
    r.seconds = seconds;
    r.fallback_used = S.fallback_used;
    r.first_stall = S.first_stall;
    res[k] = r;
  }
  return GMRES_OK;
}

// The cycle loop shared by single and batch solves; b and x are already in
// the internal buffers.
void run_persistent(gmres_ctx* h) {
  hip_check(launch_batch_persistent(h->a, h->order, h->counter, h->pv, h->stream));
  hip_check(hipMemcpyAsync(h->st_host, h->a.st, sizeof(SysState) * h->a.S, hipMemcpyDeviceToHost, h->stream));
  hip_check(hipStreamSynchronize(h->stream));
}

void run_cycles(gmres_ctx* h) {
  if (h->persistent) {
    run_persistent(h);
    return;
  }
  KArgs& a = h->a;
  hip_check(launch_init_state(a, h->stream));
  hip_check(launch_bnorm(a, h->stream));
  hip_check(launch_left_bnorm(a, h->stream));
  if (h->opt.use_graph) build_graph(h);
  const int S = a.S;
  const int64_t cap = h->opt.max_iters / 1 + 8;
  for (int64_t cyc = 0; cyc <= cap; ++cyc) {
    if (h->opt.use_graph)
      hip_check(hipGraphLaunch(h->gexec, h->stream));
    else
      hip_check(enqueue_cycle(h, h->stream));
    hip_check(hipMemcpyAsync(h->st_host, a.st, sizeof(SysState) * S, hipMemcpyDeviceToHost, h->stream));
    hip_check(hipStreamSynchronize(h->stream));
    bool running = false;
    for (int k = 0; k < S && !running; ++k) running = h->st_host[k].status == RUNNING;
    if (!running) break;
  }
}

gmres_ctx* get(gmres_handle h) {
  if (!h || h->magic != kMagic) throw Fail{GMRES_EHANDLE};
  return h;
}

// ILU(0) at create time: diagonal positions and dependency levels of the
// lower triangle on the host, the factorisation level by level on the device
// (float64, on a copy of A's values), then float32 factors for the sweeps.
// Every row must store its diagonal entry.
void setup_ilu0(gmres_ctx* h, int32_t sweeps) {
  KArgs& a = h->a;
  const int64_t ld = h->ld;
  std::vector<int32_t> ci(h->nnz);
  if (h->nnz) hip_check(hipMemcpy(ci.data(), a.ci, h->nnz * 4, hipMemcpyDeviceToHost));
  // diagonal positions and dependency levels (lower triangle: factorisation
  // and L sweeps; upper triangle: U sweeps); every stored row needs its
  // diagonal and its columns in increasing order
  plan::IluPlan ip;
  if (plan::ilu_plan(h->rp_host.data(), ci.data(), ld, ip) != plan::ILU_OK) throw Fail{GMRES_EINVAL};
  const std::vector<int32_t>& count = ip.count;
  const int32_t depth_l = ip.depth_l, depth_u = ip.depth_u;
  int32_t* d_diag = upload32(h, ip.diag);
  int32_t* d_order = upload32(h, ip.order);
  a.diagpos = d_diag;
  double* lu = h->alloc<double>(h->nnz + 4);
  const double* vals = a.asplit ? nullptr : a.a64;
  if (a.asplit) {
    hip_check(launch_merge_words(a.ahi, a.alo, lu, h->nnz, h->stream));
  } else if (h->nnz) {
    hip_check(hipMemcpyAsync(lu, vals, h->nnz * 8, hipMemcpyDeviceToDevice, h->stream));
  }
  for (int l = 0; l < depth_l; ++l)
    hip_check(launch_ilu_factor(a, lu, d_order + count[l], count[l + 1] - count[l], h->stream));
  // the factors the sweeps read: float64 as factored, or their float32 rounding
  if (a.pc64) {
    double* dinv = h->alloc<double>(ld);
    hip_check(launch_ilu_finish(a, lu, nullptr, nullptr, dinv, h->stream));
    a.ilu64 = lu;
    a.iludinv64 = dinv;
  } else {
    float* lu32 = h->alloc<float>(h->nnz + 4);
    float* dinv = h->alloc<float>(ld);
    hip_check(launch_ilu_finish(a, lu, lu32, dinv, nullptr, h->stream));
    a.ilu32 = lu32;
    a.iludinv = dinv;
  }
  const size_t eb = a.pc64 ? 8 : 4;
  a.ilu_v = h->alloc<uint8_t>(ld * eb);
  for (int k = 0; k < 3; ++k) {
    a.ilu_b[k] = h->alloc<uint8_t>(ld * eb);
    hip_check(hipMemsetAsync(a.ilu_b[k], 0, ld * eb, h->stream));
  }
  hip_check(hipMemsetAsync(a.ilu_v, 0, ld * eb, h->stream));
  a.ilu_sl = sweeps > 0 ? sweeps : std::max(1, depth_l);
  a.ilu_su = sweeps > 0 ? sweeps : std::max(1, depth_u);
  hip_check(hipStreamSynchronize(h->stream));
}

// A's float64 values as one array (merged from the two word arrays in SPLIT
// storage); enqueued on the handle's stream.
const double* a64_values(gmres_ctx* h) {
  if (!h->a.asplit) return h->a.a64;
  if (!h->a64_merged) h->a64_merged = h->alloc<double>(h->nnz + 4);
  hip_check(launch_merge_words(h->a.ahi, h->a.alo, h->a64_merged, h->nnz, h->stream));
  return h->a64_merged;
}

}  // namespace

// ===================================================================== C ABI

extern "C" {

void gmres_default_options(gmres_options* o) {
  if (!o) return;
  o->m = 50;
  o->tol = 1e-10;
  o->max_iters = 100000;
  o->ortho = GMRES_CGSR;
  o->precision = GMRES_MIXED_FP32;
  o->precond = GMRES_PRECOND_NONE;
  o->restart_improve = 0.0;
  o->stall_cycles = 10;
  o->use_graph = 1;
  o->autotune = 1;
  o->batch_schedule = GMRES_SCHEDULE_AUTO;
  o->spmv_block_nnz = 0;
  o->a_storage = GMRES_A_COPY;
  o->restart_repeat = 0;
  o->restart_on_stall = 0;
  o->orth_restart = 0.0;
  o->orth_norm = GMRES_ORTH_SPECTRAL;
  o->ilu_sweeps = 4;
  o->arnoldi_a = GMRES_ARNOLDI_A_DEFAULT;
  o->precond_precision = GMRES_PRECOND_NATIVE;
  o->persistent_spmv = 0;
  o->precond_side = GMRES_PRECOND_RIGHT;
  o->spmv_format = GMRES_SPMV_AUTO;
}

const char* gmres_strerror(int code) {
  switch (code) {
    case GMRES_OK: return "ok";
    case GMRES_EINVAL: return "invalid argument";
    case GMRES_EHIP: return "HIP runtime error";
    case GMRES_ENOMEM: return "out of device memory";
    case GMRES_EHANDLE: return "invalid handle";
    case GMRES_ESTATE: return "operation not valid for this handle";
  }
  return "unknown error";
}

int gmres_batch_create(gmres_handle* out, int32_t nsys, const int64_t* n, const int64_t* nnz,
                       const int32_t* const* row_ptr, const int32_t* const* col_idx,
                       const double* const* vals, const gmres_options* opt, void* hip_stream) {
  if (!out || nsys < 1 || !n || !nnz || !row_ptr || !col_idx || !vals || !valid_options(opt))
    return GMRES_EINVAL;
  *out = nullptr;
  for (int k = 0; k < nsys; ++k) {
    if (n[k] <= 0 || nnz[k] < 0 || !row_ptr[k] || (nnz[k] > 0 && (!col_idx[k] || !vals[k])))
      return GMRES_EINVAL;
  }
  if (!sizes_ok(nsys, n, nnz, opt)) return GMRES_EINVAL;
  gmres_ctx* h = new (std::nothrow) gmres_ctx();
  if (!h) return GMRES_ENOMEM;
  try {
    setup(h, nsys, n, nnz, row_ptr, col_idx, vals, opt, hip_stream);
  } catch (const Fail& f) {
    delete h;
    (void)hipGetLastError();
    return f.code;
  } catch (const std::bad_alloc&) {
    delete h;
    return GMRES_ENOMEM;
  } catch (...) {  // e.g. host threads that could not be started: a resource failure
    delete h;
    (void)hipGetLastError();
    return GMRES_ENOMEM;
  }
  *out = h;
  return GMRES_OK;
}

int gmres_create(gmres_handle* out, int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                 const double* vals, const gmres_options* opt, void* hip_stream) {
  return gmres_batch_create(out, 1, &n, &nnz, &row_ptr, &col_idx, &vals, opt, hip_stream);
}

int gmres_set_preconditioner(gmres_handle hh, const float* spai_vals) {
  try {
    gmres_ctx* h = get(hh);
    if (h->opt.precond != GMRES_PRECOND_SPAI) return GMRES_ESTATE;
    if (!spai_vals) return GMRES_EINVAL;
    after_caller(h);
    hip_check(hipMemcpyAsync((void*)h->a.mval, spai_vals, h->nnz * 4, hipMemcpyDeviceToDevice, h->stream));
    hip_check(hipStreamSynchronize(h->stream));
    h->spai_set = true;
    return GMRES_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

int gmres_spai_infer(gmres_handle hh, const void* params, size_t param_bytes, float* m_out) {
  try {
    gmres_ctx* h = get(hh);
    if (h->opt.precond != GMRES_PRECOND_SPAI || h->sys.size() != 1) return GMRES_ESTATE;
    if (!params || param_bytes != (size_t)SPAI_NPARAMS * 2) return GMRES_EINVAL;
    after_caller(h);
    // the handle's stream is the network's caller stream: the network waits
    // for this handle's work and vice versa (every spai call drains its stream)
    if (!h->spai) {
      const int rc = spai_create(&h->spai, h->sys[0].n, h->nnz, h->a.rp, h->a.ci, 1, h->stream);
      if (rc != GMRES_OK) return rc;
    }
    int rc = spai_set_values(h->spai, a64_values(h));
    if (rc == GMRES_OK) rc = spai_forward(h->spai, (const uint16_t*)params, (float*)h->a.mval);
    if (rc != GMRES_OK) return rc;
    if (m_out) {
      hip_check(hipMemcpyAsync(m_out, h->a.mval, h->nnz * 4, hipMemcpyDeviceToDevice, h->stream));
      hip_check(hipStreamSynchronize(h->stream));
    }
    h->spai_set = true;
    return GMRES_OK;
  } catch (const Fail& f) {
    (void)hipGetLastError();
    return f.code;
  }
}

int gmres_spai_infer_with(gmres_handle hh, spai_handle net, const void* params, size_t param_bytes, float* m_out) {
  try {
    gmres_ctx* h = get(hh);
    if (h->opt.precond != GMRES_PRECOND_SPAI || h->sys.size() != 1) return GMRES_ESTATE;
    if (!net || !params || param_bytes != (size_t)SPAI_NPARAMS * 2) return GMRES_EINVAL;
    after_caller(h);
    hip_check(hipStreamSynchronize(h->stream));  // the network's calls are ordered after this handle's work
    int32_t same = 0;
    int rc = spai_same_pattern(net, h->sys[0].n, h->nnz, h->a.rp, h->a.ci, &same);
    if (rc != GMRES_OK) return rc;
    if (!same) return GMRES_ESTATE;
    rc = spai_set_values(net, a64_values(h));
    if (rc == GMRES_OK) rc = spai_forward(net, (const uint16_t*)params, (float*)h->a.mval);
    if (rc != GMRES_OK) return rc;
    if (m_out) {
      hip_check(hipMemcpyAsync(m_out, h->a.mval, h->nnz * 4, hipMemcpyDeviceToDevice, h->stream));
      hip_check(hipStreamSynchronize(h->stream));
    }
    h->spai_set = true;
    return GMRES_OK;
  } catch (const Fail& f) {
    (void)hipGetLastError();
    return f.code;
  }
}

int gmres_solve(gmres_handle hh, const double* b, double* x, gmres_result* res) {
  try {
    gmres_ctx* h = get(hh);
    if (h->a.S != 1) return GMRES_ESTATE;
    if (!b || !x) return GMRES_EINVAL;
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = h->sys[0].n;
    after_caller(h);
    hip_check(hipMemcpyAsync(h->a.b, b, n * 8, hipMemcpyDeviceToDevice, h->stream));
    hip_check(hipMemcpyAsync(h->a.x, x, n * 8, hipMemcpyDeviceToDevice, h->stream));
    run_cycles(h);
    hip_check(hipMemcpyAsync(x, h->a.x, n * 8, hipMemcpyDeviceToDevice, h->stream));
    hip_check(hipStreamSynchronize(h->stream));
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (res) finish(h, res, 1, sec);
    return GMRES_OK;
  } catch (const Fail& f) {
    (void)hipGetLastError();
    return f.code;
  }
}

int gmres_batch_solve(gmres_handle hh, const double* const* b, double* const* x, gmres_result* res) {
  try {
    gmres_ctx* h = get(hh);
    if (!b || !x) return GMRES_EINVAL;
    const int S = h->a.S;
    for (int k = 0; k < S; ++k)
      if (!b[k] || !x[k]) return GMRES_EINVAL;
    const auto t0 = std::chrono::steady_clock::now();
    after_caller(h);
    if (!h->bptrs) {
      h->bptrs = (const double**)h->alloc<void*>(S);
      h->xptrs = (double**)h->alloc<void*>(S);
    }
    hip_check(hipMemcpyAsync((void*)h->bptrs, b, S * sizeof(void*), hipMemcpyHostToDevice, h->stream));
    hip_check(hipMemcpyAsync((void*)h->xptrs, x, S * sizeof(void*), hipMemcpyHostToDevice, h->stream));
    int64_t maxn = 0;
    for (const System& s : h->sys) maxn = std::max(maxn, s.n);
    auto gather = [&]() -> hipError_t {
      hipError_t e = launch_gather(h->bptrs, h->a.b, h->a.sys_row0, h->a.sys_n, S, maxn, h->stream);
      if (e == hipSuccess)
        e = launch_gather((const double* const*)h->xptrs, h->a.x, h->a.sys_row0, h->a.sys_n, S, maxn, h->stream);
      return e;
    };
    auto scatter = [&]() { return launch_scatter(h->a.x, h->xptrs, h->a.sys_row0, h->a.sys_n, S, maxn, h->stream); };
    if (h->persistent && h->opt.use_graph) {
      // the whole batch solve is one graph: gather, the persistent kernel, scatter
      if (!h->pexec) {
        hipGraph_t g = nullptr;
        hip_check(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = gather();
        if (e == hipSuccess) e = launch_batch_persistent(h->a, h->order, h->counter, h->pv, h->stream);
        if (e == hipSuccess) e = scatter();
        const hipError_t e2 = hipStreamEndCapture(h->stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          throw Fail{GMRES_EHIP};
        }
        e = hipGraphInstantiate(&h->pexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        hip_check(e);
      }
      hip_check(hipGraphLaunch(h->pexec, h->stream));
      hip_check(hipMemcpyAsync(h->st_host, h->a.st, sizeof(SysState) * S, hipMemcpyDeviceToHost, h->stream));
    } else {
      hip_check(gather());
      run_cycles(h);
      hip_check(scatter());
    }
    hip_check(hipStreamSynchronize(h->stream));
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (res) finish(h, res, S, sec);
    return GMRES_OK;
  } catch (const Fail& f) {
    (void)hipGetLastError();
    return f.code;
  }
}

int gmres_destroy(gmres_handle hh) {
  if (!hh) return GMRES_OK;
  if (hh->magic != kMagic) return GMRES_EHANDLE;
  (void)hipStreamSynchronize(hh->stream);
  delete hh;
  return GMRES_OK;
}

int gmres_release_cached_memory(size_t* bytes) {
  const size_t n = cache_release_all();
  if (bytes) *bytes = n;
  return GMRES_OK;
}

int gmres_residual(gmres_handle hh, const double* b, const double* x, double* r, double* norm_out) {
  try {
    gmres_ctx* h = get(hh);
    if (!b || !x) return GMRES_EINVAL;
    if (h->sys.size() != 1) return GMRES_ESTATE;
    const int64_t n = h->sys[0].n;
    // kernels index padded global rows: stage b and x in padded buffers
    after_caller(h);
    hip_check(hipMemsetAsync(h->xs, 0, h->ld * 8, h->stream));
    hip_check(hipMemsetAsync(h->ys, 0, h->ld * 8, h->stream));
    hip_check(hipMemcpyAsync(h->ys, b, n * 8, hipMemcpyDeviceToDevice, h->stream));
    hip_check(hipMemcpyAsync(h->xs, x, n * 8, hipMemcpyDeviceToDevice, h->stream));
    hip_check(launch_residual_plain(h->a, h->ys, h->xs, h->ys, h->stream));
    std::vector<double> part((size_t)h->nrb * h->a.ps);
    hip_check(hipMemcpyAsync(part.data(), h->a.part, part.size() * 8, hipMemcpyDeviceToHost, h->stream));
    if (r) hip_check(hipMemcpyAsync(r, h->ys, n * 8, hipMemcpyDeviceToDevice, h->stream));
    hip_check(hipStreamSynchronize(h->stream));
    double sq = 0.0;
    for (int i = 0; i < h->nrb; ++i) sq += part[(size_t)i];
    if (norm_out) *norm_out = std::sqrt(sq);
    return GMRES_OK;
  } catch (const Fail& f) {
    (void)hipGetLastError();
    return f.code;
  }
}

namespace {

// ||v||_2 of a device vector, float64: fixed-grid partials, summed on the host in order.
double norm2(gmres_ctx* h, const double* v, int64_t n) {
  if (!h->sq_part) h->sq_part = h->alloc<double>(kSumsqBlocks);
  const int nblk = (int)std::max<int64_t>(1, std::min<int64_t>(kSumsqBlocks, (n + kBlock - 1) / kBlock));
  hip_check(launch_sumsq(v, n, h->sq_part, nblk, h->stream));
  std::vector<double> part(nblk);
  hip_check(hipMemcpyAsync(part.data(), h->sq_part, nblk * 8, hipMemcpyDeviceToHost, h->stream));
  hip_check(hipStreamSynchronize(h->stream));
  double sq = 0.0;
  for (double p : part) sq += p;
  return std::sqrt(sq);
}

// r = b - A x (float64) into h->ys for system 0, and its norm
double residual_into_ys(gmres_ctx* h, const double* b, const double* x) {
  const int64_t n = h->sys[0].n;
  after_caller(h);
  hip_check(hipMemsetAsync(h->xs, 0, h->ld * 8, h->stream));
  hip_check(hipMemsetAsync(h->ys, 0, h->ld * 8, h->stream));
  hip_check(hipMemcpyAsync(h->ys, b, n * 8, hipMemcpyDeviceToDevice, h->stream));
  hip_check(hipMemcpyAsync(h->xs, x, n * 8, hipMemcpyDeviceToDevice, h->stream));
  hip_check(launch_residual_plain(h->a, h->ys, h->xs, h->ys, h->stream));
  return norm2(h, h->ys, n);
}

}  // namespace

int gmres_backward_error(gmres_handle hh, const double* b, const double* x, double* eta, double* rel_residual) {
  try {
    gmres_ctx* h = get(hh);
    if (!b || !x) return GMRES_EINVAL;
    if (h->sys.size() != 1) return GMRES_ESTATE;
    const int64_t n = h->sys[0].n;
    const double rn = residual_into_ys(h, b, x);
    const double bn = norm2(h, b, n);
    const double xn = norm2(h, x, n);
    if (h->afro < 0.0) h->afro = norm2(h, a64_values(h), h->nnz);
    const double den = h->afro * xn + bn;
    if (eta) *eta = den > 0.0 ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
    if (rel_residual) *rel_residual = bn > 0.0 ? rn / bn : (rn > 0.0 ? INFINITY : 0.0);
    return GMRES_OK;
  } catch (const Fail& f) {
    (void)hipGetLastError();
    return f.code;
  }
}

int gmres_residual_unit(gmres_handle hh, const double* b, const double* x, float* r_out, double* norm_out) {
  try {
    gmres_ctx* h = get(hh);
    if (!b || !x || !r_out) return GMRES_EINVAL;
    if (h->sys.size() != 1) return GMRES_ESTATE;
    const int64_t n = h->sys[0].n;
    const double rn = residual_into_ys(h, b, x);
    if (norm_out) *norm_out = rn;
    if (!(rn > 0.0) || !std::isfinite(rn)) return GMRES_EINVAL;
    hip_check(launch_scale_f32(h->ys, n, 1.0 / rn, r_out, h->stream));
    hip_check(hipStreamSynchronize(h->stream));
    return GMRES_OK;
  } catch (const Fail& f) {
    (void)hipGetLastError();
    return f.code;
  }
}

namespace {

// z = M^-1 v through the ILU application of the Arnoldi loop, with elements
// of eb bytes (4: the float32 sweeps, 8: the float64 ones)
void ilu_apply_staged(gmres_ctx* h, const void* v, void* z, size_t eb) {
  const int64_t n = h->sys[0].n;
  KArgs t = h->a;
  t.z64 = eb == 8 ? 1 : 0;  // the output in the sweeps' own precision
  after_caller(h);
  hip_check(hipMemsetAsync(t.ilu_v, 0, h->ld * eb, h->stream));
  hip_check(hipMemcpyAsync(t.ilu_v, v, n * eb, hipMemcpyDeviceToDevice, h->stream));
  void* out = h->ys;  // ld doubles of staging
  hip_check(launch_set_force(t, 1, h->stream));
  hip_check(launch_ilu_apply(t, out, h->stream));
  hip_check(launch_set_force(t, 0, h->stream));
  hip_check(hipMemcpyAsync(z, out, n * eb, hipMemcpyDeviceToDevice, h->stream));
  hip_check(hipStreamSynchronize(h->stream));
}

}  // namespace

int gmres_precond_apply(gmres_handle hh, const float* v, float* z) {
  try {
    gmres_ctx* h = get(hh);
    if (!v || !z) return GMRES_EINVAL;
    if (h->opt.precond != GMRES_PRECOND_ILU0 || h->sys.size() != 1 || h->a.pc64) return GMRES_ESTATE;
    ilu_apply_staged(h, v, z, 4);
    return GMRES_OK;
  } catch (const Fail& f) {
    (void)hipGetLastError();
    return f.code;
  }
}

int gmres_precond_apply_f64(gmres_handle hh, const double* v, double* z) {
  try {
    gmres_ctx* h = get(hh);
    if (!v || !z) return GMRES_EINVAL;
    if (h->opt.precond != GMRES_PRECOND_ILU0 || h->sys.size() != 1 || !h->a.pc64) return GMRES_ESTATE;
    ilu_apply_staged(h, v, z, 8);
    return GMRES_OK;
  } catch (const Fail& f) {
    (void)hipGetLastError();
    return f.code;
  }
}

int gmres_spmv(gmres_handle hh, int32_t precision, const void* x, void* y) {
  try {
    gmres_ctx* h = get(hh);
    if (!x || !y) return GMRES_EINVAL;
    if (precision != GMRES_FP64 && precision != GMRES_MIXED_FP32 && precision != GMRES_MIXED_LIMITED)
      return GMRES_EINVAL;
    if (precision != GMRES_FP64 && !h->a.a32 && !h->a.asplit) return GMRES_ESTATE;
    if (h->sys.size() != 1) return GMRES_ESTATE;
    const int64_t n = h->sys[0].n;
    const size_t xb = precision == GMRES_FP64 ? 8 : 4, yb = precision == GMRES_MIXED_FP32 ? 4 : 8;
    // padded staging so that the kernel's global indexing is valid
    after_caller(h);
    hip_check(hipMemsetAsync(h->xs, 0, h->ld * 8, h->stream));
    hip_check(hipMemcpyAsync(h->xs, x, n * xb, hipMemcpyDeviceToDevice, h->stream));
    const int prec = precision == GMRES_FP64 ? P64 : (precision == GMRES_MIXED_FP32 ? P32 : PL32);
    hip_check(launch_spmv_plain(h->a, prec, h->xs, h->ys, h->stream));
    hip_check(hipMemcpyAsync(y, h->ys, n * yb, hipMemcpyDeviceToDevice, h->stream));
    hip_check(hipStreamSynchronize(h->stream));
    return GMRES_OK;
  } catch (const Fail& f) {
    (void)hipGetLastError();
    return f.code;
  }
}

int gmres_encode(int32_t precision, int64_t n, const float* w, double inv_h, void* out, double* scale_out,
                 void* hip_stream) {
  if (precision != GMRES_MIXED_BF16 && precision != GMRES_MIXED_FP16) return GMRES_EINVAL;
  if (n < 0 || (n > 0 && (!w || !out)) || !(inv_h > 0.0)) return GMRES_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  const int nblk = 256;
  float* part = nullptr;
  if (hipMalloc(&part, nblk * sizeof(float)) != hipSuccess) return GMRES_ENOMEM;
  int rc = GMRES_OK;
  std::vector<float> hp(nblk);
  if (launch_absmax(w, n, part, nblk, st) != hipSuccess ||
      hipMemcpyAsync(hp.data(), part, nblk * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    rc = GMRES_EHIP;
  } else {
    float mx = 0.0f;
    for (float v : hp) mx = std::max(mx, v);
    const double vmax = (double)mx * inv_h;
    int e = 0;
    if (vmax > 0.0 && std::isfinite(vmax)) {
      int p;
      const double f = std::frexp(vmax, &p);
      e = (precision == GMRES_MIXED_FP16 ? 15 : 0) - p + (f == 0.5 ? 1 : 0);
    }
    const float fac = (float)(std::ldexp(1.0, e) * inv_h);
    if (launch_encode_plain(precision, n, w, fac, out, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
      rc = GMRES_EHIP;
    if (scale_out) *scale_out = std::ldexp(1.0, -e);
  }
  (void)hipFree(part);
  return rc;
}

int gmres_last_cycle(gmres_handle hh, int32_t sys, int32_t* k_out, double* Hbar_out, double* V_out) {
  try {
    gmres_ctx* h = get(hh);
    if (sys < 0 || sys >= h->a.S) return GMRES_EINVAL;
    SysState S{};
    hip_check(hipMemcpy(&S, h->a.st + sys, sizeof(SysState), hipMemcpyDeviceToHost));
    if (k_out) *k_out = S.k;
    const int m = h->a.m;
    if (Hbar_out)
      hip_check(hipMemcpy(Hbar_out, h->a.Hbar + (size_t)sys * (m + 1) * m, (size_t)(m + 1) * m * 8,
                          hipMemcpyDeviceToHost));
    if (V_out) {
      const int64_t n = h->sys[sys].n;
      const int ncols = std::min(S.k + 1, m + 1);
      after_caller(h);
      for (int c = 0; c < ncols; ++c)
        hip_check(launch_decode_column(h->a, sys, c, V_out + (int64_t)c * n, h->stream));
      hip_check(hipStreamSynchronize(h->stream));
    }
    return GMRES_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

int gmres_history(gmres_handle hh, int32_t sys, double* out, int32_t cap, int32_t* count) {
  try {
    gmres_ctx* h = get(hh);
    if (sys < 0 || sys >= h->a.S || cap < 0 || (cap > 0 && !out)) return GMRES_EINVAL;
    SysState S{};
    hip_check(hipMemcpy(&S, h->a.st + sys, sizeof(SysState), hipMemcpyDeviceToHost));
    const int nrec = std::min(S.nhist, kHistCap);
    if (count) *count = nrec;
    const int ncopy = std::min(nrec, (int)cap);
    if (ncopy > 0)
      hip_check(hipMemcpy(out, h->a.hist + (size_t)sys * kHistCap, ncopy * 8, hipMemcpyDeviceToHost));
    return GMRES_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

int gmres_memory_bytes(gmres_handle hh, size_t* bytes) {
  try {
    gmres_ctx* h = get(hh);
    if (!bytes) return GMRES_EINVAL;
    *bytes = h->bytes;
    return GMRES_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

int gmres_solve_profiled(gmres_handle hh, const double* b, double* x, gmres_result* res,
                         gmres_kernel_profile* prof, gmres_kernel_profile* by_col) {
  try {
    gmres_ctx* h = get(hh);
    if (h->a.S != 1 || h->persistent) return GMRES_ESTATE;
    if (!b || !x || !prof) return GMRES_EINVAL;
    const int m = h->a.m;
    for (int k = 0; k < GMRES_PK_COUNT; ++k) prof[k] = gmres_kernel_profile{};
    if (by_col)
      for (int k = 0; k < GMRES_PK_COUNT * m; ++k) by_col[k] = gmres_kernel_profile{};
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = h->sys[0].n;
    KArgs& a = h->a;
    const double sv_upd = a.precond != 0 && !a.left ? (a.z64 ? 8.0 : 4.0) : (double)vbytes(a.prec);
    after_caller(h);
    hip_check(hipMemcpyAsync(a.b, b, n * 8, hipMemcpyDeviceToDevice, h->stream));
    hip_check(hipMemcpyAsync(a.x, x, n * 8, hipMemcpyDeviceToDevice, h->stream));
    hip_check(launch_init_state(a, h->stream));
    hip_check(launch_bnorm(a, h->stream));
    hip_check(launch_left_bnorm(a, h->stream));
    ProfPool pool;
    std::vector<ProfRec> recs;
    const int64_t cap = h->opt.max_iters + 8;
    int64_t restarts_before = 0;
    for (int64_t cyc = 0; cyc <= cap; ++cyc) {
      pool.used = 0;
      recs.clear();
      enqueue_cycle_profiled(h, h->stream, pool, recs);
      hip_check(hipMemcpyAsync(h->st_host, a.st, sizeof(SysState), hipMemcpyDeviceToHost, h->stream));
      hip_check(hipStreamSynchronize(h->stream));
      const SysState& S = h->st_host[0];
      // the cycle did work past its residual iff it applied a correction
      // (the residual may have ended the solve); then S.k is its step count
      const bool ran = S.restarts > restarts_before;
      const int k = ran ? S.k : 0;
      restarts_before = S.restarts;
      for (const ProfRec& r : recs) {
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, r.e0, r.e1));
        const bool active = r.j == -1 ? (r.kind != GMRES_PK_ENCODE || ran) : r.j == -2 ? ran : r.j < k;
        const double bytes =
            r.kind == GMRES_PK_UPDATE ? r.bytes + (double)S.kk * (double)h->nrows * sv_upd : r.bytes;
        auto add = [&](gmres_kernel_profile& p) {
          p.ms += ms;
          p.launches += 1;
          if (active) {
            p.ms_active += ms;
            p.active += 1;
            p.bytes += bytes;
          }
        };
        add(prof[r.kind]);
        if (by_col && r.j >= 0) add(by_col[(size_t)r.kind * m + r.j]);
      }
      if (S.status != RUNNING) break;
    }
    hip_check(hipMemcpyAsync(x, a.x, n * 8, hipMemcpyDeviceToDevice, h->stream));
    hip_check(hipStreamSynchronize(h->stream));
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (res) finish(h, res, 1, sec);
    return GMRES_OK;
  } catch (const Fail& f) {
    (void)hipGetLastError();
    return f.code;
  }
}

int gmres_launch_config(gmres_handle hh, int32_t family, int32_t j, int32_t* grid, int32_t* block,
                        int32_t* per_cu, int64_t* basis_align) {
  try {
    gmres_ctx* h = get(hh);
    if (family < 0 || family > GMRES_PK_UPDATE || j < 0 || j >= h->a.m) return GMRES_EINVAL;
    if (h->persistent) return GMRES_ESTATE;
    hip_check(launch_config(h->a, family, j, grid, block, per_cu));
    if (basis_align) {
      const uint64_t addr = (uint64_t)(uintptr_t)h->a.V;
      int64_t al = 1;
      while (al < (int64_t(1) << 21) && (addr & (uint64_t)al) == 0) al <<= 1;
      *basis_align = al;
    }
    return GMRES_OK;
  } catch (const Fail& f) {
    (void)hipGetLastError();
    return f.code;
  }
}

int gmres_spmv_config(gmres_handle hh, int32_t* format, int32_t* block_nnz, int32_t* xcd_remap,
                      int32_t* fin_merged) {
  try {
    gmres_ctx* h = get(hh);
    if (h->persistent) return GMRES_ESTATE;
    if (format)
      *format = !h->a.use_sell ? GMRES_SPMV_CSR : h->a.sell_dcol ? GMRES_SPMV_SELL16 : GMRES_SPMV_SELL;
    if (block_nnz) *block_nnz = h->a.spmv_budget;
    if (xcd_remap) *xcd_remap = h->a.xcd_remap;
    if (fin_merged) *fin_merged = h->a.wsc_defer;
    return GMRES_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

int gmres_batch_tuning(gmres_handle hh, int32_t* variant, double* probe_us, gmres_tune_class* out, int32_t cap,
                       int32_t* count) {
  try {
    gmres_ctx* h = get(hh);
    if (cap < 0 || (cap > 0 && !out)) return GMRES_EINVAL;
    if (!h->persistent) return GMRES_ESTATE;
    if (variant) *variant = h->pv;
    if (probe_us)
      for (int v = 0; v < 3; ++v) probe_us[v] = h->tune_probe_us[v];
    if (count) *count = (int32_t)h->tune.size();
    for (int32_t k = 0; k < cap && k < (int32_t)h->tune.size(); ++k) out[k] = h->tune[k];
    return GMRES_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

int gmres_time_kernel(gmres_handle hh, int32_t kernel, int32_t j, int32_t reps, double* avg_ms, double* bytes) {
  try {
    gmres_ctx* h = get(hh);
    const KArgs& a = h->a;
    if (j < 0 || j >= a.m || reps < 1 || !avg_ms) return GMRES_EINVAL;
    if (h->persistent) return GMRES_ESTATE;  // the harness times the device-wide kernels
    const int prec = a.prec;
    const double n = (double)h->nrows, nnz = (double)h->nnz;
    const double sv = (double)vbytes(prec), sw = (double)wbytes(prec), sa = a.arn64 ? 8.0 : 4.0;
    double bts = 0.0;
    auto run = [&]() -> hipError_t {
      switch (kernel) {
        case 0: return launch_spmv_arnoldi(a, j, h->stream);
        case 1: return launch_cgs_pass1(a, j, h->stream, false);
        case 2: return launch_cgs_pass2(a, j, h->stream, false);
        case 3: return launch_final_pass(a, j, h->stream, false);
        case 4: return launch_mgs_dot(a, j, j, h->stream);
        case 5: return launch_residual(a, h->stream, false);
        case 6: return launch_update(a, h->stream);
        case 7: return launch_finalize_pass2(a, j, h->stream);
      }
      return hipErrorInvalidValue;
    };
    switch (kernel) {
      case 0: bts = nnz * (sa + 4.0) + 4.0 * (n + 1) + n * sv + n * sw; break;
      case 1: bts = (j + 1) * n * sv + n * sw; break;
      case 2: bts = (j + 1) * n * sv + 2.0 * n * sw; break;
      case 3: bts = (j + 1) * n * sv + n * sw + n * (sv == 2 ? sw : sv); break;
      case 4: bts = (j > 0 ? 2.0 : 1.0) * n * sv + (j > 0 ? 2.0 : 1.0) * n * sw; break;
      case 5: bts = nnz * 12.0 + 4.0 * (n + 1) + 16.0 * n + n * sw; break;
      case 6: bts = (j + 1) * n * sv + 16.0 * n; break;
      case 7: bts = (double)h->a.seg[kMaxOcc - 1].nseg * (j + 1) * 8.0; break;
      default: return GMRES_EINVAL;
    }
    static const char* const kRange[] = {
        "timed:k_spmv(arnoldi)",        "timed:k_mdot(cgs pass 1)",   "timed:k_axpy_mdot(cgs pass 2)",
        "timed:k_final_tile(last pass)", "timed:k_mgs(mgs step)",      "timed:k_spmv(residual)",
        "timed:k_update",               "timed:k_fin_cols(pass 2)"};
    // the marker library is looked up (a dlopen on first use) before the
    // timed region starts, so the first timing does not include it
    const Roctx& rx = roctx();
    hip_check(launch_set_force(a, 1, h->stream));
    hip_check(run());
    hip_check(hipEventRecord(h->ev0, h->stream));
    if (rx.push) rx.push(kRange[kernel]);
    hipError_t err = hipSuccess;
    for (int r = 0; r < reps && err == hipSuccess; ++r) err = run();
    if (rx.pop) rx.pop();
    hip_check(err);
    hip_check(hipEventRecord(h->ev1, h->stream));
    hip_check(hipEventSynchronize(h->ev1));
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    hip_check(launch_set_force(a, 0, h->stream));
    hip_check(hipStreamSynchronize(h->stream));
    *avg_ms = (double)ms / reps;
    if (bytes) *bytes = bts;
    return GMRES_OK;
  } catch (const Fail& f) {
    (void)hipGetLastError();
    return f.code;
  }
}

}  // extern "C"
