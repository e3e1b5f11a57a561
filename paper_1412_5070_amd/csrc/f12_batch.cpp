// Batched evaluation: quartets of every (l_a l_b|l_c l_d) shape of one class,
// from one or several quartet lists, in one captured HIP graph.
//
// The graph forks into `nbranch` branches (HIP streams during capture).  Each
// branch owns a radial-derivative scratch and runs a chain of chunks; a chunk
// is a range of one shape group small enough for that scratch, evaluated by
// the radial-derivative launch followed by the contraction launch.  Chunks are
// dealt to branches longest-first onto the least-loaded branch (estimated
// cost: primitive quartets times the shape's per-primitive work), so shapes
// with few quartets run beside the large ones instead of after them.  The
// contraction launches are persistent where the tuner found it faster: a grid
// of G work-groups walks the chunk's cost-ordered quartets with stride G.
//
// Tuning: for every shape of the batch, the contraction of one sample chunk is
// timed (HIP events, best of two) for G in {one work-group per quartet, 256,
// 512, 1024, 2048, 4096}; the fastest is kept.  Results can be read from and
// written to a small text file ("L_ab L_cd i5 G" per line), so a second run
// skips the timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <memory>
#include <numeric>
#include <tuple>
#include <vector>

#include "../../include/f12int.h"
#include "f12_internal.h"
#include "f12_launch.h"

using namespace f12;

#include "f12_handles.h"

namespace {

struct Chunk {
  const f12_quartets *Q;
  int64_t qa, qe, p0, np;
  int la, lb, lc, ld, i5;
  double *out;
  int64_t out_base;
  double cost;
};

using ShapeKey = std::tuple<int, int, int>;  // (L_ab, L_cd, i5)

inline int hs3h(int L) { return L < 0 ? 0 : (L + 1) * (L + 2) * (L + 3) / 6; }

// Work per primitive quartet of a shape (the R integrals and the ket
// transform), the weight of the longest-first dealing.
double shape_cost(int la, int lb, int lc, int ld, int i5) {
  const int Lab = la + lb, Lcd = lc + ld, L = Lab + Lcd + (i5 ? 2 : 0);
  const double ncd = (double)ncart_host(lc) * ncart_host(ld);
  return 3.0 * hs3h(L + 1) + (i5 ? 4.0 : 1.0) * 2.0 * hs3h(Lab) * hs3h(Lcd) * ncd + 50.0 * (L + 1);
}

const int64_t kGrids[] = {0, 256, 512, 1024, 2048, 4096};

bool read_tune(const char *path, std::map<ShapeKey, int64_t> &t) {
  if (!path) return false;
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  int a, b, c;
  long long g;
  while (std::fscanf(f, "%d %d %d %lld", &a, &b, &c, &g) == 4) t[ShapeKey(a, b, c)] = g;
  std::fclose(f);
  return true;
}

bool write_tune(const char *path, const std::map<ShapeKey, int64_t> &t) {
  if (!path) return true;
  FILE *f = std::fopen(path, "w");
  if (!f) return false;
  for (const auto &kv : t)
    std::fprintf(f, "%d %d %d %lld\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                 (long long)kv.second);
  std::fclose(f);
  return true;
}

}  // namespace

struct f12_batch {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<std::unique_ptr<DevBuf<double>>> scratch;
  std::map<ShapeKey, int64_t> grid;
  int64_t nquartets = 0, nprim = 0, nchunks = 0;
  ~f12_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace {

int run_chunk(const Chunk &c, const f12_kernel *k, double *A, int64_t grid, hipStream_t st, bool aux = true) {
  const PairsDev bra = c.Q->bra->dev(), ket = c.Q->ket->dev();
  const int L = c.la + c.lb + c.lc + c.ld + (c.i5 ? 2 : 0);
  if (aux && launch_aux(k->d_desc.ptr, bra, ket, c.Q->d_qb.ptr, c.Q->d_qk.ptr, c.Q->d_qprim.ptr, c.qa,
                        c.qe - c.qa, c.p0, c.np, L, A, st, aux_variant(k->host_desc)) != 0)
    return F12_EDEVICE;
  if (launch_contract(bra, ket, c.Q->d_qb.ptr, c.Q->d_qk.ptr, c.Q->d_qoff.ptr, c.Q->d_qprim.ptr, c.qa,
                      c.qe - c.qa, c.p0, c.np, A, c.la, c.lb, c.lc, c.ld, c.i5, c.out, c.out_base, st, grid) != 0)
    return F12_EDEVICE;
  return F12_OK;
}

// Times the contraction of chunk c with each candidate grid; returns the best.
int tune_shape(const Chunk &c, const f12_kernel *k, double *A, hipStream_t st, int64_t *best) {
  if (run_chunk(c, k, A, 0, st) != F12_OK) return F12_EDEVICE;  // radial derivatives + warm-up
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return F12_EDEVICE;
  float tbest = 1e30f;
  *best = 0;
  int rc = F12_OK;
  for (int64_t g : kGrids) {
    if (g > 0 && g >= c.qe - c.qa) continue;  // not persistent for this chunk
    float tg = 1e30f;
    for (int rep = 0; rep < 2 && rc == F12_OK; ++rep) {
      if (hipEventRecord(e0, st) != hipSuccess) rc = F12_EDEVICE;
      if (rc == F12_OK) rc = run_chunk(c, k, A, g, st, false);
      if (rc == F12_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
        rc = F12_EDEVICE;
      float ms = 0.f;
      if (rc == F12_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = F12_EDEVICE;
      tg = std::min(tg, ms);
    }
    if (rc != F12_OK) break;
    if (tg < tbest) {
      tbest = tg;
      *best = g;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace

extern "C" int f12_batch_create(int32_t nlists, f12_quartets *const *lists, const int64_t *q_begin,
                                const int64_t *q_end, const f12_kernel *k, double *const *d_outs,
                                const int64_t *out_caps, int32_t nbranch, int32_t tune, const char *tune_path,
                                void *stream, f12_batch **out) {
  if (!out || nlists <= 0 || !lists || !q_begin || !q_end || !k || !d_outs || !out_caps) return F12_EINVAL;
  *out = nullptr;
  if (nbranch < 1 || nbranch > 16 || (tune != 0 && tune != 1)) return F12_EINVAL;
  // ---- validate and cut into chunks
  constexpr int64_t CHUNK_PRIMS = (int64_t)1 << 21;
  std::vector<Chunk> chunks;
  int64_t nq_tot = 0, np_tot = 0;
  for (int i = 0; i < nlists; ++i) {
    const f12_quartets *Q = lists[i];
    if (!Q || !d_outs[i] || q_begin[i] < 0 || q_end[i] > Q->nq || q_begin[i] > q_end[i]) return F12_EINVAL;
    if (Q->cls != k->cls) return F12_EINVAL;
    if (Q->qoff[q_end[i]] - Q->qoff[q_begin[i]] > out_caps[i]) return F12_EBUFSIZE;
    if (Q->max_qprim > CHUNK_PRIMS) return F12_EBUFSIZE;
    const int i5 = Q->cls == 5;
    const int64_t out_base = Q->qoff[q_begin[i]];
    nq_tot += q_end[i] - q_begin[i];
    np_tot += Q->qprim[q_end[i]] - Q->qprim[q_begin[i]];
    for (const Bin &b : Q->bins) {
      const int64_t lo = std::max(b.q0, q_begin[i]), hi = std::min(b.q0 + b.nq, q_end[i]);
      int64_t qa = lo;
      while (qa < hi) {
        const int64_t limit = Q->qprim[qa] + CHUNK_PRIMS;
        int64_t qe = std::upper_bound(Q->qprim.begin() + qa + 1, Q->qprim.begin() + hi + 1, limit) -
                     Q->qprim.begin() - 1;
        if (qe <= qa) qe = qa + 1;
        Chunk c;
        c.Q = Q;
        c.qa = qa;
        c.qe = qe;
        c.p0 = Q->qprim[qa];
        c.np = Q->qprim[qe] - c.p0;
        c.la = b.la;
        c.lb = b.lb;
        c.lc = b.lc;
        c.ld = b.ld;
        c.i5 = i5;
        c.out = d_outs[i];
        c.out_base = out_base;
        c.cost = c.np * shape_cost(b.la, b.lb, b.lc, b.ld, i5);
        chunks.push_back(c);
        qa = qe;
      }
    }
  }
  std::unique_ptr<f12_batch> B(new (std::nothrow) f12_batch);
  if (!B) return F12_ENOMEM;
  B->nquartets = nq_tot;
  B->nprim = np_tot;
  B->nchunks = (int64_t)chunks.size();
  for (int i = 0; i < nbranch; ++i) {
    B->scratch.emplace_back(new DevBuf<double>);
    if (!B->scratch.back()->alloc((size_t)CHUNK_PRIMS * (LTOT_MAX + 1))) return F12_ENOMEM;
  }
  hipStream_t st = (hipStream_t)stream;
  // ---- tuning: one sample chunk per shape (the largest chunk of the shape)
  std::map<ShapeKey, int64_t> known;
  read_tune(tune_path, known);
  std::map<ShapeKey, const Chunk *> sample;
  for (const Chunk &c : chunks) {
    const ShapeKey s(c.la + c.lb, c.lc + c.ld, c.i5);
    auto it = sample.find(s);
    if (it == sample.end() || c.qe - c.qa > it->second->qe - it->second->qa) sample[s] = &c;
  }
  bool learned = false;
  for (const auto &kv : sample) {
    auto it = known.find(kv.first);
    if (it != known.end()) {
      B->grid[kv.first] = it->second;
      continue;
    }
    int64_t g = 0;
    if (tune) {
      // the sample writes its own output range, which the graph rewrites
      int s = tune_shape(*kv.second, k, B->scratch[0]->ptr, st, &g);
      if (s) return s;
      known[kv.first] = g;
      learned = true;
    }
    B->grid[kv.first] = g;
  }
  if (learned && !write_tune(tune_path, known)) return F12_EINVAL;
  // kernel attributes are set outside the capture
  for (const auto &kv : sample)
    if (run_chunk(*kv.second, k, nullptr, -1, st, false) != F12_OK) return F12_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return F12_EDEVICE;
  // ---- longest-first dealing onto the least-loaded branch
  std::vector<int> order(chunks.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return chunks[x].cost > chunks[y].cost; });
  std::vector<std::vector<int>> branch(nbranch);
  std::vector<double> load(nbranch, 0.0);
  for (int ci : order) {
    const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    branch[b].push_back(ci);
    load[b] += chunks[ci].cost;
  }
  // ---- capture: fork, one chain per branch, join
  std::vector<hipStream_t> ss(nbranch, nullptr);
  std::vector<hipEvent_t> ev(nbranch + 1, nullptr);
  int rc = F12_OK;
  for (int i = 0; i < nbranch && rc == F12_OK; ++i)
    if (hipStreamCreateWithFlags(&ss[i], hipStreamNonBlocking) != hipSuccess) rc = F12_EDEVICE;
  for (int i = 0; i <= nbranch && rc == F12_OK; ++i)
    if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) rc = F12_EDEVICE;
  bool capturing = false;
  if (rc == F12_OK) {
    if (hipStreamBeginCapture(ss[0], hipStreamCaptureModeThreadLocal) != hipSuccess)
      rc = F12_EDEVICE;
    else
      capturing = true;
  }
  if (rc == F12_OK && hipEventRecord(ev[nbranch], ss[0]) != hipSuccess) rc = F12_EDEVICE;
  for (int i = 1; i < nbranch && rc == F12_OK; ++i)
    if (hipStreamWaitEvent(ss[i], ev[nbranch], 0) != hipSuccess) rc = F12_EDEVICE;
  for (int i = 0; i < nbranch && rc == F12_OK; ++i)
    for (int ci : branch[i]) {
      const Chunk &c = chunks[ci];
      rc = run_chunk(c, k, B->scratch[i]->ptr, B->grid[ShapeKey(c.la + c.lb, c.lc + c.ld, c.i5)], ss[i]);
      if (rc) break;
    }
  for (int i = 1; i < nbranch && rc == F12_OK; ++i)
    if (hipEventRecord(ev[i], ss[i]) != hipSuccess || hipStreamWaitEvent(ss[0], ev[i], 0) != hipSuccess)
      rc = F12_EDEVICE;
  if (capturing) {
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(ss[0], &g) != hipSuccess) rc = F12_EDEVICE;
    B->graph = g;
  }
  if (rc == F12_OK && hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0) != hipSuccess)
    rc = F12_EDEVICE;
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  for (hipStream_t s : ss)
    if (s) (void)hipStreamDestroy(s);
  if (rc) return rc;
  *out = B.release();
  return F12_OK;
}

extern "C" int f12_batch_launch(f12_batch *b, void *stream) {
  if (!b || !b->exec) return F12_EINVAL;
  return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? F12_OK : F12_EDEVICE;
}

extern "C" int f12_batch_info(const f12_batch *b, int64_t *n_quartets, int64_t *n_prim_quartets,
                              int64_t *n_chunks) {
  if (!b) return F12_EINVAL;
  if (n_quartets) *n_quartets = b->nquartets;
  if (n_prim_quartets) *n_prim_quartets = b->nprim;
  if (n_chunks) *n_chunks = b->nchunks;
  return F12_OK;
}

extern "C" int f12_batch_grid(const f12_batch *b, int32_t lab, int32_t lcd, int32_t i5, int64_t *grid) {
  if (!b || !grid) return F12_EINVAL;
  auto it = b->grid.find(ShapeKey(lab, lcd, i5));
  if (it == b->grid.end()) return F12_EINVAL;
  *grid = it->second;
  return F12_OK;
}

extern "C" void f12_batch_destroy(f12_batch *b) { delete b; }
