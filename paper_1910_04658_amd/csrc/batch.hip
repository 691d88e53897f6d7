// Batched execution of many independent BinSketch problems (Section 3
// compression, Algorithms 1-4 estimation, top-k per query), each with its
// own corpus, queries, map pi, dimension d and sketch width N.
//
// The whole batch is one HIP graph. Its nodes are grouped kernels, each
// covering every problem in the batch: a flag-clearing kernel, one launch
// that packs every map to 16-bit targets, ONE sketch launch for every corpus
// and query matrix, one LUT launch per distinct width,
// then the top-k stages (sample, sample select, threshold table, scan, select),
// one launch per stage and kernel variant (a variant is fixed by the width and
// the scan tile shape). The grids are persistent (at most what fits the
// device at once) and walk a table of virtual blocks that spans all
// problems, so a 1k-row corpus and a 200k-row corpus share every launch.
// bs_batch_run replays the graph with a single hipGraphLaunch.
//
// The tile shape of the scan (queries per lane, slab length through the scan
// grid size) is chosen per width by bs_batch_autotune, which times every
// candidate shape on the batch's own data and keeps the fastest.
#include <string.h>

#include <algorithm>
#include <memory>
#include <vector>

#include "bs_common.h"
#include "sketch_group.h"
#include "topk_group.h"

namespace bs {

void launch_lut(int32_t N, double* t64, float* t32, hipStream_t s);

namespace {

__global__ void batch_clear_kernel(int32_t* p, int32_t n) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Scan tile shapes the autotuner tries for a width (queries per lane x grid waves).
std::vector<TopkTune> candidate_tunes(int32_t N) {
  std::vector<TopkTune> c;
  const int W32 = N / 32;
  const bool pow2 = (W32 & (W32 - 1)) == 0;
  const int qpls[3] = {1, 2, 4};
  // the word-split scan (256 and 512 words) also tries a finer grid
  const int waves[4] = {4096, 8192, 16384, 32768};
  if (N % 256 == 0) {  // the matrix-core scan: only the grid size varies
    for (int w : waves) {
      TopkTune t;
      t.qpl = 1;
      t.waves = w;
      c.push_back(t);
    }
    return c;
  }
  const int n_waves = W32 >= 256 ? 4 : 3;
  for (int q : qpls) {
    if ((q == 2 && !(pow2 && W32 <= 32)) || (q == 4 && !(pow2 && W32 <= 16))) continue;
    for (int i = 0; i < n_waves; ++i) {
      const int w = waves[i];
      TopkTune t;
      t.qpl = q;
      t.waves = w;
      c.push_back(t);
    }
  }
  return c;
}

size_t item_ws_bytes(const bs_batch_item& it) {
  // the largest over every shape the autotuner may pick, so that one
  // workspace serves whichever shape wins
  size_t m = topk_item_workspace(it.n_queries, it.n_rows, it.N, it.k, TopkTune());
  for (const TopkTune& t : candidate_tunes(it.N)) {
    const size_t b = topk_item_workspace(it.n_queries, it.n_rows, it.N, it.k, t);
    m = b > m ? b : m;
  }
  return align256(m);
}

bs_status check_item(const bs_batch_item& it) {
  if (it.n_rows < 1 || it.n_rows > INT32_MAX || it.nnz < 0 || it.nnz > INT32_MAX || it.n_queries < 0 ||
      it.n_queries > INT32_MAX || it.q_nnz < 0 || it.q_nnz > INT32_MAX || it.d < 1 || it.d > INT32_MAX ||
      !valid_width(it.N) || it.k < 1 || it.k > BS_MAX_K || it.k > it.n_rows)
    return BS_ERR_ARG;
  if (!it.indptr || (!it.indices && it.nnz > 0) || !it.pi || !it.sketches || !it.popcounts) return BS_ERR_NULL;
  if (it.n_queries > 0 && (!it.q_indptr || (!it.q_indices && it.q_nnz > 0) || !it.q_sketches ||
                           !it.q_popcounts || !it.out_idx))
    return BS_ERR_NULL;
  return BS_OK;
}

struct Layout {
  std::vector<int32_t> widths;     // distinct N, ascending
  std::vector<size_t> lut_off;     // per distinct N
  std::vector<size_t> map_off;     // per item: its map as 16-bit targets
  size_t sketch_meta, topk_meta;   // offsets
  std::vector<size_t> item_off;    // per item top-k scratch
  size_t total;
};

Layout make_layout(const bs_batch_item* items, int32_t n) {
  Layout L;
  for (int32_t i = 0; i < n; ++i) L.widths.push_back(items[i].N);
  std::sort(L.widths.begin(), L.widths.end());
  L.widths.erase(std::unique(L.widths.begin(), L.widths.end()), L.widths.end());
  size_t o = 0;
  for (int32_t N : L.widths) {
    L.lut_off.push_back(o);
    o += align256((size_t)(N + 1) * 4);
  }
  for (int32_t i = 0; i < n; ++i) {
    L.map_off.push_back(o);
    o += align256((size_t)items[i].d * 2);
  }
  L.sketch_meta = o;
  o += align256(sketch_group_meta_bytes(2 * n));
  L.topk_meta = o;
  o += align256(topk_group_meta_bytes(n));
  for (int32_t i = 0; i < n; ++i) {
    L.item_off.push_back(o);
    o += item_ws_bytes(items[i]);
  }
  L.total = o;
  return L;
}

}  // namespace
}  // namespace bs

struct bs_batch {
  std::vector<bs_batch_item> items;
  int32_t measure = 0;
  char* ws = nullptr;
  int32_t* err = nullptr;
  bs::Layout L;
  std::vector<bs::TopkTune> tune_of_width;  // per distinct width
  std::vector<float> tuned_ms;             // per distinct width (-1: not timed)
  bs::SketchGroup* sk = nullptr;
  bs::TopkGroup* tk = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t launches = 0;
};

namespace bs {
namespace {

int width_index(const bs_batch* b, int32_t N) {
  for (size_t j = 0; j < b->L.widths.size(); ++j)
    if (b->L.widths[j] == N) return (int)j;
  return -1;
}

void drop_graph(bs_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

bs_status build_topk(bs_batch* b, const std::vector<TopkTune>& tunes_per_item, const std::vector<int32_t>& subset,
                     TopkGroup** out) {
  std::vector<TopkItem> its;
  std::vector<TopkTune> tn;
  std::vector<void*> wss;
  for (int32_t i : subset) {
    const bs_batch_item& x = b->items[i];
    if (x.n_queries == 0) continue;
    TopkItem t;
    t.Q = x.q_sketches;
    t.popQ = x.q_popcounts;
    t.nQ = x.n_queries;
    t.C = x.sketches;
    t.popC = x.popcounts;
    t.nC = x.n_rows;
    t.N = x.N;
    t.k = x.k;
    t.out_idx = x.out_idx;
    t.out_score = x.out_score;
    t.t32 = reinterpret_cast<const float*>(b->ws + b->L.lut_off[width_index(b, x.N)]);
    its.push_back(t);
    tn.push_back(tunes_per_item[i]);
    wss.push_back(b->ws + b->L.item_off[i]);
  }
  return topk_group_create(its.data(), tn.data(), (int32_t)its.size(), b->measure, wss.data(),
                           b->ws + b->L.topk_meta, topk_group_meta_bytes((int32_t)b->items.size()), true, out);
}

std::vector<TopkTune> item_tunes(const bs_batch* b) {
  std::vector<TopkTune> t(b->items.size());
  for (size_t i = 0; i < b->items.size(); ++i) t[i] = b->tune_of_width[width_index(b, b->items[i].N)];
  return t;
}

std::vector<int32_t> all_items(const bs_batch* b) {
  std::vector<int32_t> v(b->items.size());
  for (size_t i = 0; i < v.size(); ++i) v[i] = (int32_t)i;
  return v;
}

// Everything up to (not including) the top-k stages.
bs_status enqueue_front(const bs_batch* b, hipStream_t s) {
  const int32_t n = (int32_t)b->items.size();
  if (b->err && n > 0)
    hipLaunchKernelGGL(batch_clear_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, b->err, n);
  bs_status st = sketch_group_launch(b->sk, s);
  if (st != BS_OK) return st;
  for (size_t j = 0; j < b->L.widths.size(); ++j)
    launch_lut(b->L.widths[j], nullptr, reinterpret_cast<float*>(b->ws + b->L.lut_off[j]), s);
  return launch_status();
}

bs_status enqueue_all(const bs_batch* b, hipStream_t s) {
  bs_status st = enqueue_front(b, s);
  if (st != BS_OK) return st;
  return topk_group_launch(b->tk, s);
}

}  // namespace
}  // namespace bs

extern "C" size_t bs_batch_workspace_size(const bs_batch_item* items, int32_t n_items) {
  using namespace bs;
  if (n_items < 1 || !items) return 0;
  for (int32_t i = 0; i < n_items; ++i)
    if (check_item(items[i]) != BS_OK) return 0;
  return make_layout(items, n_items).total;
}

extern "C" bs_status bs_batch_create(const bs_batch_item* items, int32_t n_items, int32_t measure,
                                     const bs_batch_shape* shapes, int32_t n_shapes, void* workspace,
                                     size_t workspace_bytes, int32_t* err_flags, bs_batch** out) {
  using namespace bs;
  if (!out) return BS_ERR_NULL;
  *out = nullptr;
  if (n_items < 1 || measure < 0 || measure > 3 || n_shapes < 0) return BS_ERR_ARG;
  if (!items || (n_shapes > 0 && !shapes)) return BS_ERR_NULL;
  for (int32_t i = 0; i < n_items; ++i) {
    const bs_status st = check_item(items[i]);
    if (st != BS_OK) return st;
  }
  const Layout L = make_layout(items, n_items);
  if (!workspace || workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return BS_ERR_WORKSPACE;
  bs_status st = check_device();
  if (st != BS_OK) return st;
  std::unique_ptr<bs_batch> b(new bs_batch);
  b->items.assign(items, items + n_items);
  b->measure = measure;
  b->ws = static_cast<char*>(workspace);
  b->err = err_flags;
  b->L = L;
  b->tune_of_width.assign(L.widths.size(), TopkTune());
  b->tuned_ms.assign(L.widths.size(), -1.0f);
  for (int32_t j = 0; j < n_shapes; ++j) {
    const int w = width_index(b.get(), shapes[j].N);
    if (w < 0) continue;
    b->tune_of_width[w].qpl = shapes[j].qpl;
    b->tune_of_width[w].waves = shapes[j].waves;
    b->tuned_ms[w] = shapes[j].ms;
  }
  // sketch items: every corpus, then every query matrix (one error flag word per problem)
  std::vector<SketchItem> sk;
  for (int32_t i = 0; i < n_items; ++i) {
    const bs_batch_item& x = items[i];
    sk.push_back(SketchItem{x.indptr, x.indices, x.n_rows, x.nnz, x.pi, x.d, x.N, x.sketches, x.popcounts,
                            err_flags ? err_flags + i : nullptr,
                            reinterpret_cast<uint16_t*>(b->ws + L.map_off[i])});
  }
  for (int32_t i = 0; i < n_items; ++i) {
    const bs_batch_item& x = items[i];
    if (x.n_queries == 0) continue;
    sk.push_back(SketchItem{x.q_indptr, x.q_indices, x.n_queries, x.q_nnz, x.pi, x.d, x.N, x.q_sketches,
                            x.q_popcounts, err_flags ? err_flags + i : nullptr,
                            reinterpret_cast<uint16_t*>(b->ws + L.map_off[i])});
  }
  st = sketch_group_create(sk.data(), (int32_t)sk.size(), b->ws + L.sketch_meta, sketch_group_meta_bytes(2 * n_items),
                           true, &b->sk);
  if (st != BS_OK) return st;
  st = build_topk(b.get(), item_tunes(b.get()), all_items(b.get()), &b->tk);
  if (st != BS_OK) {
    sketch_group_destroy(b->sk);
    return st;
  }
  *out = b.release();
  return BS_OK;
}

extern "C" bs_status bs_batch_autotune(bs_batch* b, int32_t reps, void* stream) {
  using namespace bs;
  if (!b) return BS_ERR_NULL;
  if (reps < 1) return BS_ERR_ARG;
  hipStream_t s = as_stream(stream);
  drop_graph(b);
  // sketches and tables once, then every candidate shape per width on that width's problems
  bs_status st = enqueue_front(b, s);
  if (st != BS_OK) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return BS_ERR_HIP;
  std::vector<TopkTune> per_item = item_tunes(b);
  for (size_t w = 0; w < b->L.widths.size(); ++w) {
    std::vector<int32_t> sub;
    for (size_t i = 0; i < b->items.size(); ++i)
      if (b->items[i].N == b->L.widths[w] && b->items[i].n_queries > 0) sub.push_back((int32_t)i);
    if (sub.empty()) continue;
    float best = -1.0f;
    TopkTune best_t = b->tune_of_width[w];
    for (const TopkTune& t : candidate_tunes(b->L.widths[w])) {
      for (int32_t i : sub) per_item[i] = t;
      TopkGroup* g = nullptr;
      st = build_topk(b, per_item, sub, &g);
      if (st != BS_OK) break;
      st = topk_group_launch(g, s);  // warm-up
      if (st == BS_OK) (void)hipEventRecord(e0, s);
      for (int32_t r = 0; r < reps && st == BS_OK; ++r) st = topk_group_launch(g, s);
      if (st == BS_OK) (void)hipEventRecord(e1, s);
      float ms = 0.0f;
      if (st == BS_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = BS_ERR_HIP;
      topk_group_destroy(g);
      if (st != BS_OK) break;
      ms /= (float)reps;
      if (best < 0.0f || ms < best) {
        best = ms;
        best_t = t;
      }
    }
    if (st != BS_OK) break;
    b->tune_of_width[w] = best_t;
    b->tuned_ms[w] = best;
    for (int32_t i : sub) per_item[i] = best_t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != BS_OK) return st;
  // the tuning runs reused the group tables: rebuild the full plan
  topk_group_destroy(b->tk);
  b->tk = nullptr;
  return build_topk(b, item_tunes(b), all_items(b), &b->tk);
}

extern "C" bs_status bs_batch_run(bs_batch* b, void* stream) {
  using namespace bs;
  if (!b || !b->tk || !b->sk) return BS_ERR_NULL;
  hipStream_t s = as_stream(stream);
  if (!b->exec) {
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return BS_ERR_HIP;
    bs_status st = BS_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = BS_ERR_HIP;
    if (st == BS_OK) {
      st = enqueue_all(b, cs);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(cs, &g);
      if (st == BS_OK && e != hipSuccess) st = BS_ERR_HIP;
      if (st == BS_OK) {
        size_t nodes = 0;
        (void)hipGraphGetNodes(g, nullptr, &nodes);
        b->launches = (int32_t)nodes;
        if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
          st = BS_ERR_HIP;
          b->exec = nullptr;
        }
        b->graph = g;
      } else if (g) {
        (void)hipGraphDestroy(g);
      }
    }
    (void)hipStreamDestroy(cs);
    if (st != BS_OK) {
      drop_graph(b);
      return st;
    }
  }
  ScopedTiming timing("batch_graph", s);
  return hipGraphLaunch(b->exec, s) == hipSuccess ? BS_OK : BS_ERR_HIP;
}

extern "C" bs_status bs_batch_run_eager(bs_batch* b, void* stream) {
  using namespace bs;
  if (!b || !b->tk || !b->sk) return BS_ERR_NULL;
  return enqueue_all(b, as_stream(stream));
}

extern "C" int32_t bs_batch_shapes(const bs_batch* b, bs_batch_shape* out, int32_t cap) {
  if (!b) return 0;
  const int32_t n = (int32_t)b->L.widths.size();
  for (int32_t j = 0; j < n && j < cap && out; ++j) {
    out[j].N = b->L.widths[j];
    out[j].qpl = b->tune_of_width[j].qpl;
    out[j].waves = b->tune_of_width[j].waves;
    out[j].ms = b->tuned_ms[j];
  }
  return n;
}

extern "C" int32_t bs_batch_graph_nodes(const bs_batch* b) { return b ? b->launches : 0; }

extern "C" void bs_batch_destroy(bs_batch* b) {
  if (!b) return;
  bs::drop_graph(b);
  bs::sketch_group_destroy(b->sk);
  bs::topk_group_destroy(b->tk);
  delete b;
}
