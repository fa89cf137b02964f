// window.cpp -- the mapping window: every view's forward and backward bound
// once, tuned once, captured in one HIP graph and replayed per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "runtime.h"

using namespace vpgs;

struct vpgs_window {
  vpgs_ctx* ctx = nullptr;
  vpgs_saved* sv = nullptr;  // buffers owned by the window
  std::vector<vpgs_gaussians> sets;
  std::vector<int32_t> view_set;
  std::vector<vpgs_camera> cams;
  std::vector<vpgs_images> out;
  std::vector<vpgs_image_grads> grad_out;
  std::vector<vpgs_gauss_grads> grads;
  float* d_pose = nullptr;
  std::vector<float*> accum;  // expansion accumulators per set (empty: none bound)
  vpgs_densify_accum acc_desc{};
  vpgs_window_opts cfg{};
  bool tables_dirty = false;  // the tables need a rebuild before the next run
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};       // forward, backward
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  // Sticky pair-list overflow flag in mapped pinned host memory, set by the
  // last kernel of every forward run: a later run reports VPGS_ECAPACITY
  // without synchronising.
  uint32_t* h_overflow = nullptr;
  uint32_t* d_overflow = nullptr;  // the device address of the same word
  bool tuned_from_cache = false;
};

namespace {

const int kShapes[][2] = {{16, 16}, {16, 8}, {8, 8}, {32, 8}};

// Raises the window's sticky host flag when the forward's pair list
// overflowed (the pairs the scan asked for exceed the capacity).
__global__ void publish_overflow_kernel(const Counters* cnt, uint32_t capacity, uint32_t* flag) {
  if (threadIdx.x == 0 && (cnt->overflow || cnt->pairs > capacity)) *(volatile uint32_t*)flag = 1u;
}

const vpgs_densify_accum* accum_of(vpgs_window* w) {
  if (w->accum.empty()) return nullptr;
  w->acc_desc.accum = w->accum.data();
  return &w->acc_desc;
}

int configure(vpgs_window* w, int tw, int th, int nb) {
  vpgs_ctx* ctx = w->ctx;
  vpgs_saved* sv = w->sv;
  int rc = build_tables(ctx, *sv->h_tab, (int)w->sets.size(), w->sets.data(), (int)w->view_set.size(),
                        w->view_set.data(), w->cams.data(), w->out.data(), tw, th);
  if (rc) return rc;
  rc = bind_backward(ctx, *sv->h_tab, w->grad_out.data(), w->grads.data());
  if (!rc) rc = bind_accum(ctx, *sv->h_tab, accum_of(w));
  if (rc) return rc;
  sv->tile_w = tw;
  sv->tile_h = th;
  sv->lds_batch = nb;
  return prepare_front(ctx, sv);
}

// The window's launch sequence without a graph: part 1 = forward, 2 = backward.
int enqueue_part(vpgs_window* w, int part, hipStream_t st) {
  int rc;
  if (part == 1) {
    if ((rc = enqueue_front(w->ctx, w->sv, st)) || (rc = enqueue_back(w->ctx, w->sv, st))) return rc;
    if (w->d_overflow) {
      vpgs_ctx* ctx = w->ctx;
      hipLaunchKernelGGL(publish_overflow_kernel, dim3(1), dim3(64), 0, st,
                         static_cast<const Counters*>(w->sv->counters.p), w->sv->capacity, w->d_overflow);
      HIP_TRY(hipGetLastError());
    }
    return VPGS_OK;
  }
  return enqueue_backward(w->ctx, w->sv, w->d_pose, st);
}

int enqueue_all(vpgs_window* w, hipStream_t st) {
  int rc = enqueue_part(w, 1, st);
  return rc ? rc : enqueue_part(w, 2, st);
}

// Sizes the pair list for the current tile shape: one eager front half and a
// read of the pair count.
int size_pairs(vpgs_window* w, hipStream_t st, int64_t fixed) {
  vpgs_ctx* ctx = w->ctx;
  int rc = upload_tables(ctx, w->sv, st);
  if (rc) return rc;
  uint32_t cap = 0;
  if (fixed > 0) {
    cap = (uint32_t)fixed;
  } else {
    if ((rc = enqueue_front(ctx, w->sv, st)) || (rc = read_pair_count(ctx, w->sv, st, &cap))) return rc;
    cap = (uint32_t)std::min<uint64_t>((uint64_t)cap + cap / 4 + 4096, 0x7fffffffull);
  }
  if ((rc = ensure_pairs(ctx, w->sv, cap)) || (rc = ensure_backward(ctx, w->sv, st))) return rc;
  return VPGS_OK;
}

int time_config(vpgs_window* w, hipStream_t st, int reps, float* ms) {
  vpgs_ctx* ctx = w->ctx;
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  int rc = enqueue_all(w, st);  // warm-up
  float best = 1e30f;
  for (int r = 0; r < reps && rc == 0; ++r) {
    (void)hipEventRecord(a, st);
    rc = enqueue_all(w, st);
    (void)hipEventRecord(b, st);
    if (rc == 0 && hipEventSynchronize(b) == hipSuccess) {
      float t = 0.f;
      (void)hipEventElapsedTime(&t, a, b);
      best = std::min(best, t);
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = best;
  return rc;
}

int capture(vpgs_window* w) {
  vpgs_ctx* ctx = w->ctx;
  if (!w->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&w->cap_stream, hipStreamNonBlocking));
  for (int part = 1; part <= 2; ++part) {
    const bool prof = ctx->profiling;
    ctx->profiling = false;  // no event records inside the graph
    HIP_TRY(hipStreamBeginCapture(w->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_part(w, part, w->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(w->cap_stream, &g);
    ctx->profiling = prof;
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(ctx, VPGS_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    w->graph[part - 1] = g;
    HIP_TRY(hipGraphInstantiate(&w->exec[part - 1], g, nullptr, nullptr, 0));
  }
  return VPGS_OK;
}

// ---- tuning cache ------------------------------------------------------
// A JSON object {"entries": [{"key": "...", "tile_w": .., "tile_h": ..,
// "persistent": .., "lds_batch": .., "ms": ..}, ...]}, one entry per key.

struct TuneEntry {
  std::string key;
  int tile_w = 0, tile_h = 0, persistent = 0, lds_batch = 0;
  double ms = 0.0;
};

std::string tune_key(vpgs_window* w) {
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDeviceProperties(&prop, w->ctx->device) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  for (char& c : arch)
    if (c == '"' || c == '\\') c = '_';
  uint64_t records = 0;
  for (int32_t s : w->view_set) records += (uint64_t)w->sets[s].n;
  std::ostringstream k;
  k << arch << "/" << cus << "cu/" << w->cams.size() << "views/";
  for (size_t v = 0; v < w->cams.size(); ++v) k << (v ? "," : "") << w->cams[v].width << "x" << w->cams[v].height;
  k << "/records2^" << (records > 1 ? (int)std::ceil(std::log2((double)records)) : 0);
  return k.str();
}

// The text of a "name": value field inside one entry, or "" if absent.
std::string field(const std::string& obj, const char* name) {
  const std::string tag = std::string("\"") + name + "\"";
  size_t p = obj.find(tag);
  if (p == std::string::npos) return "";
  p = obj.find(':', p + tag.size());
  if (p == std::string::npos) return "";
  ++p;
  while (p < obj.size() && (obj[p] == ' ' || obj[p] == '\t' || obj[p] == '\n')) ++p;
  if (p < obj.size() && obj[p] == '"') {
    const size_t q = obj.find('"', p + 1);
    return q == std::string::npos ? "" : obj.substr(p + 1, q - p - 1);
  }
  size_t q = p;
  while (q < obj.size() && obj[q] != ',' && obj[q] != '}') ++q;
  return obj.substr(p, q - p);
}

std::vector<TuneEntry> read_cache(const char* path) {
  std::vector<TuneEntry> out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  size_t p = text.find('[');
  while (p != std::string::npos) {
    const size_t a = text.find('{', p);
    if (a == std::string::npos) break;
    const size_t b = text.find('}', a);
    if (b == std::string::npos) break;
    const std::string obj = text.substr(a, b - a + 1);
    TuneEntry e;
    e.key = field(obj, "key");
    const std::string tw = field(obj, "tile_w"), th = field(obj, "tile_h"), pe = field(obj, "persistent"),
                      nb = field(obj, "lds_batch"), ms = field(obj, "ms");
    if (!e.key.empty() && !tw.empty() && !th.empty() && !pe.empty() && !nb.empty()) {
      e.tile_w = std::atoi(tw.c_str());
      e.tile_h = std::atoi(th.c_str());
      e.persistent = std::atoi(pe.c_str());
      e.lds_batch = std::atoi(nb.c_str());
      e.ms = ms.empty() ? 0.0 : std::atof(ms.c_str());
      out.push_back(e);
    }
    p = b + 1;
  }
  return out;
}

int write_cache(vpgs_ctx* ctx, const char* path, const TuneEntry& e) {
  std::vector<TuneEntry> all = read_cache(path);
  bool found = false;
  for (TuneEntry& x : all)
    if (x.key == e.key) { x = e; found = true; }
  if (!found) all.push_back(e);
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return fail(ctx, VPGS_EINVAL, "tuning cache %s: cannot write", path);
    f << "{\"entries\": [\n";
    for (size_t i = 0; i < all.size(); ++i) {
      char ms[32];
      std::snprintf(ms, sizeof(ms), "%.4f", all[i].ms);
      f << "  {\"key\": \"" << all[i].key << "\", \"tile_w\": " << all[i].tile_w << ", \"tile_h\": " << all[i].tile_h
        << ", \"persistent\": " << all[i].persistent << ", \"lds_batch\": " << all[i].lds_batch << ", \"ms\": " << ms
        << "}" << (i + 1 < all.size() ? "," : "") << "\n";
    }
    f << "]}\n";
    if (!f) return fail(ctx, VPGS_EINVAL, "tuning cache %s: write failed", path);
  }
  if (std::rename(tmp.c_str(), path) != 0) return fail(ctx, VPGS_EINVAL, "tuning cache %s: cannot replace", path);
  return VPGS_OK;
}

void release(vpgs_window* w) {
  for (int i = 0; i < 2; ++i) {
    if (w->exec[i]) (void)hipGraphExecDestroy(w->exec[i]);
    if (w->graph[i]) (void)hipGraphDestroy(w->graph[i]);
  }
  if (w->cap_stream) (void)hipStreamDestroy(w->cap_stream);
  if (w->sv) destroy_saved(w->sv);
  if (w->h_overflow) (void)hipHostFree(w->h_overflow);
  delete w;
}

}  // namespace

extern "C" {

int vpgs_window_create(vpgs_ctx* ctx, int n_sets, const vpgs_gaussians* sets, int n_views, const int32_t* view_set,
                       const vpgs_camera* cams, const vpgs_images* out, const vpgs_image_grads* grad_out,
                       const vpgs_gauss_grads* grads, float* d_pose, const vpgs_window_opts* opts, vpgs_window** win,
                       void* stream) {
  if (!ctx) return VPGS_EINVAL;
  if (!win) return fail(ctx, VPGS_EINVAL, "NULL window pointer");
  *win = nullptr;
  vpgs_window_opts o{};
  o.persistent = -1;
  o.use_graph = 1;
  if (opts) o = *opts;
  if (o.tune_reps <= 0) o.tune_reps = 3;
  if (o.lds_batch < 0) return fail(ctx, VPGS_EINVAL, "lds_batch must be >= 0");
  if ((o.tile_w != 0 || o.tile_h != 0) && !tile_shape_supported(o.tile_w, o.tile_h))
    return fail(ctx, VPGS_EUNSUPPORTED, "tile shape %dx%d not built", o.tile_w, o.tile_h);
  if (o.pair_capacity < 0 || o.pair_capacity > 0x7fffffffLL) return fail(ctx, VPGS_EINVAL, "pair_capacity out of range");
  vpgs_render_opts ro{};
  ro.tile_w = o.tile_w;
  ro.tile_h = o.tile_h;
  int rc = validate_forward(ctx, n_sets, sets, n_views, view_set, cams, out, &ro);
  if (rc) return rc;
  if (!grad_out || !grads) return fail(ctx, VPGS_EINVAL, "NULL gradient arrays");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));

  vpgs_window* w = new (std::nothrow) vpgs_window();
  if (!w) return fail(ctx, VPGS_ENOMEM, "out of host memory");
  w->ctx = ctx;
  w->sets.assign(sets, sets + n_sets);
  w->view_set.assign(view_set, view_set + n_views);
  w->cams.assign(cams, cams + n_views);
  w->out.assign(out, out + n_views);
  w->grad_out.assign(grad_out, grad_out + n_views);
  w->grads.assign(grads, grads + n_sets);
  w->d_pose = d_pose;
  rc = new_saved(ctx, &w->sv);
  if (rc) { release(w); return rc; }
  w->sv->in_use = true;
  w->sv->count_work = !o.skip_counts;

  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
  const bool fixed_nb = o.lds_batch > 0;
  if (fixed_nb && o.tile_w && !lds_batch_supported(o.tile_w, o.tile_h, o.lds_batch))
    { release(w); return fail(ctx, VPGS_EUNSUPPORTED, "LDS batch of %d entries not built", o.lds_batch); }
  if (o.persistent > kMaxGridCtas) { release(w); return fail(ctx, VPGS_EINVAL, "persistent grid out of range"); }

  int best_tw = 0, best_th = 0, best_mode = 0, best_nb = 0;
  float best_ms = 1e30f;
  bool from_cache = false;
  std::string key;
  if (o.tune_cache) {
    key = tune_key(w);
    for (const TuneEntry& e : read_cache(o.tune_cache)) {
      const bool fits = e.key == key && tile_shape_supported(e.tile_w, e.tile_h) &&
                        lds_batch_supported(e.tile_w, e.tile_h, e.lds_batch) && e.persistent >= 0 &&
                        e.persistent <= kMaxGridCtas && (!o.tile_w || (o.tile_w == e.tile_w && o.tile_h == e.tile_h)) &&
                        (o.persistent < 0 || o.persistent == e.persistent) && (!fixed_nb || o.lds_batch == e.lds_batch);
      if (fits) {
        best_tw = e.tile_w; best_th = e.tile_h; best_mode = e.persistent; best_nb = e.lds_batch;
        best_ms = (float)e.ms;
        from_cache = true;
      }
    }
  }

  // candidates of the search
  std::vector<std::pair<int, int>> shapes;
  if (o.tile_w && o.tile_h) shapes.push_back({o.tile_w, o.tile_h});
  else for (auto& s : kShapes) shapes.push_back({s[0], s[1]});
  std::vector<int> modes;
  if (o.persistent >= 0) modes.push_back(o.persistent);
  else { modes.push_back(0); modes.push_back(2 * cus); modes.push_back(4 * cus); modes.push_back(8 * cus); }

  if (!from_cache) {
    const bool search = shapes.size() * modes.size() > 1 || !fixed_nb;
    best_tw = shapes[0].first; best_th = shapes[0].second; best_mode = modes[0];
    best_nb = fixed_nb ? o.lds_batch : best_tw * best_th;
    // stage 1: shape x grid at one batch per tile's pixels (or the given batch)
    for (auto& sh : shapes) {
      const int nb = fixed_nb ? o.lds_batch : sh.first * sh.second;
      if (!lds_batch_supported(sh.first, sh.second, nb)) continue;
      if ((rc = configure(w, sh.first, sh.second, nb)) || (rc = size_pairs(w, st, o.pair_capacity))) { release(w); return rc; }
      if (!search) break;
      for (int m : modes) {
        w->sv->persistent_blocks = (uint32_t)m;
        float ms = 0.f;
        rc = time_config(w, st, o.tune_reps, &ms);
        if (rc) { release(w); return rc; }
        if (ms < best_ms) { best_ms = ms; best_tw = sh.first; best_th = sh.second; best_mode = m; best_nb = nb; }
      }
    }
    // stage 2: the other batch sizes of the best shape and grid
    if (search && !fixed_nb) {
      const int px = best_tw * best_th;
      for (int nb : {px / 2, 2 * px}) {
        if (!lds_batch_supported(best_tw, best_th, nb)) continue;
        if ((rc = configure(w, best_tw, best_th, nb)) || (rc = size_pairs(w, st, o.pair_capacity))) { release(w); return rc; }
        w->sv->persistent_blocks = (uint32_t)best_mode;
        float ms = 0.f;
        rc = time_config(w, st, o.tune_reps, &ms);
        if (rc) { release(w); return rc; }
        if (ms < best_ms) { best_ms = ms; best_nb = nb; }
      }
    }
  }
  o.tile_w = best_tw;
  o.tile_h = best_th;
  o.persistent = best_mode;
  o.lds_batch = best_nb;
  if ((rc = configure(w, best_tw, best_th, best_nb)) || (rc = size_pairs(w, st, o.pair_capacity))) { release(w); return rc; }
  w->sv->persistent_blocks = (uint32_t)best_mode;
  if (o.tune_cache && !from_cache && best_ms < 1e30f) {
    TuneEntry e;
    e.key = key;
    e.tile_w = best_tw; e.tile_h = best_th; e.persistent = best_mode; e.lds_batch = best_nb; e.ms = best_ms;
    if ((rc = write_cache(ctx, o.tune_cache, e))) { release(w); return rc; }
  }
  w->tuned_from_cache = from_cache;
  o.pair_capacity = w->sv->capacity;
  o.tune_cache = nullptr;  // the caller's path is not kept
  w->cfg = o;
  HIP_TRY(hipStreamSynchronize(st));
  {
    hipError_t e = hipHostMalloc((void**)&w->h_overflow, sizeof(uint32_t), hipHostMallocMapped);
    if (e == hipSuccess) {
      *(volatile uint32_t*)w->h_overflow = 0u;
      e = hipHostGetDevicePointer((void**)&w->d_overflow, w->h_overflow, 0);
    }
    if (e != hipSuccess) {
      release(w);
      return fail(ctx, VPGS_ENOMEM, "pinned overflow flag: %s", hipGetErrorString(e));
    }
  }
  if (o.use_graph) {
    rc = capture(w);
    if (rc) { release(w); return rc; }
  }
  *win = w;
  return VPGS_OK;
}

int vpgs_window_set_cameras(vpgs_window* w, const vpgs_camera* cams) {
  if (!w) return VPGS_EINVAL;
  vpgs_ctx* ctx = w->ctx;
  if (!cams) return fail(ctx, VPGS_EINVAL, "NULL cameras");
  for (size_t v = 0; v < w->cams.size(); ++v)
    if (cams[v].width != w->cams[v].width || cams[v].height != w->cams[v].height)
      return fail(ctx, VPGS_EINVAL, "view %zu: image size changed", v);
  std::vector<vpgs_camera> old = w->cams;
  w->cams.assign(cams, cams + old.size());
  vpgs_render_opts ro{};
  int rc = validate_forward(ctx, (int)w->sets.size(), w->sets.data(), (int)w->cams.size(), w->view_set.data(),
                            w->cams.data(), w->out.data(), &ro);
  if (rc) { w->cams = old; return rc; }
  w->tables_dirty = true;
  return VPGS_OK;
}

int vpgs_window_set_accum(vpgs_window* w, const vpgs_densify_accum* acc) {
  if (!w) return VPGS_EINVAL;
  vpgs_ctx* ctx = w->ctx;
  if (!acc) {
    w->accum.clear();
  } else {
    if (acc->grad_space != 0 && acc->grad_space != 1) return fail(ctx, VPGS_EINVAL, "grad_space must be 0 or 1");
    if (!acc->accum) return fail(ctx, VPGS_EINVAL, "NULL accumulator array");
    for (size_t s = 0; s < w->sets.size(); ++s)
      if (acc->accum[s] && (reinterpret_cast<uintptr_t>(acc->accum[s]) & 15u) != 0)
        return fail(ctx, VPGS_EINVAL, "set %zu: accumulators must be 16-byte aligned", s);
    w->accum.assign(acc->accum, acc->accum + w->sets.size());
    w->acc_desc = *acc;
  }
  w->tables_dirty = true;
  return VPGS_OK;
}

int vpgs_window_run(vpgs_window* w, int parts, void* stream) {
  if (!w) return VPGS_EINVAL;
  vpgs_ctx* ctx = w->ctx;
  if (parts < 1 || parts > 3) return fail(ctx, VPGS_EINVAL, "parts must be 1 (forward), 2 (backward) or 3 (both)");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  if (*(volatile uint32_t*)w->h_overflow)
    return fail(ctx, VPGS_ECAPACITY, "the pair list of an earlier run overflowed its capacity of %u pairs: its "
                "outputs were invalid; recreate the window with a larger pair_capacity", w->sv->capacity);
  if (w->tables_dirty) {
    // rebuild the tables for the new poses (same shapes, same buffers) and upload
    int rc = build_tables(ctx, *w->sv->h_tab, (int)w->sets.size(), w->sets.data(), (int)w->view_set.size(),
                          w->view_set.data(), w->cams.data(), w->out.data(), w->cfg.tile_w, w->cfg.tile_h);
    if (!rc) rc = bind_backward(ctx, *w->sv->h_tab, w->grad_out.data(), w->grads.data());
    if (!rc) rc = bind_accum(ctx, *w->sv->h_tab, accum_of(w));
    if (!rc) rc = upload_tables(ctx, w->sv, st);
    if (rc) return rc;
    w->tables_dirty = false;
  }
  for (int part = 1; part <= 2; ++part) {
    if (!(parts & part)) continue;
    if (w->exec[part - 1]) {
      HIP_TRY(hipGraphLaunch(w->exec[part - 1], st));
    } else {
      int rc = enqueue_part(w, part, st);
      if (rc) return rc;
    }
  }
  return VPGS_OK;
}

int vpgs_window_stats(vpgs_window* w, vpgs_stats* out, void* stream) {
  if (!w) return VPGS_EINVAL;
  return vpgs_saved_stats(w->ctx, w->sv, out, stream);
}

int vpgs_window_config(const vpgs_window* w, vpgs_window_opts* out) {
  if (!w || !out) return VPGS_EINVAL;
  *out = w->cfg;
  return VPGS_OK;
}

int vpgs_window_destroy(vpgs_window* w) {
  if (!w) return VPGS_EINVAL;
  (void)hipSetDevice(w->ctx->device);
  (void)hipDeviceSynchronize();
  release(w);
  return VPGS_OK;
}

}  // extern "C"
