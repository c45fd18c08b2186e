// autotune.hip -- the library's own search over the launch shape of a frame
// or a batch (hdof_tuning: persistent-trace blocks per CU, refill batch,
// queue segments, traversal form, overlapped gather and its ray quantum).
//
// The knobs change only how work is scheduled, never the results, so the
// search times the caller's real workload through the public entry points
// and keeps the fastest shape.  Coordinate descent from the defaults: each
// knob in turn over its candidate values with the others held, twice over,
// a change kept only when it is faster by more than HDOF_AT_GAIN; each
// candidate is the median of several timed runs after warm runs, HIP events
// on the caller's stream around each run.
//
// The cache is a JSON-lines file: one object per workload class,
//   {"key": "gfx950|256|frame 1920x1080 spp8 ...", "blocks_per_cu": 10, ...,
//    "ms": 0.39, "default_ms": 0.40}
// keyed by the device's architecture, its CU count and the workload's class
// (image sizes, ray budget, post-filter tile, scene size in powers of two,
// view count, the optional stages), so one search serves every frame of
// that class on that kind of device.
#include "hdof_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#define HDOF_AT_GAIN 0.005  // relative gain a candidate needs to replace the current shape

namespace {

std::string workload_key(const hdof_ctx* ctx, const hdof_scene* scene, const hdof_frame_params* p, int n_views,
                         const hdof_view* views, bool history) {
  hipDeviceProp_t prop;
  char arch[64] = "unknown";
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) {
    snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    char* colon = strchr(arch, ':');  // drop feature suffixes (":sramecc+:xnack-")
    if (colon) *colon = 0;
  }
  char buf[512];
  int tris_log2 = 0;
  while ((1 << (tris_log2 + 1)) <= scene->n_tris) ++tris_log2;
  long px = 0;
  for (int v = 0; v < n_views; ++v) px += (long)views[v].cam.width * views[v].cam.height;
  if (n_views == 1)
    snprintf(buf, sizeof buf, "%s|%d|frame %dx%d spp%d mtile%d pptile%d tris2^%d recon%d spatial%d spec%d hist%d",
             arch, ctx->n_cu, views[0].cam.width, views[0].cam.height, p->mask.spp_max, p->mask.tile, p->pp.tile,
             tris_log2, p->recon.enable, p->spatial.enable, scene->spec && p->comp.spec_y > 0.0f ? 1 : 0,
             history ? 1 : 0);
  else
    snprintf(buf, sizeof buf, "%s|%d|batch %d views %.1fMpx spp%d mtile%d pptile%d tris2^%d", arch, ctx->n_cu,
             n_views, (double)px / 1e6, p->mask.spp_max, p->mask.tile, p->pp.tile, tris_log2);
  return buf;
}

bool read_int(const char* line, const char* name, int* out) {
  char pat[64];
  snprintf(pat, sizeof pat, "\"%s\":", name);
  const char* q = strstr(line, pat);
  return q && sscanf(q + strlen(pat), " %d", out) == 1;
}

bool line_key(const char* line, std::string* key) {
  const char* q = strstr(line, "\"key\":");
  if (!q) return false;
  q = strchr(q + 6, '"');
  if (!q) return false;
  const char* e = strchr(q + 1, '"');
  if (!e) return false;
  key->assign(q + 1, e - q - 1);
  return true;
}

std::vector<std::string> read_lines(const char* path) {
  std::vector<std::string> out;
  FILE* f = fopen(path, "r");
  if (!f) return out;
  char buf[2048];
  while (fgets(buf, sizeof buf, f)) {
    size_t n = strlen(buf);
    while (n && (buf[n - 1] == '\n' || buf[n - 1] == '\r')) buf[--n] = 0;
    if (n) out.push_back(buf);
  }
  fclose(f);
  return out;
}

bool cache_lookup(const char* path, const std::string& key, hdof_tuning* t, float* ms, float* dms) {
  for (const std::string& l : read_lines(path)) {
    std::string k;
    if (!line_key(l.c_str(), &k) || k != key) continue;
    hdof_tuning r;
    if (!read_int(l.c_str(), "blocks_per_cu", &r.blocks_per_cu) || !read_int(l.c_str(), "refill", &r.refill) ||
        !read_int(l.c_str(), "segments", &r.segments) || !read_int(l.c_str(), "wave", &r.wave) ||
        !read_int(l.c_str(), "overlap", &r.overlap) ||
        !read_int(l.c_str(), "overlap_ray_quantum", &r.overlap_ray_quantum))
      continue;
    const char* q = strstr(l.c_str(), "\"ms\":");
    *ms = q ? (float)atof(q + 5) : 0.0f;
    q = strstr(l.c_str(), "\"default_ms\":");
    *dms = q ? (float)atof(q + 13) : 0.0f;
    *t = r;
    return true;
  }
  return false;
}

hdof_status cache_store(const char* path, const std::string& key, const hdof_tuning& t, float ms, float dms) {
  std::vector<std::string> keep;
  for (const std::string& l : read_lines(path)) {
    std::string k;
    if (line_key(l.c_str(), &k) && k == key) continue;  // replaced below
    keep.push_back(l);
  }
  char line[1024];
  snprintf(line, sizeof line,
           "{\"key\": \"%s\", \"blocks_per_cu\": %d, \"refill\": %d, \"segments\": %d, \"wave\": %d, "
           "\"overlap\": %d, \"overlap_ray_quantum\": %d, \"ms\": %.5f, \"default_ms\": %.5f}",
           key.c_str(), t.blocks_per_cu, t.refill, t.segments, t.wave, t.overlap, t.overlap_ray_quantum, ms, dms);
  keep.push_back(line);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return hdof_set_error(HDOF_ERR_INVALID_ARG, "autotune cache %s: cannot write", tmp.c_str());
  for (const std::string& l : keep) fprintf(f, "%s\n", l.c_str());
  if (fclose(f) != 0 || rename(tmp.c_str(), path) != 0)
    return hdof_set_error(HDOF_ERR_INVALID_ARG, "autotune cache %s: cannot replace", path);
  return HDOF_OK;
}

struct Workload {
  hdof_ctx* ctx;
  const hdof_scene* scene;
  const hdof_light* light;
  const hdof_frame_params* params;
  int n_views;
  const hdof_view* views;
  const hdof_camera* prev;  // single frames: the previous camera (NULL: no history)
  hipStream_t st;

  hdof_status run() const {
    if (n_views == 1) {
      const hdof_view& v = views[0];
      return hdof_frame(ctx, scene, &v.cam, prev, &v.lens, light, params, v.seed, v.frame, v.view, v.d_out,
                        nullptr, st);
    }
    return hdof_frame_batched(ctx, scene, light, params, n_views, views, st);
  }
};

// median over `reps` timed runs of the workload under tuning t
hdof_status time_tuning(const Workload& w, const hdof_tuning& t, int warm, int reps, hipEvent_t* ev, float* ms) {
  hdof_status s = hdof_set_tuning(w.ctx, &t);
  if (s != HDOF_OK) return s;
  for (int i = 0; i < warm; ++i)
    if ((s = w.run()) != HDOF_OK) return s;
  std::vector<float> v(reps);
  HDOF_HIP(hipEventRecord(ev[0], w.st));
  for (int i = 0; i < reps; ++i) {
    if ((s = w.run()) != HDOF_OK) return s;
    HDOF_HIP(hipEventRecord(ev[i + 1], w.st));
  }
  HDOF_HIP(hipEventSynchronize(ev[reps]));
  for (int i = 0; i < reps; ++i) HDOF_HIP(hipEventElapsedTime(&v[i], ev[i], ev[i + 1]));
  std::nth_element(v.begin(), v.begin() + reps / 2, v.end());
  *ms = v[reps / 2];
  return HDOF_OK;
}

}  // namespace

extern "C" hdof_status hdof_autotune(hdof_ctx* ctx, const hdof_scene* scene, const hdof_light* light,
                                     const hdof_frame_params* params, int32_t n_views, const hdof_view* views,
                                     const hdof_camera* prev, const char* cache_path, int32_t force,
                                     hdof_tuning* out, hdof_autotune_report* report, hdof_stream stream) {
  if (!ctx) return hdof_set_error(HDOF_ERR_INVALID_ARG, "context is NULL");
  if (!scene || !light || !params || !views || !out)
    return hdof_set_error(HDOF_ERR_INVALID_ARG, "scene, light, params, views and out must be non-NULL");
  if (n_views < 1 || n_views > HDOF_MAX_VIEWS)
    return hdof_set_error(HDOF_ERR_INVALID_ARG, "n_views must be in [1, %d]", HDOF_MAX_VIEWS);
  if (prev && n_views != 1)
    return hdof_set_error(HDOF_ERR_INVALID_ARG, "a previous camera applies to single frames only");
  hipStream_t st = (hipStream_t)stream;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HDOF_HIP(hipStreamIsCapturing(st, &cap));
  if (cap != hipStreamCaptureStatusNone)
    return hdof_set_error(HDOF_ERR_UNSUPPORTED, "the autotuner times its candidates: not under stream capture");
  const std::string key = workload_key(ctx, scene, params, n_views, views, prev != nullptr);
  hdof_autotune_report rep;
  memset(&rep, 0, sizeof rep);
  snprintf(rep.key, sizeof rep.key, "%s", key.c_str());
  if (cache_path && !force) {
    hdof_tuning t;
    float ms = 0.0f, dms = 0.0f;
    if (cache_lookup(cache_path, key, &t, &ms, &dms)) {
      hdof_status s = hdof_set_tuning(ctx, &t);
      if (s != HDOF_OK) return s;  // a cache entry outside the valid ranges
      *out = t;
      rep.best_ms = ms;
      rep.default_ms = dms;
      rep.from_cache = 1;
      if (report) *report = rep;
      return HDOF_OK;
    }
  }
  const Workload w{ctx, scene, light, params, n_views, views, prev, st};
  const hdof_tuning entry = ctx->tune;  // restored when the search fails
  const bool frame = n_views == 1;
  // a batch is ~30x a frame: fewer repetitions of each candidate
  const int warm = frame ? 3 : 1, reps = frame ? 15 : 5;
  std::vector<hipEvent_t> ev(reps + 1, nullptr);
  for (auto& e : ev) {
    const hipError_t he = hipEventCreate(&e);
    if (he != hipSuccess) {
      for (auto& x : ev)
        if (x) hipEventDestroy(x);
      return hdof_set_error(HDOF_ERR_HIP, "autotune events: %s", hipGetErrorString(he));
    }
  }
  const hdof_tuning defaults = {HDOF_DEFAULT_BPC, 64, 8, 0, 1, 140000};
  hdof_tuning best = defaults;
  float best_ms = 0.0f;
  hdof_status s = HDOF_OK;
  // the GPU's clocks ramp up over the first tens of milliseconds of load:
  // run the workload before the first measurement
  for (int i = 0; i < (frame ? 150 : 8) && s == HDOF_OK; ++i) s = w.run();
  if (s == HDOF_OK) s = time_tuning(w, best, warm, reps, ev.data(), &best_ms);
  rep.default_ms = best_ms;
  rep.candidates = 1;
  // candidate values per knob (the batched form keeps every trace block: the
  // ray quantum applies to single frames only)
  static const int bpc_v[] = {4, 6, 8, 10, 12, 16};
  static const int refill_v[] = {16, 32, 64};
  static const int seg_v[] = {1, 2, 4, 8};
  static const int wave_v[] = {0, 1};
  static const int ovl_v[] = {0, 1};
  static const int quantum_v[] = {80000, 100000, 120000, 140000, 170000, 200000, 260000};
  struct Knob {
    int32_t hdof_tuning::*field;
    const int* vals;
    int n;
    bool frame_only;
  };
  const Knob knobs[] = {{&hdof_tuning::wave, wave_v, 2, false},
                        {&hdof_tuning::overlap, ovl_v, 2, false},
                        {&hdof_tuning::overlap_ray_quantum, quantum_v, 7, true},
                        {&hdof_tuning::blocks_per_cu, bpc_v, 6, false},
                        {&hdof_tuning::segments, seg_v, 4, false},
                        {&hdof_tuning::refill, refill_v, 3, false}};
  for (int pass = 0; pass < 2 && s == HDOF_OK; ++pass) {
    bool changed = false;
    for (const Knob& kb : knobs) {
      if (kb.frame_only && !frame) continue;
      if (kb.field == &hdof_tuning::overlap_ray_quantum && !best.overlap) continue;
      if (kb.field == &hdof_tuning::refill && best.wave == 1) continue;  // the wave form takes whole batches
      for (int i = 0; i < kb.n && s == HDOF_OK; ++i) {
        hdof_tuning c = best;
        c.*kb.field = kb.vals[i];
        if (c.*kb.field == best.*kb.field) continue;
        float ms = 0.0f;
        s = time_tuning(w, c, warm, reps, ev.data(), &ms);
        ++rep.candidates;
        if (s == HDOF_OK && ms < best_ms * (1.0 - HDOF_AT_GAIN)) {
          best = c;
          best_ms = ms;
          changed = true;
        }
      }
    }
    if (!changed) break;
  }
  for (auto& e : ev) hipEventDestroy(e);
  if (s != HDOF_OK) {
    ctx->tune = entry;
    return s;
  }
  s = hdof_set_tuning(ctx, &best);
  if (s != HDOF_OK) return s;
  rep.best_ms = best_ms;
  *out = best;
  if (report) *report = rep;
  if (cache_path) return cache_store(cache_path, key, best, best_ms, rep.default_ms);
  return HDOF_OK;
}
