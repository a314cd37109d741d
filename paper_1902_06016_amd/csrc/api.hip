// Context lifetime, operator build entry point, inspection and event timers.
#include <algorithm>
#include <initializer_list>
#include <iterator>

#include "common.h"

namespace gfcc {

void build_operator(gfcc_ctx* ctx, int o, int v, const double* eps, const double* t1,
                    const double* t2, const double* l1, const double* l2, const double* oooo,
                    const double* ooov, const double* oovv, const double* ovvo,
                    const double* ovvv, int keep);
void first_order_t2(gfcc_ctx* ctx, int o, int v, const double* eps, const double* oovv,
                    double* t2);
void eval_scratch_setup(int device);

struct NamedArray {
  const double* p;
  int64_t n;
  const char* name;
};

// Shared argument checks of the operator builds (throws Error).
static void check_build_args(gfcc_ctx* ctx, const char* fn, int o, int v, int precision_mask,
                             std::initializer_list<NamedArray> arrs) {
  GFCC_REQUIRE(o >= 2 && v >= 1, GFCC_EINVAL, std::string(fn) + ": need o >= 2 and v >= 1");
  GFCC_REQUIRE((int64_t)o * v <= (1 << 20) && o <= 4096, GFCC_EINVAL,
               std::string(fn) + ": o*v too large");
  for (auto& a : arrs)
    GFCC_REQUIRE(a.p != nullptr, GFCC_EINVAL, std::string(fn) + ": null pointer");
  GFCC_REQUIRE((precision_mask & ~(GFCC_KEEP_FP64 | GFCC_KEEP_FP32 | GFCC_KEEP_TRANSPOSE)) == 0,
               GFCC_EINVAL, std::string(fn) + ": unknown precision_mask bits");
  std::vector<std::pair<const double*, int64_t>> list;
  for (auto& a : arrs) list.emplace_back(a.p, a.n);
  const std::vector<int64_t> bad = count_nonfinite(ctx, list);
  size_t k = 0;
  for (auto& a : arrs)
    GFCC_REQUIRE(bad[k++] == 0, GFCC_EINVAL, std::string(fn) + ": non-finite entries in " + a.name);
}

static hipEvent_t event_get(gfcc_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  GFCC_HIP(hipEventCreate(&e));
  return e;
}

void timer_begin(gfcc_ctx* ctx, int which, hipEvent_t* ev) {
  *ev = nullptr;
  if (!ctx->timers[which].enabled) return;
  *ev = event_get(ctx);
  GFCC_HIP(hipEventRecord(*ev, ctx->stream));
}

void timer_end(gfcc_ctx* ctx, int which, hipEvent_t ev0) {
  if (!ev0) return;
  hipEvent_t e1 = event_get(ctx);
  GFCC_HIP(hipEventRecord(e1, ctx->stream));
  ctx->timers[which].pending.emplace_back(ev0, e1);
  ctx->timers[which].launches += 1;
  if (ctx->timers[which].pending.size() > 256) timers_collect(ctx);
}

void timer_cancel(gfcc_ctx* ctx, hipEvent_t ev0) {
  if (ev0) ctx->event_pool.push_back(ev0);
}

// Fold completed event pairs into the accumulated times (waits for the recorded events).
void timers_collect(gfcc_ctx* ctx) {
  for (auto& t : ctx->timers) {
    for (auto& pr : t.pending) {
      GFCC_HIP(hipEventSynchronize(pr.second));
      float ms = 0.f;
      GFCC_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
      t.ms += ms;
      ctx->event_pool.push_back(pr.first);
      ctx->event_pool.push_back(pr.second);
    }
    t.pending.clear();
  }
}

}  // namespace gfcc

extern "C" {

int64_t gfcc_dim(int o, int v) {
  if (o < 0 || v < 0) return -1;
  return (int64_t)o + (int64_t)o * (o - 1) / 2 * v;
}

gfcc_status gfcc_create(gfcc_ctx** out, int device, void* hip_stream) {
  if (!out) return GFCC_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return GFCC_EINVAL;
  gfcc_ctx* ctx = new (std::nothrow) gfcc_ctx();
  if (!ctx) return GFCC_ENOMEM;
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return GFCC_EHIP;
  }
  try {
    gfcc::eval_scratch_setup(device);   // with `device` current: once per device
  } catch (const gfcc::Error& e) {
    delete ctx;
    return e.status;
  }
  *out = ctx;
  return GFCC_OK;
}

gfcc_status gfcc_destroy(gfcc_ctx* ctx) {
  if (!ctx) return GFCC_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& t : ctx->timers)
    for (auto& pr : t.pending) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  for (auto& kv : ctx->step_graphs) (void)hipGraphExecDestroy(kv.second);
  if (ctx->hflags) (void)hipHostFree(ctx->hflags);
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  delete ctx;
  return GFCC_OK;
}

const char* gfcc_last_error(const gfcc_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

gfcc_status build_hbar_operands(gfcc_ctx* ctx, int o, int v, const double* eps,
                                const double* t1, const double* t2, const double* l1,
                                const double* l2, const double* oooo, const double* ooov,
                                const double* oovv, const double* ovvo, const double* ovvv,
                                int precision_mask) {
  if (!ctx) return GFCC_EINVAL;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  GFCC_HIP(hipSetDevice(ctx->device));
  const int64_t O = o, V = v;
  check_build_args(ctx, "build_hbar_operands", o, v, precision_mask,
                   {{eps, O + V, "eps"}, {t1, O * V, "t1"}, {t2, O * O * V * V, "t2"},
                    {l1, O * V, "l1"}, {l2, O * O * V * V, "l2"}, {oooo, O * O * O * O, "oooo"},
                    {ooov, O * O * O * V, "ooov"}, {oovv, O * O * V * V, "oovv"},
                    {ovvo, O * V * V * O, "ovvo"}, {ovvv, O * V * V * V, "ovvv"}});
  build_operator(ctx, o, v, eps, t1, t2, l1, l2, oooo, ooov, oovv, ovvo, ovvv,
                 precision_mask | GFCC_KEEP_FP64);
  GFCC_API_END(ctx)
}

gfcc_status build_hbar_first_order(gfcc_ctx* ctx, int o, int v, const double* eps,
                                   const double* oooo, const double* ooov, const double* oovv,
                                   const double* ovvo, const double* ovvv, int precision_mask) {
  if (!ctx) return GFCC_EINVAL;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  GFCC_HIP(hipSetDevice(ctx->device));
  const int64_t O = o, V = v;
  check_build_args(ctx, "build_hbar_first_order", o, v, precision_mask,
                   {{eps, O + V, "eps"}, {oooo, O * O * O * O, "oooo"},
                    {ooov, O * O * O * V, "ooov"}, {oovv, O * O * V * V, "oovv"},
                    {ovvo, O * V * V * O, "ovvo"}, {ovvv, O * V * V * V, "ovvv"}});
  std::vector<double> he(O + V);
  GFCC_HIP(hipMemcpyAsync(he.data(), eps, sizeof(double) * (O + V), hipMemcpyDeviceToHost,
                          ctx->stream));
  GFCC_HIP(hipStreamSynchronize(ctx->stream));
  double homo = he[0], lumo = he[O];
  for (int64_t i = 1; i < O; ++i) homo = std::max(homo, he[i]);
  for (int64_t a = O + 1; a < O + V; ++a) lumo = std::min(lumo, he[a]);
  GFCC_REQUIRE(homo < lumo, GFCC_EINVAL,
               "build_hbar_first_order: every occupied energy must lie below every virtual one");
  DevBuf bt2, bz;
  bt2.alloc(sizeof(double) * (size_t)(O * O * V * V));
  bz.alloc(sizeof(double) * (size_t)(O * V));
  fill(ctx, bz.as<double>(), O * V, 0.0);
  first_order_t2(ctx, o, v, eps, oovv, bt2.as<double>());
  build_operator(ctx, o, v, eps, bz.as<double>(), bt2.as<double>(), bz.as<double>(),
                 bt2.as<double>(), oooo, ooov, oovv, ovvo, ovvv, precision_mask | GFCC_KEEP_FP64);
  GFCC_HIP(hipStreamSynchronize(ctx->stream));  // the amplitudes are freed on return
  GFCC_API_END(ctx)
}

gfcc_status gfcc_autotune(gfcc_ctx* ctx, int enable) {
  if (!ctx || enable < 0 || enable > 2) return GFCC_EINVAL;
  ctx->tune_mode = enable;
  ctx->tune.clear();
  ctx->tune_pins.clear();
  gfcc::drop_step_graphs(ctx);
  return GFCC_OK;
}

gfcc_status gfcc_graphs(gfcc_ctx* ctx, int enable) {
  if (!ctx || enable < 0 || enable > 1) return GFCC_EINVAL;
  ctx->graphs = enable != 0;
  gfcc::drop_step_graphs(ctx);
  return GFCC_OK;
}

gfcc_status gfcc_compact(gfcc_ctx* ctx, int enable) {
  if (!ctx || enable < 0 || enable > 1) return GFCC_EINVAL;
  ctx->compact = enable != 0;
  return GFCC_OK;
}

gfcc_status gfcc_autotune_pin(gfcc_ctx* ctx, int kind, int tile_m, int tile_n, int splits) {
  if (!ctx) return GFCC_EINVAL;
  if (kind != gfcc::TUNE_SIGMA_1H && kind != gfcc::TUNE_SIGMA_2H1P) return GFCC_EINVAL;
  const bool unfused = tile_m == 0 && tile_n == 0;
  if (!unfused && ((tile_m != 32 && tile_m != 64 && tile_m != 128) ||
                   (tile_n != 64 && tile_n != 128) || splits < 1))
    return GFCC_EINVAL;
  ctx->tune_pins[kind] = {tile_m, tile_n, unfused ? 0 : splits};
  gfcc::drop_step_graphs(ctx);
  return GFCC_OK;
}

gfcc_status gfcc_autotune_entry(const gfcc_ctx* ctx, int index, int64_t* desc, double* us) {
  if (!ctx || !desc || index < 0 || (size_t)index >= ctx->tune.size()) return GFCC_EINVAL;
  auto it = ctx->tune.begin();
  std::advance(it, index);
  const gfcc::TuneKey& k = it->first;
  desc[0] = k[0];
  desc[1] = k[1];
  desc[2] = it->second.M;
  desc[3] = it->second.N;
  desc[4] = it->second.K;
  desc[5] = it->second.splits;
  desc[6] = it->second.tile_m;
  desc[7] = it->second.tile_n;
  if (us) {
    us[0] = it->second.best_us;
    us[1] = it->second.generic_us;
  }
  return GFCC_OK;
}

gfcc_status gfcc_export(gfcc_ctx* ctx, int which, void* dst) {
  if (!ctx) return GFCC_EINVAL;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  Operator& op = ctx->op;
  GFCC_REQUIRE(op.built, GFCC_ESTATE, "gfcc_export: no operator built");
  GFCC_REQUIRE(dst, GFCC_EINVAL, "gfcc_export: null pointer");
  const DevBuf* src = nullptr;
  switch (which) {
    case 0: src = &op.Foo; break;
    case 1: src = &op.Fov; break;
    case 2: src = &op.Fvv; break;
    case 3: src = &op.Woooo; break;
    case 4: src = &op.Wooov; break;
    case 5: src = &op.Wovvo; break;
    case 6: src = &op.Wovoo; break;
    case 7: src = &op.diag; break;
    default: throw Error(GFCC_EINVAL, "gfcc_export: unknown block");
  }
  GFCC_HIP(hipMemcpyAsync(dst, src->p, src->bytes, hipMemcpyDeviceToDevice, ctx->stream));
  GFCC_HIP(hipStreamSynchronize(ctx->stream));
  GFCC_API_END(ctx)
}

gfcc_status gfcc_timer(gfcc_ctx* ctx, int which, int enable, int reset, double* ms_out,
                       int64_t* launches_out) {
  if (!ctx) return GFCC_EINVAL;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  GFCC_REQUIRE(which >= 0 && which <= 2, GFCC_EINVAL, "gfcc_timer: unknown timer");
  timers_collect(ctx);
  TimerSlot& t = ctx->timers[which];
  if (ms_out) *ms_out = t.ms;
  if (launches_out) *launches_out = t.launches;
  if (reset) {
    t.ms = 0.0;
    t.launches = 0;
  }
  t.enabled = enable != 0;
  GFCC_API_END(ctx)
}

}  // extern "C"
