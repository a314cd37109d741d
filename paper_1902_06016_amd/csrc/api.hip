// Context lifetime, operator build entry point, inspection and event timers.
#include "common.h"

namespace gfcc {

void build_operator(gfcc_ctx* ctx, int o, int v, const double* eps, const double* t1,
                    const double* t2, const double* l1, const double* l2, const double* oooo,
                    const double* ooov, const double* oovv, const double* ovvo,
                    const double* ovvv, int keep);

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
  GFCC_REQUIRE(o >= 2 && v >= 1, GFCC_EINVAL, "build_hbar_operands: need o >= 2 and v >= 1");
  GFCC_REQUIRE((int64_t)o * v <= (1 << 20) && o <= 4096, GFCC_EINVAL,
               "build_hbar_operands: o*v too large");
  GFCC_REQUIRE(eps && t1 && t2 && l1 && l2 && oooo && ooov && oovv && ovvo && ovvv, GFCC_EINVAL,
               "build_hbar_operands: null pointer");
  GFCC_REQUIRE((precision_mask & ~(GFCC_KEEP_FP64 | GFCC_KEEP_FP32 | GFCC_KEEP_TRANSPOSE)) == 0,
               GFCC_EINVAL, "build_hbar_operands: unknown precision_mask bits");
  const int64_t O = o, V = v;
  struct { const double* p; int64_t n; const char* name; } arrs[] = {
      {eps, O + V, "eps"}, {t1, O * V, "t1"}, {t2, O * O * V * V, "t2"}, {l1, O * V, "l1"},
      {l2, O * O * V * V, "l2"}, {oooo, O * O * O * O, "oooo"}, {ooov, O * O * O * V, "ooov"},
      {oovv, O * O * V * V, "oovv"}, {ovvo, O * V * V * O, "ovvo"}, {ovvv, O * V * V * V, "ovvv"}};
  for (auto& a : arrs)
    GFCC_REQUIRE(count_nonfinite(ctx, a.p, a.n) == 0, GFCC_EINVAL,
                 std::string("build_hbar_operands: non-finite entries in ") + a.name);
  build_operator(ctx, o, v, eps, t1, t2, l1, l2, oooo, ooov, oovv, ovvo, ovvv,
                 precision_mask | GFCC_KEEP_FP64);
  GFCC_API_END(ctx)
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
  GFCC_REQUIRE(which == 0 || which == 1, GFCC_EINVAL, "gfcc_timer: unknown timer");
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
