// The perceptron trainer behind the C ABI (veckm_trainer_*): device state,
// argument checks and the launch of one training step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>

#include "veckm_internal.h"

using namespace veckm;

struct veckm_trainer {
  TrainState s;
  int device = 0;
  int64_t t = 0;  // Adam steps taken
};

namespace {

constexpr int kHeadBlocks = 512;
constexpr int kMaxSplits = 64;

void free_state(TrainState& s) {
  float* bufs[] = {s.theta, s.grad, s.m1, s.m2, s.H, s.dZ, s.head_part, s.w1_part};
  for (float* b : bufs)
    if (b) (void)hipFree(b);
  s = TrainState{};
}

}  // namespace

extern "C" {

int veckm_trainer_create(int32_t d, int32_t hidden, int64_t max_rows, const float* W1,
                         const float* b1, const float* W2, const float* b2, veckm_trainer** out) {
  if (!out) return VECKM_E_INVAL;
  *out = nullptr;
  if (d < 1 || d > 256 || hidden < 64 || hidden > 512 || hidden % 64 || max_rows < 1 ||
      max_rows > (int64_t)1 << 30 || !W1 || !b1 || !W2 || !b2)
    return VECKM_E_INVAL;
  int dev = 0, n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1 || hipGetDevice(&dev) != hipSuccess)
    return VECKM_E_NODEVICE;
  veckm_trainer* tr = new (std::nothrow) veckm_trainer();
  if (!tr) return VECKM_E_NOMEM;
  tr->device = dev;
  TrainState& s = tr->s;
  s.k2 = 2 * d;
  s.hidden = hidden;
  s.max_rows = max_rows;
  s.head_blocks = kHeadBlocks;
  s.max_splits = kMaxSplits;
  const int64_t np = (int64_t)hidden * s.k2 + 3 * (int64_t)hidden + 2;
  auto alloc = [](float** p, int64_t count) {
    return dev_malloc(reinterpret_cast<void**>(p), (size_t)count * sizeof(float));
  };
  bool ok = alloc(&s.theta, np) && alloc(&s.grad, np + 1) && alloc(&s.m1, np) &&
            alloc(&s.m2, np) && alloc(&s.H, max_rows * hidden) && alloc(&s.dZ, max_rows * hidden) &&
            alloc(&s.head_part, (int64_t)kHeadBlocks * (3 * hidden + 3)) &&
            alloc(&s.w1_part, (int64_t)kMaxSplits * hidden * s.k2);
  if (ok) {
    float* p = s.theta;
    ok = hipMemcpy(p, W1, (size_t)hidden * s.k2 * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(p + (int64_t)hidden * s.k2, b1, (size_t)hidden * 4, hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemcpy(p + (int64_t)hidden * s.k2 + hidden, W2, (size_t)2 * hidden * 4,
                   hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(p + (int64_t)hidden * s.k2 + 3 * hidden, b2, 2 * 4, hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemset(s.m1, 0, (size_t)np * 4) == hipSuccess &&
         hipMemset(s.m2, 0, (size_t)np * 4) == hipSuccess &&
         hipDeviceSynchronize() == hipSuccess;
  }
  if (!ok) {
    free_state(s);
    delete tr;
    return VECKM_E_NOMEM;
  }
  *out = tr;
  return VECKM_OK;
}

void veckm_trainer_destroy(veckm_trainer* tr) {
  if (!tr) return;
  (void)hipSetDevice(tr->device);
  (void)hipDeviceSynchronize();
  free_state(tr->s);
  delete tr;
}

int veckm_trainer_step(veckm_trainer* tr, const float* emb, const float* target, int64_t m,
                       int32_t optimizer, float lr, float* loss, void* stream) {
  if (!tr || m < 1 || !emb || !target || (optimizer != 0 && optimizer != 1) ||
      !(lr >= 0.f) || !std::isfinite(lr))
    return VECKM_E_INVAL;
  if (m > tr->s.max_rows) return VECKM_E_RANGE;
  float c1 = 1.f, c2 = 1.f;
  if (optimizer == 1) {
    const int64_t t = tr->t + 1;
    c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)t)));
    c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)t)));
  }
  const int rc = launch_train_step(tr->s, emb, target, m, optimizer, lr, c1, c2, stream);
  if (rc) return rc;
  if (optimizer == 1) ++tr->t;
  if (loss) {
    const int64_t np = (int64_t)tr->s.hidden * tr->s.k2 + 3 * (int64_t)tr->s.hidden + 2;
    if (hipMemcpyAsync(loss, tr->s.grad + np, sizeof(float), hipMemcpyDeviceToDevice,
                       (hipStream_t)stream) != hipSuccess)
      return VECKM_E_HIP;
  }
  return VECKM_OK;
}

int veckm_trainer_get(veckm_trainer* tr, float* W1, float* b1, float* W2, float* b2) {
  if (!tr || !W1 || !b1 || !W2 || !b2) return VECKM_E_INVAL;
  const TrainState& s = tr->s;
  const int64_t w1 = (int64_t)s.hidden * s.k2;
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(W1, s.theta, (size_t)w1 * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(b1, s.theta + w1, (size_t)s.hidden * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(W2, s.theta + w1 + s.hidden, (size_t)2 * s.hidden * 4, hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(b2, s.theta + w1 + 3 * s.hidden, 2 * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return VECKM_E_HIP;
  return VECKM_OK;
}

}  // extern "C"
