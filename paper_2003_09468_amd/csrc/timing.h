// Kernel classes for the optional event timing (see afqmc_kpt_timing_enable).
#pragma once

#include <hip/hip_runtime.h>

namespace afqmc {

enum KernelClass {
  KC_TAYLOR = AFQMC_KC_TAYLOR,
  KC_VHS = AFQMC_KC_VHS,
  KC_VBIAS = AFQMC_KC_VBIAS,
  KC_GREENS = AFQMC_KC_GREENS,
  KC_BHALF = AFQMC_KC_BHALF,
  KC_WEIGHTS = AFQMC_KC_WEIGHTS,
  KC_ORTHO = AFQMC_KC_ORTHO,
  KC_EXCHANGE = AFQMC_KC_EXCHANGE,
  KC_ENERGY_REST = AFQMC_KC_ENERGY_REST,
  KC_EXCHANGE_BWD = AFQMC_KC_EXCHANGE_BWD,
  KC_COUNT = AFQMC_KC_COUNT
};

bool timing_on();

// Records an event pair around the launches made in its lifetime when timing is enabled.
class TimedScope {
 public:
  TimedScope(int kc, hipStream_t s);
  ~TimedScope();

 private:
  int rec_;
  hipStream_t s_;
};

}  // namespace afqmc
