// batched.hip -- independent relaxations of many small systems (placeholder
// until the persistent batched kernel lands).
#include <hip/hip_runtime.h>

#include "fire2.h"

extern "C" void fire_batched_release(void* ws) { (void)ws; }

extern "C" int fire_batched_run(struct fire_ctx* ctx, int nsys, const long long* offsets, double* pos,
                                const fire_box* boxes, const fire_potential* pot, const fire_params* per_sys,
                                double tol, long long max_steps, fire_result* out) {
  (void)ctx; (void)nsys; (void)offsets; (void)pos; (void)boxes; (void)pot; (void)per_sys; (void)tol;
  (void)max_steps; (void)out;
  return FIRE_E_ARG;
}
