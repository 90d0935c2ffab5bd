// Differentiable unrolled PDHG (forward with checkpoints, hand-written reverse).
#include "kp_internal.h"

using namespace kp;

extern "C" {

int64_t pdhg_unrolled_ckpt_bytes(kp_plan_t plan, int K, int ckpt_every) {
    (void)plan; (void)K; (void)ckpt_every;
    return -1;
}

int pdhg_unrolled_forward(kp_plan_t, const void*, const float*, int, const float*, int, int, const void*, void*,
                          void*, void*) {
    set_error("not implemented");
    return KP_ERR_UNSUPPORTED;
}

int pdhg_unrolled_backward(kp_plan_t, const void*, const float*, int, const float*, int, int, const void*,
                           const void*, const void*, float*, void*, void*, void*) {
    set_error("not implemented");
    return KP_ERR_UNSUPPORTED;
}

}  // extern "C"
