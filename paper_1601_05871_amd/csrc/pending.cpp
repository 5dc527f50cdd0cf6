// Entry points whose device paths are not built yet: they validate their
// arguments and report FLAME_ERR_UNSUPPORTED.
#include "flame_internal.h"

extern "C" {

int flame_selector_load(const float *w, int64_t count) {
    if (w == nullptr) return -1;
    if (count != FLAME_SEL_NPARAM) return -2;
    return FLAME_ERR_UNSUPPORTED;
}

int flame_select(int64_t n, int64_t batch, int32_t dtype, double kappa, int32_t *variant, int32_t *nb) {
    if (n < 0) return -1;
    if (batch < 0) return -2;
    if (dtype != FLAME_F64 && dtype != FLAME_F32) return -3;
    if (!(kappa >= 0.0)) return -4;
    if (variant == nullptr) return -5;
    if (nb == nullptr) return -6;
    return FLAME_ERR_UNSUPPORTED;
}

int flame_select_logits(const float *features, int64_t count, float *logits) {
    if (features == nullptr && count > 0) return -1;
    if (count < 0) return -2;
    if (logits == nullptr && count > 0) return -3;
    return FLAME_ERR_UNSUPPORTED;
}

int flame_autotune(int32_t dtype, int64_t n, void *A, int64_t lda, int32_t reps, double *times_ms, void *stream) {
    (void)stream;
    if (dtype != FLAME_F64 && dtype != FLAME_F32) return -1;
    if (n < 0) return -2;
    if (A == nullptr && n > 0) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (reps < 1) return -5;
    if (times_ms == nullptr) return -6;
    return FLAME_ERR_UNSUPPORTED;
}

}  // extern "C"
