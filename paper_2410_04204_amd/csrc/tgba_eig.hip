// Dense symmetric eigensolver (placeholder until the device solver lands).
#include "tgba_internal.h"

extern "C" int tgba_eig(int64_t n, double *A, int64_t lda, double *w, int flags, void *stream) {
    (void)n; (void)A; (void)lda; (void)w; (void)flags; (void)stream;
    return tgba::set_error(TGBA_EUNSUPPORTED, "tgba_eig is not built yet");
}
