// Spectral sums (placeholder).
#include "tgba_internal.h"

extern "C" int tgba_dsf(int64_t, const double *, int64_t, const double *, const double *, int64_t, int,
                        const double *, int, double, double *, double *, void *) {
    return tgba::set_error(TGBA_EUNSUPPORTED, "tgba_dsf is not built yet");
}
extern "C" int tgba_quench(int64_t, const double *, int64_t, const double *, const double *, int64_t,
                           const double *, double, double, int, double *, double *, double *, void *) {
    return tgba::set_error(TGBA_EUNSUPPORTED, "tgba_quench is not built yet");
}
extern "C" int tgba_quench_overlaps(const tgba_basis *, int, double, int, double *, void *) {
    return tgba::set_error(TGBA_EUNSUPPORTED, "tgba_quench_overlaps is not built yet");
}
