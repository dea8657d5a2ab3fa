// C ABI: Laplacian eigensolver, distillation projector and correlators.
#include "../../include/dlma.h"
#include "runtime.h"

using namespace dlma;

extern "C" int dlma_lap_eigs(dlma_gauge_t, int, int, int, const void*, void*, double*, const dlma_eig_opts*, void*) {
    return fail(DLMA_EUNSUPPORTED, "dlma_lap_eigs: not built yet");
}
extern "C" int dlma_project(dlma_gauge_t, int, int, const void*, const void*, void*, int, int, void*) {
    return fail(DLMA_EUNSUPPORTED, "dlma_project: not built yet");
}
extern "C" int dlma_correlators(dlma_gauge_t, int, int, const void*, const void*, int, const void*, const void*, double*, void*) {
    return fail(DLMA_EUNSUPPORTED, "dlma_correlators: not built yet");
}
