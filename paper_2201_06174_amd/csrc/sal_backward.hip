// sal_backward.hip -- adjoint of the saliency path (placeholder until the adjoint kernels land).
#include "sal_aux.h"

using namespace sal;

extern "C" {

size_t sal_backward_workspace_size(int64_t, int64_t, int64_t, const sal_spec*) { return 0; }

sal_status sal_backward(const float*, int64_t, int64_t, int64_t, const sal_spec*, const sal_stencil*,
                        const sal_fusion*, const float*, const float*, const double*, const float*, const uint8_t*,
                        const float*, float*, void*, size_t, sal_stream) {
    return fail(SAL_ERR_UNSUPPORTED, "adjoint not built yet");
}

}  // extern "C"
