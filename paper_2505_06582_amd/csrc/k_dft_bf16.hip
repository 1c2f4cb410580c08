// Split-bf16 matrix-core DFT (placeholder until the MFMA kernels land).
#include "gws_internal.h"

namespace gws {

size_t dft_bf16x3_workspace(int nx, int ny, int batch)
{
    (void)nx; (void)ny; (void)batch;
    return 256;
}

hipError_t launch_dft_bf16x3(Plan &p, int batch, int direction, const float2 *in, float2 *out, void *ws, hipStream_t s)
{
    (void)p; (void)batch; (void)direction; (void)in; (void)out; (void)ws; (void)s;
    return hipErrorNotSupported;
}

}  // namespace gws
