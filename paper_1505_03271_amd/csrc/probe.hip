// Streaming-bandwidth reference kernels: what plain coalesced b128 sweeps
// reach on this device for the traffic mixes of the FV passes (one read and
// one write per byte, as the predictor; two reads and one write, as the
// corrector; reads only).  A ceiling to read the stage kernels' bandwidth
// against, not part of the method.
#include "lb_kernels.h"

namespace lbk {

typedef __attribute__((ext_vector_type(4))) float f4;

// kind 0: d = a; kind 1: d = a + b; kind 2: reads of a and b only (one
// lane-dependent store that never happens keeps them live).
template <int KIND>
__global__ void __launch_bounds__(256) stream_kernel(const f4* __restrict__ a, const f4* __restrict__ b,
                                                     f4* __restrict__ d, size_t n) {
    float acc = 0.f;
    for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += size_t(gridDim.x) * 256) {
        if (KIND == 0) d[i] = a[i];
        else if (KIND == 1) d[i] = a[i] + b[i];
        else {
            const f4 v = a[i] + b[i];
            acc += v.x + v.y + v.z + v.w;
        }
    }
    if (KIND == 2 && acc == -1.2345f) d[threadIdx.x] = f4{acc, acc, acc, acc};
}

hipError_t launch_stream(int kind, int grid, const void* a, const void* b, void* d, size_t n, hipStream_t s) {
    const f4* A = static_cast<const f4*>(a);
    const f4* B = static_cast<const f4*>(b);
    f4* D = static_cast<f4*>(d);
    if (kind == 0) hipLaunchKernelGGL(stream_kernel<0>, dim3(grid), dim3(256), 0, s, A, B, D, n);
    else if (kind == 1) hipLaunchKernelGGL(stream_kernel<1>, dim3(grid), dim3(256), 0, s, A, B, D, n);
    else hipLaunchKernelGGL(stream_kernel<2>, dim3(grid), dim3(256), 0, s, A, B, D, n);
    return hipGetLastError();
}

}  // namespace lbk
