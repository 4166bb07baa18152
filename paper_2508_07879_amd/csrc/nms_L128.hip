// Instantiations of the neural min-sum kernels for lift size L = 128.
#include "decode_nms.h"

namespace qldpc {

hipError_t launch_nms_L128(int op, const NmsArgs &n, const DecodeArgs &d, hipStream_t st) {
    using S = ShapeLP35Z;
    using G = Geo<S, 128>;
    switch (op) {
        case 0:
            hipLaunchKernelGGL((k_nms_fwd<S, 128>), dim3((unsigned)n.tiles), dim3(64), 0, st, n);
            break;
        case 1:
            hipLaunchKernelGGL((k_nms_bwd<S, 128>), dim3((unsigned)n.waves), dim3(64), 0, st, n);
            break;
        case 2: {
            const long total = (long)n.T * S::SLOTS * 128;
            hipLaunchKernelGGL((k_nms_reduce<S, 128>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n);
            break;
        }
        case 3:
            if (d.weight_iters < d.max_iters)   // neural, then plain iterations
                hipLaunchKernelGGL((k_wave<S, 128, 0, 0, false, false, 2>),
                                   dim3((unsigned)((d.batch + G::SPW - 1) / G::SPW)), dim3(64), 0, st, d);
            else
                hipLaunchKernelGGL((k_wave<S, 128, 0, 0, false, false, 1>),
                                   dim3((unsigned)((d.batch + G::SPW - 1) / G::SPW)), dim3(64), 0, st, d);
            break;
        default:
            return hipErrorNotSupported;
    }
    return hipGetLastError();
}

}  // namespace qldpc
