// Instantiations of the neural min-sum kernels for lift size L = 64.
#include "decode_nms.h"

namespace qldpc {

hipError_t launch_wreg_weighted_L64(const DecodeArgs &a, hipStream_t st);

hipError_t launch_nms_L64(int op, const NmsArgs &n, const DecodeArgs &d, hipStream_t st) {
    using S = ShapeLP35Z;
    using G = Geo<S, 64>;
    switch (op) {
        case 0:
            hipLaunchKernelGGL((k_nms_fwd<S, 64>), dim3((unsigned)n.tiles), dim3(64), 0, st, n);
            break;
        case 1:
            hipLaunchKernelGGL((k_nms_bwd<S, 64>), dim3((unsigned)n.waves), dim3(64), 0, st, n);
            break;
        case 2: {
            const long total = (long)n.T * S::SLOTS * 64;
            hipLaunchKernelGGL((k_nms_reduce<S, 64>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n);
            break;
        }
        case 3:   // inference: messages in registers
            return launch_wreg_weighted_L64(d, st);
        default:
            return hipErrorNotSupported;
    }
    return hipGetLastError();
}

}  // namespace qldpc
