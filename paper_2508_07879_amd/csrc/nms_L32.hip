// Instantiations of the neural min-sum kernels for lift size L = 32.
#include "decode_nms.h"

namespace qldpc {

hipError_t launch_wreg_weighted_L32(const DecodeArgs &a, hipStream_t st);

hipError_t launch_nms_L32(int op, const NmsArgs &n, const DecodeArgs &d, hipStream_t st) {
    using S = ShapeLP35Z;
    using G = Geo<S, 32>;
    switch (op) {
        case 0:
            hipLaunchKernelGGL((k_nms_fwd<S, 32>), dim3((unsigned)n.tiles), dim3(64), 0, st, n);
            break;
        case 1:
            hipLaunchKernelGGL((k_nms_bwd<S, 32>), dim3((unsigned)n.waves), dim3(64), 0, st, n);
            break;
        case 2: {
            const long total = (long)n.T * S::SLOTS * 32;
            hipLaunchKernelGGL((k_nms_reduce<S, 32>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n);
            break;
        }
        case 3:   // inference: messages in registers
            return launch_wreg_weighted_L32(d, st);
        default:
            return hipErrorNotSupported;
    }
    return hipGetLastError();
}

}  // namespace qldpc
