// Launcher of the edge-list decoder (decode_generic.h).
#include "decode_generic.h"
#include "kernels.h"

namespace qldpc {

namespace {

template <int FMT, bool PB, bool PO>
hipError_t launch_one(const GenCode &g, const DecodeArgs &a, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL((k_gen<FMT, PB, PO>), dim3((unsigned)a.batch), dim3(64), lds, st, g, a);
    return hipGetLastError();
}

template <int FMT>
hipError_t launch_fmt(const GenCode &g, const LaunchKey &k, const DecodeArgs &a, size_t lds, hipStream_t st) {
    if (k.per_bit) return k.post ? launch_one<FMT, true, true>(g, a, lds, st) : launch_one<FMT, true, false>(g, a, lds, st);
    return k.post ? launch_one<FMT, false, true>(g, a, lds, st) : launch_one<FMT, false, false>(g, a, lds, st);
}

}  // namespace

hipError_t launch_generic_decode(const GenCode &g, const LaunchKey &k, const DecodeArgs &a, hipStream_t stream) {
    if (k.sched != 0) return hipErrorNotSupported;
    const int b = k.fmt == 0 ? 4 : k.fmt == 2 ? 2 : 1;
    const size_t lds = gen_lds_bytes(g.m, g.n, g.max_dc, b);
    if (lds > kGenMaxLds) return hipErrorNotSupported;
    switch (k.fmt) {
        case 0: return launch_fmt<0>(g, k, a, lds, stream);
        case 1: return launch_fmt<1>(g, k, a, lds, stream);
        case 2: return launch_fmt<2>(g, k, a, lds, stream);
        default: return hipErrorNotSupported;
    }
}

}  // namespace qldpc
