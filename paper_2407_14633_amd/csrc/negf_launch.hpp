// Launch table shared by the kernel instantiation units and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>

#include "negf_kernels.hpp"

namespace negf {

struct Launchers {
    int B;
    int groups;   // chains per wavefront (64 / B)
    void (*decimate)(const DecArgs&, int grid, hipStream_t);
    void (*recur64)(const RgfArgs&, int grid, hipStream_t);
    void (*recur32)(const RgfArgs&, int grid, hipStream_t);
    void (*cdiag64)(const RgfArgs&, int nc_chunk, int grid, hipStream_t);
    void (*cdiag32)(const RgfArgs&, int nc_chunk, int grid, hipStream_t);
    void (*column64)(const RgfArgs&, int er0, int nr_chunk, int grid, hipStream_t);
    void (*column32)(const RgfArgs&, int er0, int nr_chunk, int grid, hipStream_t);
};

template <int B>
struct LaunchImpl {
    static void decimate(const DecArgs& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL(k_decimate<B>, dim3(grid), dim3(64), 0, s, a);
    }
    template <typename T>
    static void recur(const RgfArgs& a, int grid, hipStream_t s) {
        const size_t dyn = (size_t)a.n_uniq * B * a.K * (sizeof(cx<T>) + 1);
        hipLaunchKernelGGL((k_recur<T, B>), dim3(grid), dim3(64), dyn, s, a);
    }
    template <typename T>
    static void cdiag(const RgfArgs& a, int nc, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_cdiag<T, B>), dim3(grid), dim3(64), 0, s, a, nc);
    }
    template <typename T, typename S>
    static void column(const RgfArgs& a, int er0, int nr, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_column<T, S, B>), dim3(grid), dim3(64), 0, s, a, er0, nr);
    }
    static const Launchers* table() {
        static const Launchers t = {B, 64 / B, &decimate, &recur<double>, &recur<float>,
                                    &cdiag<double>, &cdiag<float>, &column<double, double>, &column<float, float>};
        return &t;
    }
};

// one accessor per supported ring size, defined in the instantiation units
#define NEGF_DECLARE_B(B) const Launchers* launchers_b##B();
NEGF_DECLARE_B(1) NEGF_DECLARE_B(2) NEGF_DECLARE_B(3) NEGF_DECLARE_B(4) NEGF_DECLARE_B(5)
NEGF_DECLARE_B(6) NEGF_DECLARE_B(7) NEGF_DECLARE_B(8) NEGF_DECLARE_B(9) NEGF_DECLARE_B(10)
NEGF_DECLARE_B(11) NEGF_DECLARE_B(12) NEGF_DECLARE_B(13) NEGF_DECLARE_B(14) NEGF_DECLARE_B(15)
NEGF_DECLARE_B(16) NEGF_DECLARE_B(17) NEGF_DECLARE_B(18) NEGF_DECLARE_B(19) NEGF_DECLARE_B(20)
NEGF_DECLARE_B(21) NEGF_DECLARE_B(22) NEGF_DECLARE_B(23) NEGF_DECLARE_B(24)
#undef NEGF_DECLARE_B

#define NEGF_DEFINE_B(B) \
    const Launchers* launchers_b##B() { return LaunchImpl<B>::table(); }
#define NEGF_STUB_B(B) \
    const Launchers* launchers_b##B() { return nullptr; }

}  // namespace negf
