// Launch table shared by the kernel instantiation units and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>

#include "negf_kernels.hpp"

namespace negf {

enum { KIND_DECIMATE = 0, KIND_DECIMATE2, KIND_DECIMATE_CIRC, KIND_RECUR64, KIND_RECUR32, KIND_CDIAG64, KIND_CDIAG32, KIND_COLUMN64, KIND_COLUMN32,
       KIND_COUNT };

struct Launchers {
    int B;
    int groups;                  // chains per wavefront (64 / B)
    // launch[kind](sched, grid, dynamic LDS bytes, stream)
    void (*launch[KIND_COUNT])(const Sched&, int grid, size_t dyn, hipStream_t);
    const void* func[KIND_COUNT];   // kernel symbols (occupancy queries)
};

template <int B>
struct LaunchImpl {
    static void decimate(const Sched& a, int grid, size_t, hipStream_t s) {
        hipLaunchKernelGGL(k_decimate<B>, dim3(grid), dim3(64), 0, s, a);
    }
    static void decimate2(const Sched& a, int grid, size_t, hipStream_t s) {
        hipLaunchKernelGGL(k_decimate2<B>, dim3(grid), dim3(64), 0, s, a);
    }
    static void decimate_circ(const Sched& a, int grid, size_t, hipStream_t s) {
        hipLaunchKernelGGL(k_decimate_circ<B>, dim3(grid), dim3(64), 0, s, a);
    }
    template <typename T>
    static void recur(const Sched& a, int grid, size_t dyn, hipStream_t s) {
        hipLaunchKernelGGL((k_recur<T, B>), dim3(grid), dim3(64), dyn, s, a);
    }
    template <typename T>
    static void cdiag(const Sched& a, int grid, size_t, hipStream_t s) {
        hipLaunchKernelGGL((k_cdiag<T, B>), dim3(grid), dim3(64), 0, s, a);
    }
    template <typename T>
    static void column(const Sched& a, int grid, size_t, hipStream_t s) {
        hipLaunchKernelGGL((k_column<T, B>), dim3(grid), dim3(64), 0, s, a);
    }
    static const Launchers* table() {
        static const Launchers t = {
            B, 64 / B,
            {&decimate, &decimate2, &decimate_circ, &recur<double>, &recur<float>, &cdiag<double>, &cdiag<float>, &column<double>,
             &column<float>},
            {reinterpret_cast<const void*>(&k_decimate<B>), reinterpret_cast<const void*>(&k_decimate2<B>),
             reinterpret_cast<const void*>(&k_decimate_circ<B>), reinterpret_cast<const void*>(&k_recur<double, B>),
             reinterpret_cast<const void*>(&k_recur<float, B>), reinterpret_cast<const void*>(&k_cdiag<double, B>),
             reinterpret_cast<const void*>(&k_cdiag<float, B>), reinterpret_cast<const void*>(&k_column<double, B>),
             reinterpret_cast<const void*>(&k_column<float, B>)}};
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
