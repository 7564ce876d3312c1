// ch_kernels.h -- host-side launchers of the HIP kernels in ch_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ch_device.h"

namespace chk {

// work-groups of the velocity check; its flags array holds 2 ints per group
constexpr int CHECK_WGS = 512;

template <typename T, typename A>
hipError_t launch_pass_x(int mi, int nwg, int nth, size_t lds, hipStream_t st,
                         const chd::BoxDesc* boxes, int nbox, const chd::PassArgs& pa,
                         const void* C, const void* U, const void* V, const void* W, void* E,
                         void* Q, bool e25);

template <typename T, typename A>
hipError_t launch_pass_line(int pass, int nwg, int nthreads, size_t lds, hipStream_t st,
                            const chd::BoxDesc* boxes, int nbox, const chd::PassArgs& pa,
                            const void* Qin, void* Qout);

template <typename T>
hipError_t launch_mass(int nblk, int nbox, hipStream_t st, const chd::BoxDesc* boxes,
                       const void* C, double* partial, const double* h3, double* out);

template <typename T>
hipError_t launch_check_velocity(hipStream_t st, const chd::BoxDesc* boxes, int nbox,
                                 const void* U, const void* V, const void* W, int* flags);

template <typename T>
hipError_t launch_interp(hipStream_t st, const void* src, int64_t sx, int64_t sy, int64_t tnx,
                         int64_t tny, int64_t tnz, const int* ix, const double* wx,
                         const int* iy, const double* wy, const int* iz, const double* wz,
                         void* dst);

}  // namespace chk
