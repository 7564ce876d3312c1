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
                         void* Q, bool e25, bool xrow, int xrm);

// The segmented x-pass program: the previous substage's E from Ein, the new
// one into Eout (different arrays).
template <typename T, typename A>
hipError_t launch_pass_x_seg(int nwg, int nth, size_t lds, hipStream_t st,
                             const chd::BoxDesc* boxes, int nbox, const chd::PassArgs& pa,
                             const void* C, const void* U, const void* V, const void* W,
                             const void* Ein, void* Eout, void* Q);

template <typename T, typename A>
hipError_t launch_pass_line(int pass, int nwg, int nthreads, size_t lds, hipStream_t st,
                            const chd::BoxDesc* boxes, int nbox, const chd::PassArgs& pa,
                            const void* Qin, void* Qout);

template <typename T>
hipError_t launch_mass(int nblk, int nbox, hipStream_t st, const chd::BoxDesc* boxes,
                       const void* C, double* partial, const double* h3, double* out);

// Mass of one field described by bd (c_off 0, nmblk blocks): partial holds
// bd.nmblk doubles of scratch, out one double (device memory).
template <typename T>
hipError_t launch_mass_one(hipStream_t st, const chd::BoxDesc& bd, const void* C,
                           double* partial, double h3, double* out);

template <typename T>
hipError_t launch_check_velocity(hipStream_t st, const chd::BoxDesc* boxes, int nbox,
                                 const void* U, const void* V, const void* W, int* flags);

// One component of the coarse-to-fine transfer.  Target rows are grouped in
// bands of `jb` (32, 16, 8, 4, 2 or 1) consecutive y-rows; band b reads the
// coarse rows band[2b], band[2b] + 1, ... (band[2b + 1] of them, cyclic in
// y), and no band spans more than `rmax` rows.  Target row j's y taps are
// given as offsets (row within its band) x sx.  With `xwin` set, the x taps
// of every 4 consecutive targets 4t .. 4t+3 lie within the 6 cyclically
// consecutive coarse points starting at target 4t's first tap.  Weights of
// the y and z stencils are in the working precision.
struct InterpArgs {
    const void* src;        // coarse component [.][sy][sx]
    void* dst;              // target [tnz][tny][tnx]
    int sx, sy;
    int64_t plane;          // sx * sy
    int tnx, tny, tnz;
    int jb, rmax;
    int xwin;
    int nwg;                // work-groups (each takes a contiguous run of items)
    size_t lds;             // bytes of LDS per work-group (interp_lds)
    const int* ix;          // 4 taps per target, x
    const double* wx;
    const int* ly;          // 4 taps per target row, y (band-local offsets)
    const void* wy;
    const int* iz;          // 4 taps per target plane, z
    const void* wz;
    const int* band;
};

// LDS of one transfer work-group: rmax coarse rows and jb target rows
constexpr size_t interp_lds(int rmax, int jb, int sx, size_t esize)
{
    return (size_t)(rmax + jb) * sx * esize;
}

template <typename T>
hipError_t launch_interp(hipStream_t st, const InterpArgs& a);

// Solenoidal transfer: the coarse normal gradient of component comp (0 u
// along x, 1 v along y, 2 w along z) at the coarse cell centres, and the
// in-place integration of a fine component along direction dir from its
// reference plane ref (u: [nz][ny], v: [nz][nx]; w starts from 0 on the
// bottom wall and the top wall plane is set to 0).  Each scan work-group
// writes its largest |closure| to part[group]; scan_groups gives how many.
constexpr int SCAN_WG = 1024;
constexpr int scan_groups(int dir, int nx, int ny, int nz)
{
    const int64_t work = dir == 0 ? ((int64_t)ny * nz + 3) / 4
                       : dir == 1 ? ((int64_t)nz * nx + 255) / 256
                                  : ((int64_t)nx * ny + 255) / 256;
    return (int)(work < SCAN_WG ? (work > 0 ? work : 1) : SCAN_WG);
}

template <typename T>
hipError_t launch_grad(hipStream_t st, const void* src, int comp, int sx, int sy, int sz,
                       const double* dzinv, void* out);

template <typename T>
hipError_t launch_scan(hipStream_t st, int dir, void* buf, const void* ref, int nx, int ny,
                       int nz, double h, double* part);

// Drops of one box (cells with C >= thr joined through faces, bc[d] == 0
// wrapping): lab[i] = the smallest linear index of i's drop, or -1.  Then
// the cells per drop into cnt (zeroed by the caller, one int per cell), and
// the roots with their counts into oroot / ocnt (at most cap entries, in no
// particular order) with the number of drops in *count (zeroed by the
// caller).  Boxes of fewer than 2^31 cells.
template <typename T>
hipError_t launch_drops_label(hipStream_t st, const void* C, int nx, int ny, int nz,
                              const int bc[3], double thr, int* lab);
hipError_t launch_drops_count(hipStream_t st, const int* lab, int64_t n, int* cnt, int cap,
                              int* oroot, int* ocnt, int* count);

// Split-density pressure step: mesh, densities of the two phases, time step.
struct PressArgs {
    int nx, ny, nz, zwalls;
    double h, rho1, rho2, dt;
};

// Phat = 2 P - Pold and Pold <- P; the eq-newpoi right-hand side; the solve
// in spectral space (z walls: per-mode Thomas along z after 2-D transforms;
// periodic z: division by the eigenvalues of the 3-D transform), scaled for
// the unnormalised inverse transform; the eq-u velocity update.
template <typename T>
hipError_t launch_press_prep(hipStream_t st, const void* P, void* Pold, void* phat, int64_t n);
template <typename T>
hipError_t launch_press_rhs(hipStream_t st, const PressArgs& a, const void* C, const void* phat,
                            const void* u, const void* v, const void* w, void* rhs);
template <typename T>
hipError_t launch_press_solve(hipStream_t st, int zwalls, void* spec, void* cp, int nx, int ny,
                              int nz, double h);
template <typename T>
hipError_t launch_press_update(hipStream_t st, const PressArgs& a, const void* C, const void* P,
                               const void* phat, void* u, void* v, void* w);

}  // namespace chk
