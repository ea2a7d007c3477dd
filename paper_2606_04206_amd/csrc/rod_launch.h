// Host-callable launchers of the rod kernels (defined in rod_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "rod_device.h"

namespace rods {

// which: 0 = forward, 1 = forward writing the substep tape, 2 = adjoint
// SC: rods with self-contact (their pair scratch in a.pblk / a.pblk_off,
//     blocks laid out by sc_block with SC_RV_FWD values per pair of records
//     for kinds 0 and 1, SC_RV_ADJ for kind 2)
// GT: the adjoint keeps a substep's projection iterates in the rod's block
//     of global scratch (sc_tape/sc_off) rather than in LDS (implied by SC)
template <typename T>
hipError_t launch_rods(int which, int C, int W, bool SC, bool GT, const RodArgs<T>& a,
                       int n_blocks, hipStream_t st);
// rods with self-contact (kernels of their own translation unit)
template <typename T>
hipError_t launch_rods_sc(int which, int C, int W, const RodArgs<T>& a, int n_blocks,
                          hipStream_t st);
template <typename T>
size_t sc_lds_bytes(int C, int W);
// rods with self-contact and moving rigid bodies (C = 2, a.bw set)
template <typename T>
hipError_t launch_rods_sc_bodies(int which, int C, int W, const RodArgs<T>& a, int n_blocks,
                                 hipStream_t st);
// rods with the twist degree of freedom and self-contact (C = 2)
template <typename T>
hipError_t launch_rods_sc_twist(int which, int C, int W, const RodArgs<T>& a, int n_blocks,
                                hipStream_t st);
// rods with the twist degree of freedom (C = 2, no self-contact)
template <typename T>
hipError_t launch_rods_twist(int which, int C, int W, bool GT, const RodArgs<T>& a,
                             int n_blocks, hipStream_t st);
// rods with the twist degree of freedom and moving rigid bodies (C = 2)
template <typename T>
hipError_t launch_rods_twist_bodies(int which, int C, int W, bool GT, const RodArgs<T>& a,
                                    int n_blocks, hipStream_t st);
// rods with moving rigid bodies (C = 2, no self-contact or twist; a.bw set)
template <typename T>
hipError_t launch_rods_bodies(int which, int C, int W, bool GT, const RodArgs<T>& a,
                              int n_blocks, hipStream_t st);
// dynamic LDS of a launch shape (kind 0/1 forward, 2 adjoint)
template <typename T>
size_t kernel_lds_bytes(int which, int C, int W, bool SC, bool GT, int n_iters);
template <typename T>
hipError_t launch_init_frames(const int32_t* voff, int R, const T* x, T* d1, hipStream_t st);
// adds to xb the position adjoint that the frame adjoint d1b induces
// through the initial-frame rule at positions x (tmp: [V][3] scratch)
template <typename T>
hipError_t launch_init_frames_vjp(const int32_t* voff, int R, const T* x, const T* d1b, T* tmp,
                                  T* xb, hipStream_t st);
template <typename T>
hipError_t launch_curvature(const int32_t* voff, const int32_t* rod_of, int V, const T* x,
                            const T* d1, T* kappa, hipStream_t st);
template <typename T>
hipError_t launch_loss(const int32_t* voff, int R, const T* x, const T* tgt, double* part,
                       T* loss, T* dldx, hipStream_t st);
template <typename T>
hipError_t launch_reduce_params(const int32_t* voff, int R, const double* ab, const double* as,
                                T* db, T* ds, hipStream_t st);
template <typename T>
hipError_t launch_fill(T* p, int64_t n, T val, hipStream_t st);
hipError_t launch_selftest_exchange(int* out, hipStream_t st);
// device address of the static loss scratch on the current device, looked
// up once per device (rod_loss.hip); out may be NULL
int loss_scratch_setup(double** out);
// optimisation driver (rod_optim.hip): one Adam update of n parameters
// (scale, nullable, multiplies the gradient), and elementwise log / exp
template <typename T>
hipError_t launch_adam(T* p, const T* g, const T* scale, T* m, T* v, int64_t n, double lr,
                       double b1, double b2, double eps, int t, hipStream_t st);
template <typename T>
hipError_t launch_log(const T* a, T* out, int64_t n, hipStream_t st);
template <typename T>
hipError_t launch_exp(const T* a, T* out, int64_t n, hipStream_t st);

}  // namespace rods
