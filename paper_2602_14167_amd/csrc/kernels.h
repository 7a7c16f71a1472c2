// Launch interfaces of the HIP kernels (host side).
#pragma once

#include "common.h"

namespace tcng {

// device copies of a circuit plan
struct DevPlan {
    const Pass* passes = nullptr;
    const Phase* phases = nullptr;
    const Op* ops = nullptr;
};

struct DevPauliPlan {
    const PPass* passes = nullptr;
    const PGroup* groups = nullptr;
    const PClass* classes = nullptr;
    const PTerm* terms = nullptr;
};

// ---- tiled passes
// opm: [batch][n_ops][16] matrix entries of the plan's ops, written by launch_build_ops
template <typename R>
hipError_t launch_build_ops(const DevPlan& dp, int n_ops, const void* params, int64_t pstride, const void* cmats,
                            int64_t batch, void* opm, hipStream_t st);
template <typename R, int RB>
hipError_t launch_tile_fwd(const DevPlan& dp, int pass_idx, int m, void* state, int64_t stride, int n, int64_t batch,
                           const void* opm, int n_ops, hipStream_t st);
template <typename R, int RB>
hipError_t launch_tile_rev(const DevPlan& dp, int pass_idx, int m, void* state, void* costate, int64_t stride, int n,
                           int64_t batch, const void* opm, int n_ops, int wgs, double* part, int total_slots,
                           hipStream_t st);
template <typename R, int RB>
hipError_t launch_pauli_tile(const DevPauliPlan& dp, int pass_idx, int n_passes, int m, const void* state,
                             void* costate, bool accumulate, int64_t stride, int n, int64_t batch, int wgs,
                             double* epart, hipStream_t st);

// ---- plain (one kernel per gate / per Pauli X-group)
template <typename R>
hipError_t launch_gate1(void* state, int64_t stride, int n, int64_t batch, int q, int kind, int p0, int mat,
                        const void* params, int64_t pstride, const void* cmats, const void* umat, bool inv,
                        hipStream_t st);
template <typename R>
hipError_t launch_gate2(void* state, int64_t stride, int n, int64_t batch, int q0, int q1, int kind, int p0, int p1,
                        int mat, const void* params, int64_t pstride, const void* cmats, const void* umat, bool inv,
                        hipStream_t st);
template <typename R>
hipError_t launch_gatek(void* state, int64_t stride, int n, int64_t batch, const int32_t* qubits, int k,
                        const void* umat, hipStream_t st);
template <typename R>
hipError_t launch_rev1(void* state, void* costate, int64_t stride, int n, int64_t batch, int q, int kind, int p0,
                       int mat, const void* params, int64_t pstride, const void* cmats, int slot, int wgs,
                       double* part, int total_slots, hipStream_t st);
template <typename R>
hipError_t launch_rev2(void* state, void* costate, int64_t stride, int n, int64_t batch, int q0, int q1, int kind,
                       int p0, int p1, int mat, const void* params, int64_t pstride, const void* cmats, int slot,
                       int wgs, double* part, int total_slots, hipStream_t st);
template <typename R>
hipError_t launch_pauli_group(const void* state, void* costate, bool accumulate, int64_t stride, int n, int64_t batch,
                              uint64_t x, const PClassFull* classes, int class_begin, int class_end,
                              const PTermFull* terms, int wgs, double* epart, int row, int n_rows, hipStream_t st);

// ---- misc
template <typename R>
hipError_t launch_init(void* state, int64_t stride, int n, int64_t batch, const void* amps_in, int64_t basis,
                       hipStream_t st);

hipError_t launch_zero(double* p, size_t count, hipStream_t st);

// grad[b][p] = sum over slots of p of sum_wg part; energy[b] = sum of erows; lie from U2 cotangents.
// scratch: batch * (total_slots + erows) doubles.
hipError_t launch_finish(const double* part, int total_slots, int wgs, const int32_t* slot_ptr,
                         const int32_t* slot_idx, int n_params, const double* epart, int erows, int ewgs,
                         int64_t batch, double* energy, double* grad, double* gate_grad, const int32_t* gate_slot,
                         const double* u2_mats_c128, const int32_t* gate_mat, int n_gates, double* scratch,
                         hipStream_t st);

}  // namespace tcng
