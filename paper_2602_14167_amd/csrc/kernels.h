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

// One unit of a tiled launch: a circuit with `batch` members sharing its plan
// (parameter sets), or one circuit of an uneven batch.  A launch covers a
// list of jobs; job j owns blocks [prefix[j], prefix[j+1]) and each member
// `per` consecutive blocks (tiles in the forward sweep, `wgs` workgroups in
// the reverse and Pauli sweeps).  All fields are 32/64-bit (scalar loads).
struct Job {
    const Pass* passes;
    const Phase* phases;
    const Op* ops;            // forward plan
    const Pass* rpasses;
    const Phase* rphases;
    const Op* rops;           // reverse plan
    const PPass* ppasses;
    const PGroup* pgroups;
    const PClass* pclasses;
    const PTerm* pterms;      // Pauli plan
    void* state;              // member b at + b * stride amplitudes
    void* costate;
    const void* opm;          // member b at + b * n_gates * 16 entries
    double* part;             // member b at + b * total_slots * wgs
    double* epart;            // member b at + b * e_rows * e_wgs
    const FPass* fpasses;     // fused plan (matrix-core blocks)
    const FPhase* fphases;
    const FPass* frpasses;
    const FPhase* frphases;
    const void* fmats;        // member b at + b * n_blocks * 2048 floats (forward and reverse operand orders)
    double* opart;            // member b at + b * n_blocks * wgs * 512 (block outer products per workgroup)
    const uint32_t* prec;     // or null: projection applied as the first fused forward pass loads its tiles,
    const double* pkeep;      // member b keeps x with (x & prec[b * prec_stride]) == prec[.. + 1], scaled by
                              // 1 / sqrt(pkeep[b]) (no projection where the mask is 0)
    int64_t stride, batch, tiles;
    int32_t n, n_gates, n_passes, n_ppasses;
    int32_t total_slots, wgs, e_rows, e_wgs;
    int32_t n_blocks, prec_stride;
    int32_t shared, pad2;     // shared: one set of block matrices for every member (fmats and the outer-product
                              // partials of member 0); the reverse grid is `wgs` workgroups over (member, tile)
    const void* src;          // or null: the first fused forward pass loads member b's tiles from
    int64_t src_stride;       // src + b * src_stride (0: one state for every member) instead of its own state
    int64_t init_basis1;      // 0, or 1 + a basis index: the first fused forward pass starts every member
                              // from that basis state (formed in LDS; the state is not read)
    const QPass* qpasses;     // rotation rounds of the tiled passes (complex64), or null:
    const QPhase* qphases;    // the forward sweep (rb register bits) ...
    const QStep* qsteps;
    const QPass* qrpasses;    // ... and the reverse sweep (rb_rev register bits)
    const QPhase* qrphases;
    const QStep* qrsteps;
    const void* qcoef;        // shear coefficients per (member, step): member b at + b * qsteps_all blocks,
    int32_t qsteps_all, qsteps_fwd;   // forward steps first
};

// job list of a launch; a single job may be passed by value (jobs == nullptr)
struct JobList {
    const Job* jobs;
    const int64_t* prefix;    // [njobs + 1] block offsets
    int32_t njobs, step;
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
// step: forward pass index, reverse step (pass n_passes - 1 - step) or Pauli pass index;
// nthreads: workgroup size (2^(m - RB) of the largest tile among the jobs)
template <typename R, int RB>
hipError_t launch_tile_fwd(const JobList& jl, const Job& single, int64_t blocks, int nthreads, hipStream_t st);
// rounds (R = float: qr = 4 or 5 register bits; R = double: qr = 3 or 4; the job's
// qpasses / qrpasses are set).  launch_rounds_coef fills the coefficient blocks
// (after launch_build_ops); rounds_coef_bytes: bytes per member for `steps` steps.
template <typename R>
hipError_t launch_rounds_coef(const QStep* fsteps, int nf, const QStep* rsteps, int nr, const void* opm, int n_gates,
                              int64_t batch, void* out, hipStream_t st);
template <typename R>
size_t rounds_coef_bytes(int steps);
// fsim: the pass's rounds are fSim rounds (QK_FSIM), else rotation rounds
template <typename R>
hipError_t launch_rounds_fwd(const JobList& jl, const Job& single, int qr, bool fsim, int wgs, int64_t blocks,
                             int nthreads, hipStream_t st);
template <typename R>
hipError_t launch_rounds_rev(const JobList& jl, const Job& single, int qr, bool fsim, int64_t blocks, int nthreads,
                             hipStream_t st);
template <typename R, int RB>
hipError_t launch_tile_rev(const JobList& jl, const Job& single, int64_t blocks, int nthreads, hipStream_t st);
template <typename R, int RB>
hipError_t launch_pauli_tile(const JobList& jl, const Job& single, int64_t blocks, int nthreads, hipStream_t st);

// ---- fused passes (complex64, matrix cores)
// block matrices of every forward phase for every member (float64 products rounded to float32);
// member b reads its constant matrices at cmats + b * cmstride (cmstride 0: one shared set)
hipError_t launch_fused_mats(const FPhase* phases, const Op* ops, int n_blocks, const void* params, int64_t pstride,
                             const void* cmats, int64_t cmstride, int64_t batch, void* out, bool want_rev,
                             hipStream_t st, int kb = FUSED_K);
// blocks: tiles * batch (forward), wgs * batch (reverse)
// m: tile bits of the plan (9..12)
// kb: block bits of the plan (4, or 5 at m = 12)
hipError_t launch_fused_fwd(const JobList& jl, const Job& single, int m, int64_t blocks, hipStream_t st,
                            int kb = FUSED_K);
hipError_t launch_fused_rev(const JobList& jl, const Job& single, int m, int64_t blocks, hipStream_t st,
                            int kb = FUSED_K);
// outer products summed over workgroups (osum: batch * n_blocks * 512), then the
// gate gradient slots slots[b][slot] (total_slots per member)
// one circuit of an uneven batch on the fused passes (batch 1): its plan, angles, constant
// matrices and workspace regions
struct FusedCircJob {
    const FPhase* phases;
    const Op* ops;
    const float* params;      // or null
    const cx<float>* cm;
    float* fmats;             // n_blocks * 2048
    const double* opart;      // n_blocks * wgs * 512
    double* osum;             // n_blocks * 512
    double* slots;            // total_slots
    int32_t n_blocks, wgs, total_slots, pad;
    int64_t pstride;
};
// block matrices of every circuit in one launch (grid: max_blocks x count)
hipError_t launch_fused_multi_mats(const FusedCircJob* jobs, int count, int max_blocks, hipStream_t st);
// outer-product sums and gradient slots of every circuit in two launches
hipError_t launch_fused_multi_grad(const FusedCircJob* jobs, int count, int max_blocks, hipStream_t st);
hipError_t launch_fused_grad(const FPhase* phases, const Op* ops, int n_blocks, const void* params, int64_t pstride,
                             const void* cmats, int64_t batch, const double* opart, int wgs, double* osum,
                             int total_slots, double* slots, hipStream_t st, int kb = FUSED_K);

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

// ---- SU(4) QML step: gate matrices U = exp(-i sum theta_k P_k / 2) (complex64 table [M][16]) and
// dU/dtheta_j (float64 complex [M][15][16]); readout, softmax cross entropy and the adjoint seed
// lambda = diag(dL/dp) psi per member; dL/dtheta from the batch-summed gate cotangents
hipError_t launch_su4(const double* theta, int M, void* utab, double* dutab, hipStream_t st);
hipError_t launch_qml_seed(const void* psi, void* lam, int64_t stride, int n, int64_t batch, int k, int C,
                           const int32_t* labels, double* loss, hipStream_t st);
hipError_t launch_qml_grad(const double* slots, const int32_t* gate_slot, const int32_t* gate_mat, const double* dutab,
                           int n_gates, double* grad, hipStream_t st);

// ---- sparse form of a Pauli sum: entry (g, r) = row row_begin + r, col row ^ gx[g],
// value sum over the group's terms [gstart[g], gstart[g+1]) of tc * (-1)^popcount(col & tz)
hipError_t launch_pauli_coo(const uint64_t* gx, const int32_t* gstart, const uint64_t* tz, const double* tc, int groups,
                            int64_t row_begin, int64_t row_count, int64_t* rows, int64_t* cols, void* vals,
                            hipStream_t st);

// ---- classical-shadow snapshots: per-snapshot rotation tables [S][n][16] (complex64),
// chunk sums [S][shadow_chunks(n)], inverse-distribution draw per snapshot
int shadow_chunks(int n);
hipError_t launch_shadow_mats(const uint8_t* bases, int n, int64_t S, void* mats, hipStream_t st);
hipError_t launch_shadow_chunks(const void* psi, int64_t stride, int n, int64_t S, double* part, hipStream_t st);
hipError_t launch_shadow_pick(const void* psi, int64_t stride, int n, int64_t S, const double* part, const double* u,
                              int64_t* out, hipStream_t st);

// ---- monitored trajectories (complex64): joint histograms of the measured
// qubits (rounds of up to 8 in increasing order, each read filtered by the
// step's earlier outcomes), the Kraus decisions, the per-step collapse.
// Collapse: wgs = mipt_wgs(n) workgroups per member; histograms:
// mipt_hist_wgs(n) per member, mipt_hist_doubles(n, batch) partials.
int mipt_wgs(int n);
int mipt_hist_wgs(int n);
int mipt_rounds(int n);
size_t mipt_hist_doubles(int n, int64_t batch);
// member lists of the rounds after the first: per round a counter and batch
// entries (round r's decisions list the members with a qubit in round r + 1)
size_t mipt_list_words(int n, int64_t batch);
hipError_t launch_mipt_lists_reset(uint32_t* lists, int n, int64_t batch, hipStream_t st);
hipError_t launch_mipt_hist(const void* psi, int64_t stride, int n, int64_t batch, const double* u, int n_steps, int s,
                            double p, int r, const uint32_t* rec, double* part, const uint32_t* lists,
                            hipStream_t st);
hipError_t launch_mipt_decide(const double* u, int n, int n_steps, int s, double p, int r, const double* part,
                              uint32_t* rec, double* keep, double* logp, double* margin, uint32_t* lists,
                              int64_t batch, hipStream_t st);
hipError_t launch_mipt_collapse(void* psi, int64_t stride, int n, int64_t batch, int n_steps, int s,
                                const uint32_t* rec, const double* keep, int wgs, hipStream_t st);
hipError_t launch_zero_u32(uint32_t* p, size_t count, hipStream_t st);

// ---- misc
template <typename R>
hipError_t launch_init(void* state, int64_t stride, int n, int64_t batch, const void* amps_in, int64_t basis,
                       hipStream_t st);

hipError_t launch_zero(double* p, size_t count, hipStream_t st);

// ---- uneven batch: per-circuit descriptors for the op-matrix build and the final sums
struct BuildJob {
    const Op* ops;            // forward plan (every gate once)
    const void* params;
    const void* cmats;
    void* opm;
    int32_t n_ops, pad;
};
struct FinishJob {
    const double* slots;      // row sums of this circuit's gradient partials
    const double* erow;       // row sums of its energy partials
    const int32_t* slot_ptr;
    const int32_t* slot_idx;
    const int32_t* gate_slot;
    const double* u2m;
    const int32_t* gate_mat;
    double* energy;           // one value
    double* grad;             // [n_params] or null
    double* gate_grad;        // [n_gates][15] or null
    int32_t n_params, n_gates, erows, pad;
};
template <typename R>
hipError_t launch_build_ops_multi(const BuildJob* jobs, const int64_t* prefix, int njobs, int64_t total,
                                  hipStream_t st);
// prefix[j]: first output thread of job j (outputs: energy, n_params gradients, n_gates gate rows if gate_grad)
hipError_t launch_finish_multi(const double* part, int64_t prows, int wgs, const double* epart, int64_t erows_total,
                               int ewgs, double* slot_sums, double* erow_sums, const FinishJob* jobs,
                               const int64_t* prefix, int njobs, int64_t total, hipStream_t st);

// grad[b][p] = sum over slots of p of sum_wg part; energy[b] = sum of erows; lie from U2 cotangents.
// scratch: batch * (total_slots + erows) doubles.
hipError_t launch_finish(const double* part, int total_slots, int wgs, const int32_t* slot_ptr,
                         const int32_t* slot_idx, int n_params, const double* epart, int erows, int ewgs,
                         int64_t batch, double* energy, double* grad, double* gate_grad, const int32_t* gate_slot,
                         const double* u2_mats_c128, const int32_t* gate_mat, int n_gates, double* scratch,
                         hipStream_t st);

}  // namespace tcng
