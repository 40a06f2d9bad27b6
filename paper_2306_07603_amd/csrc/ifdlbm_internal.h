// ifdlbm_internal.h -- launch interface between the C-ABI host code and the
// kernels of libifdlbm.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "lbm_device.h"

namespace ifd {

// A block of 256 consecutive nodes (in [j][i] order) of one cavity: the work
// unit of the per-node kernels (initialisation, staged step, residual, output).
struct NodeBlock {
    int32_t cav;     // index into the descriptor table
    int32_t first;   // first node, j * nx + i
};
constexpr int kNodeBlock = 256;

// A wavefront work item of the fused step: output columns [i0, i1) and output
// rows [j0, j1) of one cavity.  The 64 lanes cover columns [i0 - 4, i0 + 60),
// so i1 - i0 <= kStripOut.  Strips and row segments split a cavity evenly and
// hold at least two columns and rows, so a wall node and its inward
// neighbour always belong to the same item.
constexpr int kStripOut = 56;
constexpr int kWaveLanes = 64;
constexpr int kHaloCols = 4;
struct StripItem {
    int32_t cav;
    int16_t i0, i1;
    int32_t j0, j1;
    int32_t unit;   // slot of its residual partial sums (items of a cavity are consecutive slots)
};

// Residual partial sums of Eq. (2.19) per work unit:
//   0 sum |u_new - u_old|^2        1 sum |u_new|^2
//   2 sum (P_new - P_old)^2        3 sum P_new^2          (E(P) as printed)
//   4 sum (dP - r_d)               5 sum (P_new - r_p)
//   6 count of non-finite nodes
//   7 sum (dP - r_d)^2             8 sum (P_new - r_p)^2
// with dP = P_new - P_old and per-cavity shifts r_d, r_p (the means found at
// the previous evaluation).  Sums 4, 5, 7, 8 give E(P) of the pressure with
// its spatial mean removed, sum (x - r)^2 - (sum (x - r))^2 / n per variance:
// the shift keeps the subtraction from cancelling when the mean is far larger
// than the spread, as the per-step change of a drifting pressure level is.
constexpr int kPartials = 9;
// Per-cavity record of a residual evaluation: the kPartials sums, then the
// shifts r_d, r_p they were taken with.
constexpr int kResult = kPartials + 2;

struct StepArgs {
    const void* f_in;        // distributions, storage type, step start
    void* f_out;             // distributions, storage type, step end
    const void* l_in;        // lambda, step start
    void* l_out;             // lambda, step end
    const CavityDesc* desc;  // per-cavity descriptors
    const double* geo;       // metric tables a_j, s_i (FP64)
    const float* geo32;      // the same tables rounded to FP32
    double* partial;         // residual partials, kPartials per work unit
    const double* res_ref;   // per-cavity shifts (r_d, r_p) of the residual sums
    // staged schedule only: temporaries in the arithmetic type
    void* hat_plus;          // f-hat+ (Eq. 2.15), 9 planes
    void* bar_plus;          // f-bar+ (Eq. 2.16), then f(t + dt/2) (Eq. 2.17), 9 planes
    void* bar_half;          // f-bar(t + dt/2) (Eq. 3.7), 9 planes
    void* lam_new;           // lambda of this step
    // stochastic rounding: seed of this launch = mix of *seed_ctr and step
    const uint32_t* seed_ctr;
    uint32_t step;
};

// Advance the device seed counter by one (a one-thread kernel, graph-safe).
hipError_t launch_seed_bump(uint32_t* ctr, hipStream_t s);

// Staged schedule: five launches per step over the node blocks
// [b0, b0 + nb), plus the residual launch when `residual` is set.
hipError_t launch_staged_step(int prec, const StepArgs& a, const NodeBlock* blocks, int b0, int nb,
                              bool residual, hipStream_t s);

// Fused schedule: one launch over the strip items [w0, w0 + nw).
hipError_t launch_fused_step(int prec, bool implicit_lambda, const StepArgs& a, const StripItem* items, int w0, int nw,
                             bool residual, hipStream_t s);

// Step (1) on every node of the listed blocks.
hipError_t launch_init(int prec, void* f, void* l, const CavityDesc* desc, const NodeBlock* blocks, int nb,
                       hipStream_t s);

// Per-cavity deterministic reduction of residual partials:
// out[c * kResult + q] = sum over units [first[c], first[c] + count[c]) for
// q < kPartials, then the shifts ref[2 c], ref[2 c + 1] the sums were taken
// with; ref is then moved to the means of dP and P found (when finite).
hipError_t launch_reduce_partials(const double* partial, const int32_t* first, const int32_t* count,
                                  const CavityDesc* desc, int n_cav, double* ref, double* out, hipStream_t s);

// u, v, P (FP64 or FP32 by dtype) of one cavity, [j][i] packed.
hipError_t launch_fields(int prec, const void* f, const CavityDesc* desc, int cav_index, const CavityDesc& hd,
                         void* u, void* v, void* p, int dtype, hipStream_t s);

// f-hat (rho0 included, FP64, [k][j][i] packed) and lambda of one cavity to / from the state.
hipError_t launch_state_out(int prec, const void* f, const void* l, const CavityDesc& hd, double rho0,
                            double* fhat, double* lam, hipStream_t s);
hipError_t launch_state_in(int prec, void* f, void* l, const CavityDesc& hd, double rho0,
                           const double* fhat, const double* lam, hipStream_t s);

// Kinetic energy of Eq. (5.1) summed per block, reduced on the host in order.
hipError_t launch_energy(int prec, const void* f, const CavityDesc* desc, const double* geo, int cav_index,
                         const CavityDesc& hd, double* partial, hipStream_t s);

// Probe record of every cavity (centre velocity and kinetic energy of Eq. 5.1)
// into slot *rec_count % capacity, then *rec_count + 1; blocks [0, nb) are all
// node blocks, first/count their range per cavity, partial nb doubles.
hipError_t launch_probe(int prec, const void* f, const CavityDesc* desc, int n_cav, const NodeBlock* blocks, int nb,
                        double* partial, const int32_t* first, const int32_t* count, double* rec, uint32_t* rec_count,
                        int capacity, hipStream_t s);

// Tangent-linear kinetic energy of one cavity after n_steps (see ifdlbm_gradient).  The work arrays
// (tangent_workspace_elems values of three-component duals) are allocated and freed inside the call, or with
// use_scratch taken from the current device's file-scope scratch array, which holds
// tangent_scratch_capacity_elems of them.
hipError_t tangent_kinetic_energy(int nx, int ny, double re, double n, double theta_deg, double u_lid, double cfl,
                                  double mix, double gamma_min, int dt_rule, int64_t n_steps, hipStream_t s, double* J,
                                  double* grad, std::string& err, bool use_scratch);
size_t tangent_workspace_elems(int nx, int ny);
size_t tangent_scratch_capacity_elems();

// Reverse (discrete adjoint) sweep of one cavity's step in FP64.  A state is
// 9 planes of f-hat deviations then the Lambda plane, [k][j][i] packed, as
// launch_state_out writes it with rho0 = 0.  Call init once, objective on the
// final state, step_back(state t, state t + 1) for t = T - 1 down to 0, then
// finish for J and dJ/d(theta [rad], n, u_lid).
class AdjointSweep {
public:
    AdjointSweep();
    ~AdjointSweep();
    AdjointSweep(const AdjointSweep&) = delete;
    AdjointSweep& operator=(const AdjointSweep&) = delete;
    hipError_t init(const CavityDesc& c, hipStream_t s);
    hipError_t objective(const double* state, hipStream_t s);
    hipError_t step_back(const double* st, const double* st1, hipStream_t s);
    // dt_dcot, lam0_dU, K_dn, K_dU: derivatives of the handle's parameter rules
    hipError_t finish(const CavityDesc& c, double dt_dcot, double lam0_dU, double K_dn, double K_dU, hipStream_t s,
                      double* J, double grad[3]);

private:
    struct Impl;
    Impl* d;
};

}  // namespace ifd
