// Internal declarations shared by the eigseis kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>

#include "../../include/eigseis.h"

namespace eig {

constexpr int kNT = EIG_NTHETA;  // seven source parameters
constexpr int kWavesPerBlock = 4;
constexpr int kPitchAlign = 128; // row pitch (nodes) is a multiple of the widest tile
constexpr int kSrcW = 7;         // source window: union of two 6x6 stencils
constexpr int kCoefStride = 16;  // floats per row of a layered coefficient table

// Coefficient slots of a layered table row (all pre-multiplied by
// dt^2 / (rho_k h^2) except kFco = dt^2 / rho_k for the body force).
enum CoefSlot {
    kCxxU = 0,   // (u_{i+1} - 2u + u_{i-1})
    kCzpU = 1,   // (u_{k+1} - u)
    kCzmU = 2,   // (u - u_{k-1})
    kCmpU = 3,   // Dx v at row k+1
    kCmmU = 4,   // Dx v at row k-1
    kCm0U = 5,   // Dx v at row k (traction-free row only)
    kCxxV = 6,
    kCzpV = 7,
    kCzmV = 8,
    kCmpV = 9,   // Dx u at row k+1
    kCmmV = 10,  // Dx u at row k-1
    kCm0V = 11,  // Dx u at row k (traction-free row only)
    kFco = 12,
    kCeP = 13,   // c_p dt / h       (absorbing edges)
    kCeS = 14,   // c_s dt / h
    kCeL = 15,   // lambda dt / (rho c_p h)
};

// Nodal media store, per node, (lambda, mu, dt^2/(rho h^2)) as three float
// planes [3][nz][pitch]; the operator is assembled on the fly.

// One forward solve as seen by the stencil kernel.
struct SolveDesc {
    float2* buf0;            // u at even levels (and u^{-1}) ...
    float2* buf1;            // ... and odd levels; [nz][pitch] (x, depth)
    float2* buf2;            // two-steps-per-launch kernels rotate over four
    float2* buf3;            // buffers: level l in buffer (l + 1) mod 4
    const float* coef;       // layered: [nz][kCoefStride]; nodal: [3][nz][pitch]
    const float* srcw;       // [2][kSrcW][kSrcW] forcing window
    const float* srcs;       // [nsteps] forcing time series
    const int32_t* recmap;   // [pitch]: receiver index of a surface column or -1
    float2* traces;          // [nsteps+1][nrec]
    int32_t nx, nz, pitch, nsteps;
    int32_t start;           // launch index at which this solve takes step 0
    int32_t nrec;
    int32_t src_i0, src_k0;  // window corner (column, row)
    int32_t medium_kind;     // EIG_MEDIUM_*
    float h2;                // h^2 (nodal media scale the body force by s h^2)
    // dual (adjoint) solves only, one-step kernels: force density added at the
    // surface receivers at step m, [nsteps][nrec] (NULL otherwise), and the
    // new level recorded on the forcing window, [nsteps][kSrcW * kSrcW]
    const float2* rforce;
    float2* wrec;
    // three-steps-per-launch kernels: per strip boundary b = 128 (i + 1) and
    // free row k, u^{m+1} and u^{m+2} at columns b-1 and b: [nb][nz][4]
    float2* side;
};

// One forcing table to build (FP64 arithmetic, FP32 result).
struct SourceJob {
    double theta[kNT];
    double step;             // deviation step (unused for nominal)
    double h, dt;
    int32_t param;           // -1 nominal, else the perturbed parameter
    int32_t kx, kz;          // cell of the unperturbed source
    int32_t kx2, kz2;        // cell of the perturbed source
    int32_t i0, k0;          // window corner
    int32_t nsteps;
    int32_t stf;
    int32_t deriv;           // 1: forcing dF/dtheta_param instead of a difference
    float* srcw;
    float* srcs;
};

// Per-sample inputs of the Jacobian / Hessian assembly.
struct SampleDesc {
    const float2* dev[2 * kNT];  // deviation traces: +d_j at 2j, -d_j at 2j+1;
                                 // sensitivity traces at 2j with 2j+1 NULL
    const float2* nominal;
    double inv2d[kNT];           // 1 / (2 d_j)
    double* J;                   // optional output [nt][nrec][2][7]
    int32_t nt, nrec;
    // optional misfit gradient (Gauss-Newton): data y = ystar + sigma noise,
    // grad_j = -sum J_j (y - nominal) / sigma^2 written to grad[7]
    const float2* ystar;
    const float2* noise;
    double* grad;
    // stability check of the sample's step (sample_check only; rho NULL:
    // not checked): its medium's FP64 arrays ([nz] or [nz][nx]) and dt^2/h^2
    const double* rho;
    const double* lam;
    const double* mu;
    int32_t med_kind, nx, nz;
    double dt2_h2;
};

// One H_2 contraction (Theorem 2, through the dual solve of Section 3.3.2):
// H_2 = - sum_n sum_window W psi^{N-n} d^2 F^n / dtheta dtheta.
struct H2Job {
    double theta[kNT];           // theta^ (the MAP point)
    double h, dt;
    int32_t nsteps, stf;
    int32_t kx, kz, i0, k0;      // source cell and window corner
    const float2* wrec;          // dual field on the window, level q at [q-1][49]
    double* H2;                  // [7][7] output
};

struct DualJob {
    const float2* ystar;         // truth traces g(theta*) [N+1][nrec]
    const float2* noise;         // standard normal draws [N+1][nrec]
    const float2* ghat;          // traces at the MAP point [N+1][nrec]
    float2* rforce;              // [N][nrec] output
    double sigma, w_inv;
    int32_t nsteps, nrec;
};

// Looks up (once per device, with that device current) the device address
// of the file-scope scratch array that design_greedy_noalloc works in.
int noalloc_scratch_init(int device);

// launchers (all asynchronous on `s`)
void launch_fill_zero(void* p, size_t bytes, hipStream_t s);
void launch_layered_coef(const double* rho, const double* lam, const double* mu,
                         int nz, double h, double dt, float* coef, hipStream_t s);
void launch_nodal_coef(const double* rho, const double* lam, const double* mu,
                       int nx, int nz, int pitch, double h, double dt, float* coef,
                       hipStream_t s);
void launch_source_tables(const SourceJob* jobs, int njobs, int max_nsteps,
                          hipStream_t s);
// Stencil kernel variants: tile geometry (columns x rows per wavefront) and
// the medium kind they serve.  All variants of a medium kind produce
// bitwise-identical results; they differ only in speed.
struct StencilVariant {
    int cols, rows, medium_kind;
    int steps;  // leapfrog steps per launch (2, 3, 4: four field buffers per solve)
    int edges;  // 1: runs edge tiles (absorbing edges in the same launch)
    int resident;  // 1: one workgroup per solve, fields in LDS, all steps in one launch
    int forced_only;  // 1: runs only when forced (not a tuning candidate)
};
// Tile entries (solve, kEdgeStrip << 16 | part) of a variant with `edges`:
// absorbing edge nodes part * kEdgeTileNodes .. +kEdgeTileNodes of a solve.
constexpr int kEdgeStrip = 0x7fff;
constexpr int kEdgeTileNodes = 128;
inline int edge_tiles_of(int nx, int nz) {
    return (2 * nz + nx - 2 + kEdgeTileNodes - 1) / kEdgeTileNodes;
}
constexpr int kNumVariants = 26;
extern const StencilVariant kVariants[kNumVariants];
// tiles: (solve index, strip << 16 | chunk) per wavefront
void launch_stencil(const SolveDesc* descs, const int2* tiles, int ntiles, int step,
                    int variant, hipStream_t s);
// Tiled depth-only variants (0..5, 7..16) of launch_stencil.
void launch_layered_stencil(const SolveDesc* descs, const int2* tiles, int ntiles, int step,
                            int variant, hipStream_t s);
// Variants 23 (depth-only) and 24, 25 (nodal) of launch_stencil: K steps
// per launch with the tile in LDS, one workgroup per tile.
void launch_blocked_stencil(const SolveDesc* descs, const int2* tiles, int ntiles, int pass,
                            int variant, hipStream_t s);
// Nodal-media variants (6, 17..20) of launch_stencil.
void launch_nodal_stencil(const SolveDesc* descs, const int2* tiles, int ntiles, int step,
                          int variant, hipStream_t s);
void launch_zero_level0(const SolveDesc* descs, int n, hipStream_t s);
// Resident solves: both field levels of a solve in one workgroup's LDS
// (2 nx nz float2, the forcing window weights and for depth-only media the
// nz x kCoefStride float coefficient table, at most kResidentLdsBytes);
// tiles are (solve, absorbing) pairs, one workgroup each, and one launch
// takes every step.
constexpr size_t kResidentLdsBytes = (size_t)160 << 10;
constexpr int kResSrcwFloats = 128;  // forcing window weights (2 x 7 x 7, padded)
constexpr int kResidentMaxEdge = 3 * 1024;  // edge nodes: three per thread at most
inline size_t resident_lds_bytes(int kind, int nx, int nz) {
    return (size_t)nx * nz * 2 * sizeof(float2) + kResSrcwFloats * sizeof(float) +
           (kind == EIG_MEDIUM_LAYERED ? (size_t)nz * kCoefStride * sizeof(float) : 0);
}
void launch_resident(const SolveDesc* descs, const int2* tiles, int ntiles, int kind,
                     size_t lds_bytes, hipStream_t s);
// Halo values of the three-steps-per-launch kernels; htiles: (solve,
// boundary << 16 | 64-row chunk).
void launch_tb3_halo(const SolveDesc* descs, const int2* htiles, int nhtiles, int pass,
                     hipStream_t s);
// Nested Monte Carlo log ratios (and their mean when eig != NULL); work
// holds nested_workspace() bytes: per-split partial sums, squared norms, and
// FP64 k-major copies of the outer data and inner outputs.
int nested_splits(int nouter, int ninner);
size_t nested_workspace(int nouter, int ninner, int nobs);
void launch_nested(const float* gout, const float* noise, const float* gin, int nouter,
                   int ninner, int nobs, double sigma, double* logratio, double* eig,
                   double* work, hipStream_t s);
// Absorbing-edge update of level step+1 for descs[0..n) (one-step buffers).
void launch_ce_edges(const SolveDesc* descs, int n, int step, hipStream_t s);
// Per-sample checks and H_1: each sample's (level, receiver) elements are cut
// into contiguous ranges of at least kRangeMin elements, at most kSampleSplit
// of them, one block each, and the block partials are combined in range
// order by a second kernel.  The cut depends only on the sample's element
// count, so a sample's result does not depend on the batch it runs in.
// work: sample_work_bytes(nsample) of device scratch (the two launches may
// share it in stream order).
constexpr int kSampleSplit = 16;
constexpr int kRangeMin = 4096;
inline size_t sample_work_bytes(int nsample) {
    return (size_t)nsample * kSampleSplit * (kNT * (kNT + 1) / 2 + kNT) * sizeof(double);
}
void launch_sample_check(const SampleDesc* samples, int nsample, const double* given,
                         int mode, double* sigma, int32_t* status, double* work,
                         hipStream_t s);
// Per-receiver H_1 (per_receiver != 0): each sample's levels are cut into
// at most kRecvSplit ranges of at least kRecvLevelsMin levels; work holds
// receiver_stride doubles per sample (receiver_work_doubles of the largest).
constexpr int kRecvSplit = 32;
constexpr int kRecvLevelsMin = 125;
inline size_t receiver_work_doubles(int nt, int nrec) {
    const int nb = std::min(kRecvSplit, std::max(1, nt / kRecvLevelsMin));
    return (size_t)nb * (kNT * (kNT + 1) / 2) * (size_t)nrec;
}
void launch_hessian(const SampleDesc* samples, int nsample, int per_receiver,
                    int ngroup, const double* sigma, double* H1, double* work, hipStream_t s,
                    size_t receiver_stride = 0);
void launch_laplace(const double* H1, int nsample, const eig_prior* prior_dev,
                    const double* theta, const double* w, double* dkl,
                    double* logdet, int32_t* status, double* eig, hipStream_t s);
void launch_design_eval(const double* H1r, int nsample, int ncand,
                        const uint8_t* mask, int ndesign,
                        const eig_prior* prior_dev, const double* theta,
                        const double* w, double* work, double* eig, hipStream_t s);
void launch_greedy_step(const double* H1r, int nsample, int ncand,
                        const eig_prior* prior_dev, const double* theta,
                        const double* w, double* Hcur, uint8_t* chosen,
                        double* work, double* ival, int k, int32_t* order,
                        double* curve, hipStream_t s);
void launch_surface_peak(const float2* traces, int count, double rel,
                         double* out, hipStream_t s);
void launch_h2(const H2Job* jobs, int njobs, hipStream_t s);
// Receiver forcing of the dual solves, one job per solve:
// rforce[s][r] = w_inv * ((ystar - ghat) + sigma noise)[N - s][r] / sigma^2,
// s = 0..N-1 (traces [N+1][nrec]); max_elems = the largest N * nrec.
void launch_dual_force(const DualJob* jobs, int njobs, size_t max_elems, hipStream_t s);
// Theorem 3 integrand per sample and the weighted average.
void launch_theorem3(const double* H1, const double* H2, int nsample,
                     const eig_prior* prior_dev, const double* theta_hat, const double* w,
                     double* val, int32_t* status, double* eig, hipStream_t s);

}  // namespace eig
