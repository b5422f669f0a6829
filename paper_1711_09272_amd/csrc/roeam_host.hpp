// roeam_host.hpp -- host-side objects behind the opaque C handles, shared by
// the runtime and batch-engine translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/roeam.h"
#include "roeam_internal.hpp"

using roeam::DevSolve;
using roeam::Slot;

constexpr int kStepsPerGraph = 50;

struct GraphCache {
    bool valid = false;
    const double *q = nullptr;
    roeam_params params{};
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int chunk = 0;
    int shape = 0;
    void release()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        valid = false;
    }
};

struct BatchEngine;

struct roeam_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err = "no error";
    BatchEngine *batch = nullptr;
};

struct roeam_grid {
    roeam_ctx *ctx = nullptr;
    int nx = 0, ny = 0;
    long long pitch = 0;
    int metric = 0;
    double dx = 0, dy = 0;
    double *d_xn = nullptr, *d_yn = nullptr;
    int bc[4] = {0, 0, 0, 0};
    double bcq[4][4] = {};
    double spl_a[4] = {HUGE_VAL, HUGE_VAL, HUGE_VAL, HUGE_VAL};  // moving sides: split at a + b t
    double spl_b[4] = {0, 0, 0, 0};
    int spl_hi[4] = {ROEAM_BC_SLIPWALL, ROEAM_BC_SLIPWALL, ROEAM_BC_SLIPWALL, ROEAM_BC_SLIPWALL};
    int spl_lo[4] = {ROEAM_BC_DIRICHLET, ROEAM_BC_DIRICHLET, ROEAM_BC_DIRICHLET, ROEAM_BC_DIRICHLET};
    double bcq_hi[4][4] = {};                    // moving sides: conserved state above the split
    double t_res = 0.0;                          // time of moving sides in roeam_residual
    int nsc = 0;                                 // transported scalars (rows 4 .. 3 + nsc)
    double bcs[4][roeam::kMaxScalars] = {};      // Dirichlet rho k_m per side
    double *d_qa = nullptr, *d_qb = nullptr;
    Slot *d_slot = nullptr;
    Slot *h_slot = nullptr;  // pinned readback
    GraphCache gc;
    int shape_forced = -1;   // tile shape set by the caller, or -1
    int shape_tuned[2][2] = {{-1, -1}, {-1, -1}};  // autotuned shape per [order-1][precision]
    int final_parity = 0;    // parity of the step state after the last roeam_step
    double *d_norm_part = nullptr;  // scratch of roeam_residual_norms (allocated at its first call)
    DevSolve *d_solve = nullptr;  // descriptor read by the single-grid kernels
    DevSolve *h_solve = nullptr;  // pinned staging copy of the last descriptor sent
    bool solve_valid = false;
};

roeam_status roeam_fail(roeam_ctx *ctx, roeam_status st, const std::string &msg);
roeam_status roeam_check_params(roeam_ctx *ctx, const roeam_params *p, bool need_cfl);
// Descriptor of a solve on grid g with parameters p and state buffers q, qa, qb.
DevSolve roeam_make_solve(const roeam_grid *g, const roeam_params *p, double *q, double *qa, double *qb, Slot *slot);
