// 2D (n x n Dirichlet) part of the RIDC library: fast-diagonalisation solves on MFMA.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "ridc.h"

namespace ridc {

struct Plan2D;

int plan2d_validate(const ridc_problem* p);
size_t plan2d_workspace_bytes(const ridc_problem* p);
int plan2d_create(const ridc_problem* p, double h, double* const* ring, const int* R,
                  const double* W, const int64_t* woff, char* ws, size_t ws_bytes,
                  hipStream_t stream, Plan2D** out);
void plan2d_destroy(Plan2D* pl);
int plan2d_arm(Plan2D* pl, int64_t nt, hipStream_t stream);
// Advance plans by `steps` pipeline steps; plan i's own step during launch step s is
// sigma_before[i] + s.  Plans sharing (precision, n) share every launch.
int plan2d_advance(Plan2D* const* pls, int count, const int64_t* sigma_before, int64_t steps,
                   hipStream_t stream);
void plan2d_cost(const Plan2D* pl, double* bytes, double* flops);
// Launch shape of the transform passes (bits; every shape gives bitwise the same results):
// kPassWide64 = 64-column waves, 4 per block (FP32/FP64 passes, n/2 a multiple of 64 or no
// fold); kPassNarrowK = 32-wide k-slices in two LDS stages (split-BF16 pass, instead of 64-wide
// slices in one); kPassPlainA = row-major intermediates folded while staging, instead of the
// folded planes the passes otherwise exchange when n is a multiple of 256.
constexpr int kPassWide64 = 1;
constexpr int kPassNarrowK = 2;
constexpr int kPassPlainA = 4;
int plan2d_tile(const Plan2D* pl);
// The shapes this plan's side and precision allow (0 first).
void plan2d_tile_candidates(const Plan2D* pl, std::vector<int>* out);
// Errors: RIDC_E_INVAL for a shape the plan does not allow.
int plan2d_set_tile(Plan2D* pl, int tile);
// Average duration (us) of `reps` back-to-back launches of the second transform pass of step
// `sigma` (every level active; the kind of most passes of a step), after computing that step's
// right-hand side and first pass once.
int plan2d_time_pass(Plan2D* pl, int64_t sigma, int reps, hipStream_t stream, double* us);
// Average duration (us) of `reps` back-to-back launches of the right-hand-side kernel of step
// `sigma` (every level active) and its algorithmic HBM bytes per launch.
int plan2d_time_rhs(Plan2D* pl, int64_t sigma, int reps, hipStream_t stream, double* us,
                    double* bytes);

}  // namespace ridc
