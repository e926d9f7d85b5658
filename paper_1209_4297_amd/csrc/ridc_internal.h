// Internal declarations shared by the host runtime and the HIP kernels of the RIDC library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "ridc.h"

namespace ridc {

constexpr int kMaxPcr = 48;

// Coefficient of the explicit stencil of f_E: a/(2h) (centred advection), a/h (upwind),
// 1/(4h) (Burgers flux), unused otherwise.
inline double explicit_coeff(int fe, double a, double h) {
  if (fe == RIDC_FE_ADVECT_C2) return a / (2.0 * h);
  if (fe == RIDC_FE_ADVECT_UPWIND) return a / h;
  if (fe == RIDC_FE_BURGERS) return 1.0 / (4.0 * h);
  return 0.0;
}          // PCR stages kept in a level descriptor
constexpr int kMaxOrder = RIDC_MAX_ORDER;

// ---------------------------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define RIDC_HIP_TRY(expr)                                                             \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return ::ridc::fail(RIDC_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// ---------------------------------------------------------------------------------------------
// plan helpers (plan.cpp)
// ---------------------------------------------------------------------------------------------
// Quadrature weights of corrector j, start-up row r, in units of dt (ascending nodes), from
// exact rational arithmetic.
bool quadrature_weights(int j, int r, double* out);

// PCR plan for (I - r D2) on a cycle of length m: stage coefficients gamma_k = a_k / b_k,
// the shift of each stage modulo m, and the final divisor.  `exact` is true when the stages end
// with a diagonal system (2^K = 0 mod m) rather than a negligible coupling.
struct PcrPlan {
  int stages = 0;
  bool exact = false;
  double divisor = 1.0;
  double gamma[kMaxPcr];
  int64_t shift[kMaxPcr];
};
bool pcr_plan(double r, int64_t m, PcrPlan* out);

// IMEX pairs (section II) as doubles from exact rationals: s stages, order, the stiff and
// explicit tableaux and the abscissae (also as multiples of 1/6).
constexpr int kMaxStages = 7;
struct ImexPair {
  int s = 0, order = 0;
  double AS[kMaxStages][kMaxStages];
  double AN[kMaxStages][kMaxStages];
  double c[kMaxStages];
  int32_t c6[kMaxStages];
};
bool imex_pair(int pair, ImexPair* out);

// Lagrange basis on the S nodes 0..S-1 at x = r + c6/6 (interp) and its integral over
// [r, r + c6/6] (quad), from exact integer arithmetic, rounded once.
bool stage_weights(int S, int r, int c6, double* interp, double* quad);

// Ring slots of level j in a P-level pipeline: 2j+3 for j < P-1 (the live window that level
// j+1 reads plus the slot being written), 2 for the top level.
inline int ring_slots(int j, int P) { return j == P - 1 ? 2 : 2 * j + 3; }

// ---------------------------------------------------------------------------------------------
// 1D level-step descriptor: one (instance, level) work item, static for a handle
// ---------------------------------------------------------------------------------------------
struct Lvl1D {
  double* own;             // ring of this level (R_own slots of n values)
  const double* prev;      // ring of level j-1 (R_prev slots), null for j = 0
  const double* W;         // weights of this level: j rows x (j+1), ascending nodes
  int64_t nt;              // time steps of the integration
  int64_t sigma0;          // pipeline step at which this instance's step 0 sits
  int32_t n, j, R_own, R_prev;
  int32_t bc, fe;          // ridc_bc, ridc_fe_kind
  int32_t stages;          // PCR stages
  int32_t wrap;            // 1: whole cycle in one workgroup; 0: chunk + halo
  int32_t M;               // cycle length (periodic n, Dirichlet 2n+2)
  int32_t B;               // rows per chunk (chunk mode)
  int32_t H;               // halo rows each side (chunk mode) = 2^stages - 1
  int32_t nchunks;
  double dt;
  double ce;               // coefficient of the explicit stencil (see explicit_coeff)
  double nu_h2;            // nu / h^2
  double inv_divisor;      // 1 / final PCR divisor
  double gamma[kMaxPcr];
  int32_t shift[kMaxPcr];  // 2^k mod M
};

// The descriptor of a single instance's step, passed by value in the kernel arguments.
struct Solo1D {
  double* ring[kMaxOrder];     // level rings
  const double* W[kMaxOrder];  // weights per level (j rows x (j+1))
  const double* gamma;         // PCR stage coefficients (device)
  const int32_t* shift;        // PCR stage shifts (device)
  int32_t R[kMaxOrder];        // ring slots per level
  int64_t nt;
  int32_t nchunks, n, M, bc, fe, stages, wrap, B, H, nt_store;
  double dt, ce, nu_h2, inv_divisor;
};

// One instance integrated by the fused kernel (one workgroup): pipeline steps
// sigma_first+1 .. sigma_last of its own schedule (own step = sigma - sigma0).
constexpr int kMaxJ1024 = 5;   // highest level index instantiated in 1024-thread kernels
struct Fused1D {
  double* ring[kMaxOrder];
  const double* W[kMaxOrder];
  const double* gamma;
  const int32_t* shift;
  int32_t R[kMaxOrder];
  int64_t nt, sigma0, sigma_first, sigma_last;
  int32_t P, group, n, M, bc, fe, stages, pad;
  double dt, ce, nu_h2, inv_divisor;
};

struct Blk1D {
  int32_t item;
  int32_t chunk;
};

// Allow `lds_bytes` of dynamic LDS for the level-step kernels with `threads` threads that cover
// orders up to max_order (host call, made when a tiling is chosen, never inside graph capture).
hipError_t prepare_1d_step(int threads, int max_order, size_t lds_bytes);

// Launch one pipeline step of a grouped 1D batch whose highest order is max_order.
hipError_t launch_1d_step(const Lvl1D* d_items, const Blk1D* d_blocks, int nblocks, int threads,
                          int max_order, size_t lds_bytes, int64_t sigma, hipStream_t stream);

// Launch one pipeline step of a single instance of order max_order (descriptor in the kernel
// arguments); block b covers level b / nchunks, chunk b % nchunks.
hipError_t launch_1d_solo(const Solo1D& a, int nblocks, int threads, int max_order,
                          size_t lds_bytes, int64_t sigma, hipStream_t stream);

// Launch the fused integration of `count` instances (one workgroup of `threads` = 512 or 1024
// each, two LDS buffers of n (periodic) or n+2 (Dirichlet) doubles per level, level groups of
// Fused1D::group = (threads / P) rounded down to whole waves).  `one` (nullable): a single instance whose descriptor goes in the
// kernel arguments; otherwise d_items holds `count` device descriptors.  max_order: the
// largest order among the instances (at most kMaxJ1024 + 1; at most 4 with 1024 threads).
hipError_t launch_fused_1d(const Fused1D* d_items, const Fused1D* one, int count, int max_order,
                           int threads, size_t lds_bytes, hipStream_t stream);

// One vector copy of a batched copy launch: dst[0..n) = src[0..n); if flag is not null, *flag is
// set to 1 when a copied value is not finite.
struct CopyItem {
  const double* src;
  double* dst;
  int64_t n;
  int* flag;
};

// Copy every item of d_items[0..count) (count <= 65535; max_n: the longest item) in one launch.
hipError_t launch_copy_items(const CopyItem* d_items, int count, int64_t max_n,
                             hipStream_t stream);

// Set *flag to 1 if any of x[0..count) is not finite.
hipError_t launch_nonfinite_check(const double* x, int64_t count, int* flag, hipStream_t stream);

// LDS bytes a 1D item needs.
size_t lds_bytes_1d(const Lvl1D& it);

// ---------------------------------------------------------------------------------------------
// IMEX level step (kernels_imex1d.hip): ARK-based RIDC and a nonlinear stiff term, 1D
// ---------------------------------------------------------------------------------------------
constexpr int kImexMaxThreads = 512;   // threads per workgroup at most
constexpr int kImexMaxRows = 16;       // rows per thread at most: n <= 8192

// One (instance, level) work item.  The level computes t_m, m = sigma - sigma0 - delay, at
// launch step sigma (1 <= m <= nt).
struct ImexLvl {
  double* own;            // level values: R_own slots of n
  double* ownF;           // f^S + f^N of the level values, same slots; null for the top level
  const double* prev;     // previous level's values (R_prev slots); null for the predictor
  const double* prevF;    // previous level's f
  const double* wt;       // corrector weights: [row r = 0..S-2][stage i][interp S, quad S]
  double* ks;             // stage workspace: K^S_l, K^N_l (l < s-1), then 3 scratch vectors
  int64_t nt, sigma0, delay;
  int32_t n, j, s, S;     // unknowns, level, stages of the pair, window nodes (corrector)
  int32_t R_own, R_prev;
  int32_t bc, fe, fs, maxit;
  double dt, ce, nu_h2, kappa;
  double AS[kMaxStages][kMaxStages];
  double AN[kMaxStages][kMaxStages];
};

// Rows per thread (2, 4, 8 or 16) and threads per workgroup (a multiple of 64, at most 512)
// of the IMEX level step for n unknowns.
void imex_shape(int64_t n, int* M, int* threads);

// One launch over d_items[0..count) (all of the shape M, threads and of one boundary kind) at
// launch step sigma; init: instead, write f of every level's initial value (slot 0).
hipError_t launch_imex1d(const ImexLvl* d_items, int count, int M, int threads, bool periodic,
                         int64_t sigma, bool init, hipStream_t stream);

// ---------------------------------------------------------------------------------------------
// persistent table of measured launch shapes (tune.cpp)
// ---------------------------------------------------------------------------------------------
// 1D level-step tiling per (n, boundary, PCR stages), as ridc_set_tile's (threads, rows, flags)
bool tune_get_1d(int64_t n, int bc, int stages, int* threads, int* rows, int* flags);
void tune_put_1d(int64_t n, int bc, int stages, int threads, int rows, int flags);
// grouped 1D tiling, as ridc_set_batch_tile's (threads, rows)
bool tune_get_batch(int* threads, int* rows);
void tune_put_batch(int threads, int rows);
// 2D transform-pass shape per (n, precision)
bool tune_get_2d(int64_t n, int prec, int* tile);
void tune_put_2d(int64_t n, int prec, int tile);
int tune_save(const char* path);   // nullptr: the default file
int tune_load(const char* path);
void tune_clear();

// ---------------------------------------------------------------------------------------------
// allocation-free 1D integration (noalloc.hip): a fixed scratch array per GPU
// ---------------------------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;   // 32 MiB per GPU
constexpr int kNoAllocMaxOrder = 6;
constexpr int kNoAllocWeights = 70;          // sum of j(j+1) over j = 1..5
constexpr size_t kNoAllocWeightsOffset = 0;
constexpr size_t kNoAllocGammaOffset = 1024;
constexpr size_t kNoAllocShiftOffset = 1536;
constexpr size_t kNoAllocRingsOffset = 4096;

// Tables written into the scratch array by one small kernel (passed by value, so the call
// needs no host staging buffer).
struct NoAllocTables {
  double w[kNoAllocWeights];   // weights of levels 1..P-1, level after level (j rows of j+1)
  double gamma[kMaxPcr];
  int32_t shift[kMaxPcr];
  int32_t nw, stages;
};

// Device address of this GPU's scratch array (looked up once per device, on first use).
int noalloc_scratch(void** ptr);

// Write the weight and PCR tables into the scratch array at `base`.
hipError_t launch_noalloc_tables(const NoAllocTables& t, void* base, hipStream_t stream);

}  // namespace ridc
