// 2D (n x n, zero Dirichlet) part of the RIDC pipeline for gfx950.
//
// Every level step is taken in increment form, which is algebraically the step of the paper:
//   predictor (section II, eq. imex_diffusion):
//     (I - dt L) d = dt (f_E + L)(eta[0]_n),               eta[0]_{n+1} = eta[0]_n + d
//   corrector (section III-C, eq. corr, with the (j+1)-node quadrature Q of f along level j-1):
//     (I - dt L) e = eta[j]_n - eta[j-1]_{n+1} + dt Q + dt [f_E(eta[j]_n) - f_E(eta[j-1]_n)],
//     eta[j]_{n+1} = eta[j-1]_{n+1} + e
// (subtract (I - dt L) eta[j-1]_{n+1}, resp. (I - dt L) eta[0]_n, from both sides of the
// paper's equation).  The right-hand side is small (O(dt) resp. O(dt^j)), so the rounding of
// the transforms scales with the increment, not with u; the sums and level differences are
// FP64 in every precision.
//
// Solve: fast diagonalisation.  With the orthonormal type-I sine matrix Q (symmetric,
// Q_{ik} = sqrt(2/(n+1)) sin(pi (i+1)(k+1)/(n+1))) and mu_k = (4/h^2) sin^2(pi (k+1)/(2(n+1))),
// (I - dt nu Lap_h)^{-1} B = Q [(Q B Q) ./ (1 + dt nu (mu_i + mu_k))] Q.
// Each product by Q is one pass C = (A Q)^T: two passes give Q B Q in the original orientation.
// A pass is a GEMM on the matrix cores (v_mfma_f64_16x16x4f64, v_mfma_f32_16x16x4f32, or three
// v_mfma_f32_16x16x32_bf16 products of hi/lo BF16 splits), batched over every active level of
// every instance in one launch; the eigenvalue divide and the final update are fused into the
// epilogues of passes 2 and 4.  Sides that are multiples of 64 fold Q by its reflection
// symmetry, Q_{n-1-k, j} = (-1)^j Q_{k, j}, which halves the contraction (k_pass2d).  When n is
// a multiple of 256 the passes of a solve hand each other their intermediates already folded
// (sums and differences of mirrored columns; split into BF16 hi/lo on the split-BF16 path);
// otherwise, and for the first pass of a solve, the intermediates are row-major (FP32 on the
// reduced-precision paths) and a pass folds (and splits) its operand while staging it.
//
// Reduced precision (FP32 or split BF16) adds one FP64 residual refinement:
//   x1 = S~(b),  rho = b - (x1 - dt nu Lap_h x1)  (FP64 5-point),  x = x1 + S~(rho);
// x1 is held in FP32: the pass that produces it accumulates in FP32 (no divide), so x1 is an
// FP32 value and storing it in FP32 loses nothing.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>

#include "ridc2d.h"
#include "ridc_internal.h"

namespace ridc {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2 };
enum { OUT_F64 = 0, OUT_F32 = 1, OUT_FINAL = 3, OUT_FOLD = 4 };

// One (instance, level) of the 2D pipeline: static for a handle.
struct Lvl2D {
  double* own;          // ring of this level (R_own slots of n*n)
  const double* prev;   // ring of level j-1 (null for j = 0)
  const double* W;      // weights, j rows x (j+1)
  double* b64;          // FP64 right-hand side (kept for the residual)
  double* x64;          // FP64 first solve (refinement) or FP64 intermediate
  void* lo0;            // FP32-sized buffers of the reduced-precision paths (row-major FP32 or
                        // folded planes)
  void* lo1;
  int64_t nt, sigma0;
  int32_t n, j, R_own, R_prev, fe, prec;
  double dt, nu_h2;
};

// One batch entry of a transform pass.
struct Pass2D {
  const void* A;        // input: row-major n x n (FP64, or FP32 in the reduced-precision paths),
                        // or the folded planes of the previous pass
  void* C;              // output (unless final)
  const float* add;     // final epilogue: extra term (x1 of the refinement, FP32), nullable
  const void* Q;        // transform matrix in the input precision (BF16: hi, lo at +n*n)
  const double* lam;    // dt nu mu_k (divide epilogue)
  int32_t level;        // index into the level table
  int32_t divide;       // divide by 1 + lam_i + lam_k
};

struct Plan2D {
  ridc_problem p{};
  int P = 1, prec = 0;
  int64_t n = 0;
  double h = 0;
  std::vector<Lvl2D> levels;        // host copy (nt filled at arm)
  Lvl2D* d_levels = nullptr;
  // pass tables: npass passes x P entries, device
  int npass = 0;
  std::vector<Pass2D> passes;
  Pass2D* d_passes = nullptr;
  // transform data (shared per n)
  const double* Q64 = nullptr;
  const float* Q32 = nullptr;
  const u16* Qbf = nullptr;         // hi then lo
  double* lam = nullptr;
  hipStream_t stream = nullptr;
  int tile = 0;                     // pass launch shape: kPassWide64 | kPassNarrowK (results
                                    // are bitwise the same for every shape)
};

// ---------------------------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ bool level_active(const Lvl2D& L, int64_t sigma, int64_t* m_out) {
  const int64_t m = sigma - L.sigma0 - (int64_t)L.j * (L.j + 1) / 2;
  *m_out = m;
  return m >= 1 && m <= L.nt;
}

__device__ __forceinline__ double fe2(int fe, double u) {
  return fe == RIDC_FE_LOGISTIC ? u * (1.0 - u) : 0.0;
}

// Loads and stores through pointers read from the launch tables.  The compiler cannot tell
// their address space and would emit flat instructions, which also count against the LDS wait
// counter (every LDS wait would then wait for the outstanding global loads too); these name the
// global space.
template <typename V>
__device__ __forceinline__ V gld(const void* p) {
  return *(const __attribute__((address_space(1))) V*)p;
}
template <typename V>
__device__ __forceinline__ void gst(void* p, V v) {
  *(__attribute__((address_space(1))) V*)p = v;
}

// The FP32 copy of a right-hand side or residual that the first pass of a reduced-precision
// solve reads (row-major; that pass folds it, and the split-BF16 pass splits it, while staging).
__device__ __forceinline__ void store_lo(void* base, int64_t idx, double v) {
  gst<float>((float*)base + idx, (float)v);
}

// ---------------------------------------------------------------------------------------------
// stencil kernels: a wave owns 64 columns of ST_RY consecutive rows and walks down them, keeping
// the rows above and below in registers, so each stencil vector is read once per point.  Column
// neighbours come from the adjacent lanes (DPP wave shifts); the columns just outside the wave's
// 64, which lanes 0 and 63 take, come from one load per half-wave at one address.  Columns at or
// beyond n hold zero, which is also the Dirichlet ghost value, so a wave that straddles the last
// column needs no special case.
// ---------------------------------------------------------------------------------------------
constexpr int ST_RY = 16;    // rows per wave
constexpr int ST_WAVES = 4;  // waves per block, stacked in rows

__device__ __forceinline__ double lane_below(double v) {   // lane l gets lane l-1's v (lane 0: 0)
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_above(double v) {   // lane l gets lane l+1's v (lane 63: 0)
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_below(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_above(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}

// The block a workgroup runs: column strip bx, block row by, level bz.  Workgroups go to the 8
// XCDs round-robin by linear id.  When the block rows of all levels (grid y times z) are a
// multiple of 8, block row R = 8k + x runs whole on XCD x, so the strips beside a block, whose
// edge columns it reads, sit in the same L2; the levels still spread over every XCD.
struct StBlock {
  unsigned x, y, z;
};
__device__ __forceinline__ StBlock stencil_block() {
  const unsigned gx = gridDim.x, rows = gridDim.y * gridDim.z;
  if (rows % 8 != 0) return StBlock{blockIdx.x, blockIdx.y, blockIdx.z};
  const unsigned id = blockIdx.x + gx * (blockIdx.y + gridDim.y * blockIdx.z);
  const unsigned r = id / 8;
  const unsigned row = (r / gx) * 8 + id % 8;
  return StBlock{r % gx, row % gridDim.y, row / gridDim.y};
}

// Where a block's wave sits: the first row and column it owns, or false when it owns none.
__device__ __forceinline__ bool stencil_tile(int n, const StBlock& b, int* iy0, int* ix0) {
  *ix0 = (int)b.x * 64;
  *iy0 = ((int)b.y * ST_WAVES + (int)(threadIdx.x >> 6)) * ST_RY;
  return *ix0 < n && *iy0 < n;
}

// ---------------------------------------------------------------------------------------------
// right-hand side (increment form), FP64; also writes the low-precision copy.  The quadrature
// of f along level j-1 is taken as sum_i w_i f_E(v_i) + nu Lap_h (sum_i w_i v_i): the stencil
// is linear, so one stencil of the weighted window replaces j+1 stencils.
// ---------------------------------------------------------------------------------------------
// The values of one grid row that the right-hand side needs at a column.
struct RhsRow {
  double V;     // sum_i w_i v_i (level 0: the own value u)
  double fq;    // sum_i w_i f_E(v_i) (level 0: f_E(u))
  double fen;   // f_E(v at node n)
  double vn1;   // v at node n+1
  double u;     // own value at node n
};

// JT = the number of window vectors j + 1 when it is fixed at compile time (0 for the
// predictor), or -1: any j, up to the largest order.  This kernel uses no LDS, and its plain
// (flat) loads measured faster than global ones (31.2 against 33.2 us per launch at 1024^2,
// FP64).
template <int JT>
__device__ __forceinline__ void rhs_level(const Lvl2D& L, int64_t m, int iy0, int ix0) {
  constexpr int JN = JT < 0 ? RIDC_MAX_ORDER : (JT == 0 ? 1 : JT);
  const int n = L.n;
  const int ix = ix0 + (threadIdx.x & 63);
  const bool col = ix < n;
  const int64_t nn = (int64_t)n * n;
  const int64_t nidx = m - 1;
  const double* __restrict__ u = L.own + (nidx % L.R_own) * nn;
  const int nv = JT < 0 ? L.j + 1 : JT;        // window vectors
  const double* __restrict__ vp[JN];
  double w[JN];
  int rn = 0;                                  // window index of node n (node n+1 is rn + 1)
  if (JT == 0) {
    vp[0] = u;
    w[0] = 1.0;
  } else {
    const int64_t s = m - L.j > 0 ? m - L.j : 0;
    rn = (int)(nidx - s);
#pragma unroll
    for (int i = 0; i < JN; ++i) {
      if (i < nv) {
        vp[i] = L.prev + ((s + i) % L.R_prev) * nn;
        w[i] = gld<double>(L.W + (nidx - s) * (L.j + 1) + i);
      }
    }
  }
  auto window_sum = [&](int64_t c) {           // sum_i w_i v_i at one point
    if (JT == 0) return u[c];
    double V = 0.0;
#pragma unroll
    for (int i = 0; i < JN; ++i)
      if (i < nv) V += w[i] * vp[i][c];
    return V;
  };
  // The walk down the strip goes RG rows at a time, each group unrolled and without a branch,
  // so that the loads of a group's rows are issued together: lanes past n and rows outside the
  // grid load a clamped in-range address and take zero instead, lanes 0 and 63 take their edge
  // column by a select, and the stores follow each group.  Every wave has ST_RY rows (n is a
  // multiple of 32).  Measured at 1024^2, FP64: 29.1 us per launch with a branch per row and
  // edge, 22.6 us with RG = 2 (114 registers), 22.8 with 1, 26.5 with 4 (148), 27.7 with 8
  // (228), 38.5 with the whole strip unrolled (388 registers, one wave per SIMD).
  const int ixc = col ? ix : n - 1;
  auto load = [&](int iy) {
    const bool in = iy >= 0 && iy < n && col;
    const int64_t c = (int64_t)(iy < 0 ? 0 : (iy < n ? iy : n - 1)) * n + ixc;
    RhsRow r{0.0, 0.0, 0.0, 0.0, 0.0};
    if (JT == 0) {
      r.u = u[c];
      r.V = r.u;
      r.fq = fe2(L.fe, r.u);
    } else {
      r.u = u[c];
#pragma unroll
      for (int i = 0; i < JN; ++i) {
        if (i < nv) {
          const double v = vp[i][c];
          const double f = fe2(L.fe, v);
          r.V += w[i] * v;
          r.fq += w[i] * f;
          if (i == rn) r.fen = f;
          if (i == rn + 1) r.vn1 = v;
        }
      }
    }
    const RhsRow z{0.0, 0.0, 0.0, 0.0, 0.0};
    return in ? r : z;
  };
  // the column just outside the strip that lane 0 (west) or lane 63 (east) takes: every lane
  // of a half reads that one address (zero outside the grid, the Dirichlet ghost value)
  const int lane = threadIdx.x & 63;
  const int xo = lane < 32 ? ix0 - 1 : ix0 + 64;
  const bool xok = xo >= 0 && xo < n;
  const int xoc = xok ? xo : ixc;
  const double dt = L.dt;
  double up = load(iy0 - 1).V;
  RhsRow mid = load(iy0);
  constexpr int RG = 2;
#pragma unroll
  for (int q = 0; q < ST_RY; q += RG) {
    double bs[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      const int iy = iy0 + q + r;
      const RhsRow dn = load(iy + 1);
      const double ev = window_sum((int64_t)iy * n + xoc);
      double vw = lane_below(mid.V), ve = lane_above(mid.V);
      vw = lane == 0 ? (xok ? ev : 0.0) : vw;
      ve = lane == 63 ? (xok ? ev : 0.0) : ve;
      const double lap = ((vw + ve) + (up + dn.V)) - 4.0 * mid.V;
      const double quad = mid.fq + L.nu_h2 * lap;
      bs[r] = JT == 0 ? dt * quad
                      : (mid.u - mid.vn1) + dt * quad + dt * (fe2(L.fe, mid.u) - mid.fen);
      up = mid.V;
      mid = dn;
    }
    if (col) {
#pragma unroll
      for (int r = 0; r < RG; ++r) {
        const int64_t c = (int64_t)(iy0 + q + r) * n + ix;
        L.b64[c] = bs[r];
        if (L.prec != PREC_F64) store_lo(L.lo0, c, bs[r]);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_rhs2d(const Lvl2D* __restrict__ levels, int64_t sigma) {
  const StBlock blk = stencil_block();
  const Lvl2D& L = levels[blk.z];
  int64_t m;
  if (!level_active(L, sigma, &m)) return;
  int iy0, ix0;
  if (!stencil_tile(L.n, blk, &iy0, &ix0)) return;
  switch (L.j) {
    case 0: rhs_level<0>(L, m, iy0, ix0); break;
    case 1: rhs_level<2>(L, m, iy0, ix0); break;
    case 2: rhs_level<3>(L, m, iy0, ix0); break;
    case 3: rhs_level<4>(L, m, iy0, ix0); break;
    default: rhs_level<-1>(L, m, iy0, ix0); break;
  }
}

// rho = b - (x1 - dt nu Lap_h x1), FP64, written in low precision.  The first solve x1 is held in
// FP32 (in the x64 buffer; it leaves an FP32 accumulator, so nothing is lost).  Every row of the
// wave's column strip is loaded before any is used, so all of a wave's loads are in flight at
// once.
__global__ __launch_bounds__(256) void k_resid2d(const Lvl2D* __restrict__ levels, int64_t sigma) {
  const StBlock blk = stencil_block();
  const Lvl2D& L = levels[blk.z];
  int64_t m;
  if (!level_active(L, sigma, &m)) return;
  const int n = L.n;
  int iy0, ix0;
  if (!stencil_tile(n, blk, &iy0, &ix0)) return;
  const int lane = threadIdx.x & 63;
  const int ix = ix0 + lane;
  const bool col = ix < n;
  const float* __restrict__ x1 = (const float*)L.x64;
  // No load sits behind a branch, so that all of them issue back to back: lanes past n and the
  // rows beyond the grid read a clamped in-range address and take zero instead, and the column
  // just outside the strip, which lane 0 (west) or 63 (east) takes, is read by every lane of
  // its half at that one address.  Every wave has ST_RY rows (n is a multiple of 32).
  const int ixc = col ? ix : n - 1;
  const int xo = lane < 32 ? ix0 - 1 : ix0 + 64;
  const bool xok = xo >= 0 && xo < n;
  const int xoc = xok ? xo : ixc;
  float xr[ST_RY + 2], xe[ST_RY];
  double br[ST_RY];
#pragma unroll
  for (int r = 0; r < ST_RY + 2; ++r) {
    const int iy = iy0 - 1 + r;
    const int iyc = iy < 0 ? 0 : (iy < n ? iy : n - 1);
    const float v = gld<float>(x1 + (int64_t)iyc * n + ixc);
    xr[r] = iy >= 0 && iy < n && col ? v : 0.0f;
  }
#pragma unroll
  for (int r = 0; r < ST_RY; ++r) {
    const int64_t row = (int64_t)(iy0 + r) * n;
    const double b = gld<double>(L.b64 + row + ixc);
    const float e = gld<float>(x1 + row + xoc);
    br[r] = col ? b : 0.0;
    xe[r] = xok ? e : 0.0f;
  }
  double res[ST_RY];
#pragma unroll
  for (int r = 0; r < ST_RY; ++r) {
    double xw = (double)lane_below(xr[r + 1]), xa = (double)lane_above(xr[r + 1]);
    xw = lane == 0 ? (double)xe[r] : xw;
    xa = lane == 63 ? (double)xe[r] : xa;
    const double x = (double)xr[r + 1];
    const double lap = ((xw + xa) + ((double)xr[r] + (double)xr[r + 2])) - 4.0 * x;
    res[r] = br[r] - (x - L.dt * L.nu_h2 * lap);
  }
  if (col) {
#pragma unroll
    for (int r = 0; r < ST_RY; ++r) store_lo(L.lo0, (int64_t)(iy0 + r) * n + ix, res[r]);
  }
}

// one launch of a stencil kernel over `cnt` levels of sides up to nmax
static void launch_stencil(void (*k)(const Lvl2D*, int64_t), const Lvl2D* lv, int cnt, int64_t nmax,
                    int64_t sigma, hipStream_t st) {
  const unsigned gx = (unsigned)((nmax + 63) / 64);
  const unsigned gy = (unsigned)((nmax + ST_RY * ST_WAVES - 1) / (ST_RY * ST_WAVES));
  hipLaunchKernelGGL(k, dim3(gx, gy, cnt), dim3(64 * ST_WAVES), 0, st, lv, sigma);
}

// ---------------------------------------------------------------------------------------------
// transform pass C = (A Q)^T on the matrix cores
//   block tile 128 x 128, 8 waves in 2 (rows) x 4 (columns), each wave 64 x 32 = 4 x 2 MFMA
//   tiles of 16 x 16; k staged through LDS in slices of BK with 16-byte global loads
// ---------------------------------------------------------------------------------------------
constexpr int BT = 128;      // block tile (rows of A x columns of Q)
// A wave computes 64 rows x WC columns of the block tile: WC = 32 (8 waves of 512 threads, two
// per SIMD) or WC = 64 (4 waves of 256 threads, one per SIMD with the whole register file,
// fewer LDS reads per MFMA).
template <int WC>
constexpr int pass_threads() {
  return WC == 64 ? 256 : 512;
}

template <int PREC>
struct Tr;

template <>
struct Tr<PREC_F64> {
  typedef double T;
  static constexpr int BK = 16;
  typedef dbl4 Acc;
};
template <>
struct Tr<PREC_F32> {
  typedef float T;
  static constexpr int BK = 32;
  typedef flt4 Acc;
};
template <>
struct Tr<PREC_BF16> {
  typedef u16 T;
  static constexpr int BK = 32;
  typedef flt4 Acc;
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// Folding by the reflection symmetry of the sine matrix, Q_{n-1-k, j} = (-1)^j Q_{k, j}:
//   (A Q)_{ij} = sum_{k < n/2} (A_{ik} + (-1)^j A_{i, n-1-k}) Q_{kj},
// so the even output columns take the sums and the odd ones the differences of mirrored columns
// of A, against half of Q.  a holds columns k .. k+e-1 of a row, m the mirrored chunk
// n-k-e .. n-k-1 (its elements in reverse order pair with a's).
__device__ __forceinline__ void fold_f64(u32x4 a, u32x4 m, u32x4* sum, u32x4* dif) {
  const dbl2 x = __builtin_bit_cast(dbl2, a), y = __builtin_bit_cast(dbl2, m);
  *sum = __builtin_bit_cast(u32x4, dbl2{x[0] + y[1], x[1] + y[0]});
  *dif = __builtin_bit_cast(u32x4, dbl2{x[0] - y[1], x[1] - y[0]});
}
__device__ __forceinline__ void fold_f32(u32x4 a, u32x4 m, u32x4* sum, u32x4* dif) {
  const flt4 x = __builtin_bit_cast(flt4, a), y = __builtin_bit_cast(flt4, m);
  *sum = __builtin_bit_cast(u32x4, flt4{x[0] + y[3], x[1] + y[2], x[2] + y[1], x[3] + y[0]});
  *dif = __builtin_bit_cast(u32x4, flt4{x[0] - y[3], x[1] - y[2], x[2] - y[1], x[3] - y[0]});
}
// 4 FP32 values -> BF16 hi (round to nearest) and BF16 lo (of the remainder), 8 bytes each
__device__ __forceinline__ void split4_bf16(flt4 v, uint2* hi, uint2* lo) {
  unsigned short h[4], l[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const __bf16 b = (__bf16)v[e];
    h[e] = __builtin_bit_cast(unsigned short, b);
    l[e] = __builtin_bit_cast(unsigned short, (__bf16)(v[e] - (float)b));
  }
  *hi = uint2{(unsigned)h[0] | ((unsigned)h[1] << 16), (unsigned)h[2] | ((unsigned)h[3] << 16)};
  *lo = uint2{(unsigned)l[0] | ((unsigned)l[1] << 16), (unsigned)l[2] | ((unsigned)l[3] << 16)};
}

// only the sums (sg = 1) or only the differences (sg = -1), for blocks whose output columns all
// have one parity
__device__ __forceinline__ u32x4 fold1_f64(u32x4 a, u32x4 m, double sg) {
  const dbl2 x = __builtin_bit_cast(dbl2, a), y = __builtin_bit_cast(dbl2, m);
  return __builtin_bit_cast(u32x4, dbl2{x[0] + sg * y[1], x[1] + sg * y[0]});
}
__device__ __forceinline__ u32x4 fold1_f32(u32x4 a, u32x4 m, float sg) {
  const flt4 x = __builtin_bit_cast(flt4, a), y = __builtin_bit_cast(flt4, m);
  return __builtin_bit_cast(u32x4, flt4{x[0] + sg * y[3], x[1] + sg * y[2], x[2] + sg * y[1],
                                        x[3] + sg * y[0]});
}


// Instruction order of one pipelined k-slice step (a single basic block): NR LDS reads, then
// NW LDS writes and global loads, each placed after one of the step's NM MFMAs, and the rest of
// the MFMAs after them.  Groups with no instruction left to take stay empty.
template <int NM, int NR, int NW>
__device__ __forceinline__ void interleave_step() {
  static_assert(NR + NW <= NM, "one MFMA per memory instruction");
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
  }
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
    __builtin_amdgcn_sched_group_barrier(0x210, 1, 0);   // LDS write or global load
  }
  __builtin_amdgcn_sched_group_barrier(0x008, NM - NR - NW, 0);
}

// FOLD (n a multiple of 64): the contraction runs over k < n/2 with the folded A operands and
// E.Q the folded transform: row j' (n rows) holds Q_{k, perm(j')} for k < n/2, perm(j') = 2j'
// for j' < n/2 and 2(j' - n/2) + 1 above; output column j' of the block grid is column perm(j').
// KX = 2 doubles the k-slice (one slice in flight instead of two).  A k-slice has two LDS stages
// (the next slice is stored while the current one feeds the matrix cores, one barrier per
// slice), except the wide split-BF16 slices, whose operands fill one stage's worth of the LDS
// twice over.  Most variants need more than 64 KB, so every variant takes its LDS dynamically
// (pass_lds_bytes).
template <int PREC, int KX>
constexpr int lds_stages() {
  return PREC == PREC_BF16 && KX == 2 ? 1 : 2;
}
// A operand tiles per LDS stage: the folded sums and differences when the pass folds while
// staging (a block with output columns on both sides of n/2 needs both), else one
template <int FOLD, int AIN>
constexpr int a_tiles() {
  return FOLD && !AIN ? 2 : 1;
}
template <int PREC, int KX, int AIN>
constexpr size_t pass_lds_bytes(int fold) {
  typedef typename Tr<PREC>::T T;
  constexpr int BK = Tr<PREC>::BK * KX;
  constexpr int LDE = (BK * (int)sizeof(T) + 16) / (int)sizeof(T);
  constexpr int NSPLIT = PREC == PREC_BF16 ? 2 : 1;
  const int na = fold && !AIN ? 2 : 1;
  return (size_t)lds_stages<PREC, KX>() * (na * NSPLIT + NSPLIT) * BT * LDE * sizeof(T);
}

template <int PREC, int OUT, int FOLD, int KX, int WC, int AIN>
__global__ __launch_bounds__(pass_threads<WC>()) void k_pass2d(const Pass2D* __restrict__ passes,
                                                               const Lvl2D* __restrict__ levels,
                                                               int64_t sigma) {
  constexpr int NTHR = pass_threads<WC>();
  constexpr int NB = WC / 16;                         // 16-column MFMA tiles per wave
  typedef Tr<PREC> TR;
  typedef typename TR::T T;
  typedef typename TR::Acc Acc;
  constexpr int BK = TR::BK * KX;
  constexpr int ROWB = BK * (int)sizeof(T) + 16;     // LDS row stride in bytes (16-aligned)
  constexpr int LDE = ROWB / (int)sizeof(T);          // ... in elements
  constexpr int CH = BK * (int)sizeof(T) / 16;        // 16-byte chunks per row
  constexpr int NSPLIT = PREC == PREC_BF16 ? 2 : 1;
  constexpr int CPT = BT * CH / NTHR;                 // chunks per thread per operand and split
  constexpr int NA = a_tiles<FOLD, AIN>();           // A operands in LDS (folded sums, diffs)
  static_assert(!AIN || FOLD, "prefolded operands exist for folded transforms only");
  static_assert(OUT != OUT_FOLD || FOLD, "a folded output needs the folded transform");
  extern __shared__ __attribute__((aligned(16))) unsigned char pass_smem[];
  // LDS stage b of a k-slice: the A operands, then Q
  constexpr size_t A_BYTES = (size_t)NA * NSPLIT * BT * LDE * sizeof(T);
  constexpr size_t STAGE_BYTES = A_BYTES + (size_t)NSPLIT * BT * LDE * sizeof(T);
  auto stage_a = [&](int b) {
    return reinterpret_cast<T (*)[NSPLIT][BT * LDE]>(pass_smem + b * STAGE_BYTES);
  };
  auto stage_b = [&](int b) {
    return reinterpret_cast<T (*)[BT * LDE]>(pass_smem + b * STAGE_BYTES + A_BYTES);
  };
  T (*As)[NSPLIT][BT * LDE] = stage_a(0);      // also the epilogue's staging area

  // XCD-aware tile order: workgroups go to the 8 XCDs round-robin by linear id, so tile q of
  // XCD x is x * (T / 8) + (id / 8): each XCD takes a contiguous run of tiles, and the column
  // tiles of one row tile of A meet in one L2 (identity when T is not a multiple of 8)
  unsigned bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  {
    const unsigned t = gridDim.x;
    const unsigned tiles = t * gridDim.y * gridDim.z;
    const unsigned id = bx + t * (by + gridDim.y * bz);
    if (tiles % 8 == 0) {
      const unsigned q = (id % 8) * (tiles / 8) + id / 8;
      bx = q % t;
      by = (q / t) % gridDim.y;
      bz = q / (t * gridDim.y);
    }
  }
  const Pass2D& E = passes[bz];
  const Lvl2D& L = levels[E.level];
  int64_t m;
  if (!level_active(L, sigma, &m)) return;
  const int n = L.n;
  // Rows of A (i) of the block: BT consecutive rows from row0, or, when the epilogue folds its
  // output for the next pass, the mirrored pairs row0 + t and n-1-row0-t (t < BT/2) at local
  // rows t and BT/2 + t, so that the block holds both columns of every folded pair of C^T.
  constexpr bool MIRROR = OUT == OUT_FOLD;
  constexpr int HB = BT / 2;
  const int row0 = MIRROR ? by * HB : by * BT;
  const int col0 = bx * BT;                  // columns of Q (j)
  if ((MIRROR ? 2 * row0 : row0) >= n || col0 >= n) return;
  auto a_row = [&](int r) { return MIRROR ? (r < HB ? row0 + r : n - 1 - row0 - (r - HB)) : row0 + r; };
  const int64_t nn = (int64_t)n * n;
  // A arrives row-major in FP64 or FP32 (the split-BF16 pass splits it while staging), or as
  // prefolded planes of T (AIN); Q in T
  typedef typename std::conditional<PREC == PREC_BF16, float, T>::type TA;
  constexpr int EA = 16 / (int)sizeof(TA);          // A elements per 16-byte chunk
  constexpr int CHA = BK * (int)sizeof(TA) / 16;    // A chunks per row
  constexpr int NAC = BT * CHA / NTHR;              // A chunks per thread
  const TA* A = (const TA*)E.A;
  const T* Q = (const T*)E.Q;
  const int K = FOLD ? n / 2 : n;                   // contraction length
  const int64_t qsplit = (int64_t)n * K;            // BF16: lo part of the transform
  constexpr int E16 = 16 / (int)sizeof(T);          // elements per 16-byte chunk
  // prefolded operands: planes (side, split) of n rows x n/2 elements of T, side 0 the sums
  // A_{i,k} + A_{i,n-1-k} and side 1 the differences (BF16: split into hi, lo), each n x n/2
  const T* Ap = (const T*)E.A;
  const int64_t plane = (int64_t)n * K;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave / (BT / WC)) * 64;    // wave tile origin inside the block
  const int wn = (wave % (BT / WC)) * WC;

  Acc acc[4][NB];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = Acc{0, 0, 0, 0};

  // global -> register staging of one k-slice (A, its mirrored columns when folding, Q); a
  // slice's loads are issued one MFMA phase before they are stored into LDS.  Rows past n (a
  // partial block tile) read row n-1 instead: they only reach output rows or columns past n,
  // which the epilogue never stores, and no select on the loaded values makes a step wait for
  // its loads.
  struct Slice {
    u32x4 ra[NAC], rm[NAC], rp[NSPLIT][CPT], rb[NSPLIT][CPT];
  };
  Slice sl0;
  const int side = FOLD && col0 >= (n >> 1) ? 1 : 0;
  auto gload = [&](Slice& S, int k0) {
    if constexpr (AIN) {
#pragma unroll
      for (int s = 0; s < NSPLIT; ++s)
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          const int id = tid + c * NTHR;
          const int r = id / CH, q = id % CH;
          S.rp[s][c] = gld<u32x4>(Ap + (side * NSPLIT + s) * plane + (int64_t)a_row(r) * K + k0 +
                                  q * E16);
        }
    }
#pragma unroll
    for (int c = 0; c < (AIN ? 0 : NAC); ++c) {
      const int id = tid + c * NTHR;
      const int r = id / CHA, q = id % CHA;
      const int ga = a_row(r);
      const int64_t ko = k0 + q * EA;
      const TA* arow = A + (int64_t)(ga < n ? ga : n - 1) * n;
      S.ra[c] = gld<u32x4>(arow + ko);
      if constexpr (FOLD) S.rm[c] = gld<u32x4>(arow + (n - ko - EA));
    }
#pragma unroll
    for (int s = 0; s < NSPLIT; ++s)
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int id = tid + c * NTHR;
        const int r = id / CH, q = id % CH;
        const int gb = col0 + r;                        // Q symmetric: row j of Q = column j
        const int64_t ko = k0 + q * E16;
        S.rb[s][c] = gld<u32x4>(Q + s * qsplit + (int64_t)(gb < n ? gb : n - 1) * K + ko);
      }
  };
  // a block whose output columns all lie on one side of n/2 needs only the sums (side 0) or
  // only the differences (side 1)
  const bool one_side = FOLD && (col0 + BT <= (n >> 1) || col0 >= (n >> 1));
  // The main loops take one_side at compile time (os: std::true_type when the block needs one
  // side of the fold), so that a pipelined step holds no branch.
  auto with_side = [&](auto&& loop) {
    if constexpr (FOLD && !AIN) {
      if (one_side) loop(std::true_type{});
      else loop(std::false_type{});
    } else {
      loop(std::false_type{});
    }
  };
  // FP32/FP64 operand rows keep a k-slice permuted, k at (k % 4) * KQ + k / 4, so that the KQ
  // values one lane consumes over the slice (k = 4i + lane/16) are contiguous; BF16 rows keep
  // k in order (its instruction takes 8 consecutive k per lane).
  constexpr int KQ = BK / 4;
  auto put = [&](T* row_base, int q, u32x4 v) {
    if constexpr (PREC == PREC_BF16) {
      *(u32x4*)((char*)row_base + q * 16) = v;
    } else {
      constexpr int EV = 16 / (int)sizeof(T);
      struct Ev {
        T x[EV];
      };
      const Ev ev = __builtin_bit_cast(Ev, v);
#pragma unroll
      for (int e = 0; e < EV; ++e) {
        const int k = q * EV + e;
        row_base[(k & 3) * KQ + (k >> 2)] = ev.x[e];
      }
    }
  };
  auto sstore = [&](const Slice& S, int stage, auto os) {
    T (*As)[NSPLIT][BT * LDE] = stage_a(stage);
    T (*Bs)[BT * LDE] = stage_b(stage);
    if constexpr (AIN) {
#pragma unroll
      for (int s = 0; s < NSPLIT; ++s)
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          const int id = tid + c * NTHR;
          const int r = id / CH, q = id % CH;
          put(As[0][s] + r * LDE, q, S.rp[s][c]);
        }
    }
#pragma unroll
    for (int c = 0; c < (AIN ? 0 : NAC); ++c) {
      const int id = tid + c * NTHR;
      const int r = id / CHA, q = id % CHA;
      const int ro = r * LDE;                        // row start, in elements
      if constexpr (PREC == PREC_BF16) {
        // 4 FP32 values (folded when FOLD) -> BF16 hi and lo at elements 4q .. 4q+3
        auto put4 = [&](int a, u32x4 v) {
          uint2 hi, lo;
          split4_bf16(__builtin_bit_cast(flt4, v), &hi, &lo);
          *(uint2*)(As[a][0] + ro + q * 4) = hi;
          *(uint2*)(As[a][1] + ro + q * 4) = lo;
        };
        if constexpr (!FOLD) {
          put4(0, S.ra[c]);
        } else if constexpr (decltype(os)::value) {
          put4(side, fold1_f32(S.ra[c], S.rm[c], side ? -1.0f : 1.0f));
        } else {
          u32x4 su, di;
          fold_f32(S.ra[c], S.rm[c], &su, &di);
          put4(0, su);
          put4(1, di);
        }
      } else if constexpr (!FOLD) {
        put(As[0][0] + ro, q, S.ra[c]);
      } else if constexpr (decltype(os)::value) {
        if constexpr (PREC == PREC_F64)
          put(As[side][0] + ro, q, fold1_f64(S.ra[c], S.rm[c], side ? -1.0 : 1.0));
        else
          put(As[side][0] + ro, q, fold1_f32(S.ra[c], S.rm[c], side ? -1.0f : 1.0f));
      } else {
        u32x4 su, di;
        if constexpr (PREC == PREC_F64)
          fold_f64(S.ra[c], S.rm[c], &su, &di);
        else
          fold_f32(S.ra[c], S.rm[c], &su, &di);
        put(As[0][0] + ro, q, su);
        put(As[1][0] + ro, q, di);
      }
    }
#pragma unroll
    for (int s = 0; s < NSPLIT; ++s)
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int id = tid + c * NTHR;
        const int r = id / CH, q = id % CH;
        put(Bs[s] + r * LDE, q, S.rb[s][c]);
      }
  };

  // the A operand of this wave's WC output columns: sums (0) for even output columns,
  // differences (1) for odd ones -- uniform per wave, since n/2 and the wave's first column are
  // multiples of WC (the launcher takes WC = 64 only when n/2 is a multiple of 64)
  const int half = n >> 1;
  const int pa0 = FOLD && !AIN && col0 + wn >= half ? 1 : 0;
  const int KT = K / BK;
  const int r16 = lane & 15;
  auto mfma_slice = [&](int stage) {
    T (*As)[NSPLIT][BT * LDE] = stage_a(stage);
    T (*Bs)[BT * LDE] = stage_b(stage);
    if constexpr (PREC == PREC_BF16) {
#pragma unroll
    for (int ks = 0; ks < KX; ++ks) {
      // lane holds 8 consecutive k of row (l % 16), k offset 8 (l / 16), of k-step ks of 32
      const int kb = (lane >> 4) * 16 + ks * 64;       // byte offset of the 8 k values
      static_assert(NB == 2, "the split-BF16 pass takes 32-column waves");
      bf16x8 ahi[4], alo[4], bhi[2], blo[2];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int ro = (wm + t * 16 + r16) * ROWB + kb;
        ahi[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)((const char*)As[pa0][0] + ro));
        alo[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)((const char*)As[pa0][1] + ro));
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int ro = (wn + t * 16 + r16) * ROWB + kb;
        bhi[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)((const char*)Bs[0] + ro));
        blo[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)((const char*)Bs[1] + ro));
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[a], bhi[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[a], blo[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[a], bhi[b], acc[a][b], 0, 0, 0);
        }
    }
    }
  };
  // FP32/FP64 k-steps of 4: lane holds element (row l % 16, k 4i + l / 16) of step i; its KQ
  // values of a slice are contiguous in the permuted rows, read 16 bytes at a time
  constexpr int EV = 16 / (int)sizeof(T);
  struct Frag {
    T x[KQ];
  };
  auto frag = [&](const T* row) {
    Frag f;
    const int k4 = lane >> 4;
#pragma unroll
    for (int v = 0; v < KQ / EV; ++v) {
      const u32x4 w = *(const u32x4*)(row + k4 * KQ + v * EV);
      struct Ev {
        T x[EV];
      };
      const Ev ev = __builtin_bit_cast(Ev, w);
#pragma unroll
      for (int e = 0; e < EV; ++e) f.x[v * EV + e] = ev.x[e];
    }
    return f;
  };
  // this wave's fragments of the slice in LDS stage `stage`: 4 tiles of A rows, 2 of Q rows
  auto read_frags = [&](int stage, Frag (&fa)[4], Frag (&fb)[NB]) {
    T (*As)[NSPLIT][BT * LDE] = stage_a(stage);
    T (*Bs)[BT * LDE] = stage_b(stage);
#pragma unroll
    for (int t = 0; t < 4; ++t) fa[t] = frag(As[pa0][0] + (wm + t * 16 + r16) * LDE);
#pragma unroll
    for (int t = 0; t < NB; ++t) fb[t] = frag(Bs[0] + (wn + t * 16 + r16) * LDE);
  };
  auto mfma_frags = [&](const Frag (&fa)[4], const Frag (&fb)[NB]) {
    if constexpr (PREC != PREC_BF16) {
#pragma unroll
      for (int i = 0; i < KQ; ++i)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            if constexpr (PREC == PREC_F64)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a].x[i], fb[b].x[i],
                                                               acc[a][b], 0, 0, 0);
            else
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a].x[i], fb[b].x[i],
                                                               acc[a][b], 0, 0, 0);
          }
    }
  };
  if constexpr (PREC != PREC_BF16) {
    // Two LDS stages and two register sets of fragments.  Step kt issues the MFMAs of slice kt
    // from registers while the fragments of slice kt+1 are read from LDS, slice kt+2 is stored
    // into the stage slice kt came from (read into registers before the previous barrier) and
    // slice kt+3 is loading from global memory: one barrier per slice.  A step is one basic
    // block (the slices past the end re-read the last one and are never used), so that its LDS
    // and global memory instructions can be issued one between each pair of MFMAs
    // (interleave_step): the memory work runs under the matrix cores instead of between them.
    with_side([&](auto os) {
      Frag fa0[4], fb0[NB], fa1[4], fb1[NB];
      auto kslice = [&](int k) { return (k < KT ? k : KT - 1) * BK; };
      gload(sl0, 0);
      sstore(sl0, 0, os);
      gload(sl0, kslice(1));
      __syncthreads();
      read_frags(0, fa0, fb0);
      sstore(sl0, 1, os);
      gload(sl0, kslice(2));
      __syncthreads();
      auto step = [&](int kt, const Frag (&ca)[4], const Frag (&cb)[NB], Frag (&na)[4],
                      Frag (&nb)[NB]) {
        read_frags((kt + 1) & 1, na, nb);
        sstore(sl0, kt & 1, os);
        gload(sl0, kslice(kt + 3));
        mfma_frags(ca, cb);
        constexpr int NM = KQ * 4 * NB, NR = 2 * (4 + NB);   // MFMAs, 16-byte fragment reads
        interleave_step<NM, NR, (NM - NR < 24 ? NM - NR : 24)>();
        __syncthreads();
      };
      for (int kt = 0; kt < KT; kt += 2) {
        step(kt, fa0, fb0, fa1, fb1);
        if (kt + 1 < KT) step(kt + 1, fa1, fb1, fa0, fb0);
      }
    });
  } else if constexpr (lds_stages<PREC, KX>() == 2) {
    // split BF16, 32-wide slices in two LDS stages: the schedule of the FP32/FP64 passes, with
    // the hi/lo fragments of a slice (one 32-wide k-step) double-buffered in registers
    struct FragB {
      bf16x8 ahi[4], alo[4], bhi[2], blo[2];
    };
    auto read_frags_bf = [&](int stage, FragB& f) {
      T (*As)[NSPLIT][BT * LDE] = stage_a(stage);
      T (*Bs)[BT * LDE] = stage_b(stage);
      const int kb = (lane >> 4) * 16;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int ro = (wm + t * 16 + r16) * ROWB + kb;
        f.ahi[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)((const char*)As[pa0][0] + ro));
        f.alo[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)((const char*)As[pa0][1] + ro));
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int ro = (wn + t * 16 + r16) * ROWB + kb;
        f.bhi[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)((const char*)Bs[0] + ro));
        f.blo[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)((const char*)Bs[1] + ro));
      }
    };
    // each accumulator takes lo*hi, hi*lo, hi*hi in that order; the eight accumulators are
    // independent, so one kind of product is issued over all of them before the next
    auto mfma_bf = [&](const FragB& f) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.alo[a], f.bhi[b], acc[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ahi[a], f.blo[b], acc[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ahi[a], f.bhi[b], acc[a][b], 0, 0, 0);
    };
    with_side([&](auto os) {
      FragB f0, f1;
      auto kslice = [&](int k) { return (k < KT ? k : KT - 1) * BK; };
      gload(sl0, 0);
      sstore(sl0, 0, os);
      gload(sl0, kslice(1));
      __syncthreads();
      read_frags_bf(0, f0);
      sstore(sl0, 1, os);
      gload(sl0, kslice(2));
      __syncthreads();
      auto step_bf = [&](int kt, const FragB& cur, FragB& next) {
        read_frags_bf((kt + 1) & 1, next);
        sstore(sl0, kt & 1, os);
        gload(sl0, kslice(kt + 3));
        mfma_bf(cur);
        interleave_step<24, 12, 12>();
        __syncthreads();
      };
      for (int kt = 0; kt < KT; kt += 2) {
        step_bf(kt, f0, f1);
        if (kt + 1 < KT) step_bf(kt + 1, f1, f0);
      }
    });
  } else {
    // wide slices: one in flight, its loads cover a whole MFMA phase of twice the length
    with_side([&](auto os) {
      gload(sl0, 0);
      for (int kt = 0; kt < KT; ++kt) {
        __syncthreads();
        sstore(sl0, 0, os);
        __syncthreads();
        if (kt + 1 < KT) gload(sl0, (kt + 1) * BK);
        mfma_slice(0);
      }
    });
  }

  // epilogue: acc[a][b] holds C[i][j] for the 16 x 16 tile at local rows wm + 16a (A row
  // a_row(.)), columns col0 + wn + 16b (column l%16 of lane l); the pass stores the transpose,
  // out[j][i].  The tile goes through LDS (the A staging area) RJ output rows at a time, so that
  // each thread then finishes and writes a contiguous run of ET elements of one output row (or,
  // folding, EF mirrored pairs of one output row).
  typedef typename std::conditional<PREC == PREC_F64, double, float>::type ST;
  constexpr int RJ = PREC == PREC_F64 ? 16 : 32;              // output rows per round
  constexpr int SS = BT + 16 / (int)sizeof(ST);               // LDS row stride, 16-byte rows
  constexpr int ET = RJ * BT / NTHR;                          // elements per thread: 4 to 16
  static_assert(RJ * SS * sizeof(ST) <= sizeof(As[0]), "staging fits the A buffer");
  ST* stg = reinterpret_cast<ST*>(&As[0][0][0]);
  double* out64 = nullptr;
  const double* base = nullptr;
  if constexpr (OUT == OUT_FINAL) {
    out64 = L.own + (m % L.R_own) * nn;
    base = L.j == 0 ? L.own + ((m - 1) % L.R_own) * nn : L.prev + (m % L.R_prev) * nn;
  }
  // output row of accumulator element r: FP32 tiles hold rows 4(l/16) + r, FP64 tiles hold
  // rows (l/16) + 4r (measured lane layouts of the two instructions)
  const int i_base = PREC == PREC_F64 ? (lane >> 4) : 4 * (lane >> 4);
  // folded output: thread's output row in a round and its first pair (pairs t, HB + t of the
  // local rows, i.e. A rows row0 + t and n-1-row0-t, fold into element row0 + t of the planes)
  constexpr int EF = RJ * HB / NTHR;                          // pairs per thread: 2 to 8
  const int frow = tid / (HB / EF);
  const int ft = (tid % (HB / EF)) * EF;
  constexpr int i_step = PREC == PREC_F64 ? 4 : 1;
  const int j_l = lane & 15;
  const int orow = tid / (BT / ET);                   // this thread's output row in a round
  const int oc = (tid % (BT / ET)) * ET;              // and its first element
  // the final update's FP64 operands (base, add) of this thread's run, loaded one round ahead
  dbl2 bq[2][ET / 2];
  typedef float flt2 __attribute__((ext_vector_type(2)));
  flt2 aq[2][ET / 2];
  auto fetch = [&](int jr, int slot) {
    if constexpr (OUT == OUT_FINAL) {
      const int jp = col0 + jr + orow;
      const int i0 = row0 + oc;
      if (jp >= n || i0 >= n) return;
      const int j = FOLD ? (jp < half ? 2 * jp : 2 * (jp - half) + 1) : jp;
      const int64_t o = (int64_t)j * n + i0;
#pragma unroll
      for (int e = 0; e < ET / 2; ++e) {
        bq[slot][e] = gld<dbl2>(base + o + 2 * e);
        aq[slot][e] = E.add ? gld<flt2>(E.add + o + 2 * e) : flt2{0.0f, 0.0f};
      }
    }
  };
  fetch(0, 0);
  for (int jr = 0; jr < BT; jr += RJ) {
    const int cur = (jr / RJ) & 1;
    __syncthreads();                                  // the buffer is free
    if (wn <= jr && jr < wn + WC) {                   // this wave holds rows jr .. jr + RJ
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int jl0 = wn + 16 * b;
        if (jl0 < jr || jl0 >= jr + RJ) continue;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          ST* dst = stg + (jl0 - jr + j_l) * SS + wm + 16 * a + i_base;
          if constexpr (PREC == PREC_F64) {
#pragma unroll
            for (int r = 0; r < 4; ++r) dst[i_step * r] = acc[a][b][r];
          } else {
            // FP32 tiles hold 4 consecutive rows per lane: one 16-byte store (16-byte aligned:
            // SS, wm, 16a and i_base are multiples of 4)
            *(flt4*)dst = acc[a][b];
          }
        }
      }
    }
    __syncthreads();
    if (jr + RJ < BT) fetch(jr + RJ, cur ^ 1);
    if constexpr (OUT == OUT_FOLD) {
      // sums (side 0) and differences (side 1) of out[j][i] over mirrored i, in the precision
      // the next pass would fold in: FP64, else the FP32 values it would have loaded (BF16:
      // then split into hi, lo)
      const int jp = col0 + jr + frow;
      const int j = jp < half ? 2 * jp : 2 * (jp - half) + 1;
      double x[EF], y[EF];
#pragma unroll
      for (int e = 0; e < EF; ++e) {
        x[e] = (double)stg[frow * SS + ft + e];
        y[e] = (double)stg[frow * SS + HB + ft + e];
      }
      if (E.divide) {
        const double lj = gld<double>(E.lam + j);
#pragma unroll
        for (int e = 0; e < EF; ++e) {
          x[e] = x[e] / (1.0 + (gld<double>(E.lam + row0 + ft + e) + lj));
          y[e] = y[e] / (1.0 + (gld<double>(E.lam + n - 1 - row0 - ft - e) + lj));
        }
      }
      T* Cp = (T*)E.C + (int64_t)j * K + row0 + ft;   // plane (0, 0); side s, split p at
      if constexpr (PREC == PREC_F64) {                 // + (s * NSPLIT + p) * plane
#pragma unroll
        for (int e = 0; e < EF; e += 2) {
          gst<dbl2>(Cp + e, dbl2{x[e] + y[e], x[e + 1] + y[e + 1]});
          gst<dbl2>(Cp + plane + e, dbl2{x[e] - y[e], x[e + 1] - y[e + 1]});
        }
      } else {
#pragma unroll
        for (int e = 0; e < EF; e += 4) {
          flt4 su, di;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const float xf = (float)x[e + t], yf = (float)y[e + t];
            su[t] = xf + yf;
            di[t] = xf - yf;
          }
          if constexpr (PREC == PREC_F32) {
            gst<flt4>(Cp + e, su);
            gst<flt4>(Cp + plane + e, di);
          } else {
            typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
            uint2 hi, lo;
            split4_bf16(su, &hi, &lo);
            gst<u32x2>(Cp + e, __builtin_bit_cast(u32x2, hi));
            gst<u32x2>(Cp + plane + e, __builtin_bit_cast(u32x2, lo));
            split4_bf16(di, &hi, &lo);
            gst<u32x2>(Cp + 2 * plane + e, __builtin_bit_cast(u32x2, hi));
            gst<u32x2>(Cp + 3 * plane + e, __builtin_bit_cast(u32x2, lo));
          }
        }
      }
      continue;
    }
    const int jp = col0 + jr + orow;                  // column of the block grid
    const int i0 = row0 + oc;
    if (jp >= n || i0 >= n) continue;                 // n is a multiple of 32: whole runs
    const int j = FOLD ? (jp < half ? 2 * jp : 2 * (jp - half) + 1) : jp;
    const int64_t o = (int64_t)j * n + i0;
    double v[ET];
    if constexpr (PREC == PREC_F64) {
#pragma unroll
      for (int e = 0; e < ET; e += 2) {
        const dbl2 w = *(const dbl2*)(stg + orow * SS + oc + e);
        v[e] = w[0];
        v[e + 1] = w[1];
      }
    } else {
#pragma unroll
      for (int e = 0; e < ET; e += 4) {
        const flt4 w = *(const flt4*)(stg + orow * SS + oc + e);
#pragma unroll
        for (int t = 0; t < 4; ++t) v[e + t] = (double)w[t];
      }
    }
    if (E.divide) {
      const double lj = gld<double>(E.lam + j);
#pragma unroll
      for (int e = 0; e < ET; ++e) v[e] = v[e] / (1.0 + (gld<double>(E.lam + i0 + e) + lj));
    }
    if constexpr (OUT == OUT_F64) {
#pragma unroll
      for (int e = 0; e < ET; e += 2) gst<dbl2>((double*)E.C + o + e, dbl2{v[e], v[e + 1]});
    } else if constexpr (OUT == OUT_F32) {
#pragma unroll
      for (int e = 0; e < ET; e += 4)
        gst<flt4>((float*)E.C + o + e,
                  flt4{(float)v[e], (float)v[e + 1], (float)v[e + 2], (float)v[e + 3]});
    } else {
#pragma unroll
      for (int e = 0; e < ET; e += 2) {
        const dbl2 bs = bq[cur][e / 2];
        const dbl2 ad = dbl2{(double)aq[cur][e / 2][0], (double)aq[cur][e / 2][1]};
        gst<dbl2>(out64 + o + e, dbl2{bs[0] + (ad[0] + v[e]), bs[1] + (ad[1] + v[e + 1])});
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------
namespace {

// Systems whose side is a multiple of 64 use the folded transform (their plans hold it).
bool folded(int64_t n) { return n % 64 == 0; }

struct Transform {
  double* q64 = nullptr;
  float* q32 = nullptr;
  u16* qbf = nullptr;
};
std::mutex g_tf_mu;
std::map<int64_t, Transform> g_tf;  // per n, per device id in the high bits; kept until exit

int get_transform(int64_t n, int prec, Transform* out) {
  int dev = 0;
  RIDC_HIP_TRY(hipGetDevice(&dev));
  const int64_t key = ((int64_t)dev << 40) | n;
  std::lock_guard<std::mutex> lk(g_tf_mu);
  Transform& t = g_tf[key];
  const int64_t nn = n * n;
  if ((prec == PREC_F64 && !t.q64) || (prec == PREC_F32 && !t.q32) ||
      (prec == PREC_BF16 && !t.qbf)) {
    // Q_{ik} = sqrt(2/(n+1)) sin(pi (i+1)(k+1)/(n+1)), argument reduced exactly mod 2(n+1)
    std::vector<double> q(nn);
    const long double scale = std::sqrt(2.0L / (long double)(n + 1));
    const long double pi = 3.141592653589793238462643383279502884L;
    const int64_t period = 2 * (n + 1);
    std::vector<long double> s(period);
    for (int64_t k = 0; k < period; ++k) s[k] = scale * std::sin(pi * (long double)k / (n + 1));
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = 0; k < n; ++k) q[i * n + k] = (double)s[((i + 1) * (k + 1)) % period];
    // folded systems keep rows j' of Q_{k, perm(j')}, k < n/2 (see k_pass2d); others all of Q
    int64_t cnt = nn;
    if (folded(n)) {
      const int64_t K = n / 2;
      std::vector<double> qh(n * K);
      for (int64_t jp = 0; jp < n; ++jp) {
        const int64_t j = jp < K ? 2 * jp : 2 * (jp - K) + 1;
        for (int64_t k = 0; k < K; ++k) qh[jp * K + k] = q[k * n + j];
      }
      q.swap(qh);
      cnt = n * K;
    }
    if (prec == PREC_F64) {
      if (hipMalloc(&t.q64, cnt * sizeof(double)) != hipSuccess) return fail(RIDC_E_NOMEM, "Q64");
      RIDC_HIP_TRY(hipMemcpy(t.q64, q.data(), cnt * sizeof(double), hipMemcpyHostToDevice));
    } else if (prec == PREC_F32) {
      std::vector<float> qf(cnt);
      for (int64_t i = 0; i < cnt; ++i) qf[i] = (float)q[i];
      if (hipMalloc(&t.q32, cnt * sizeof(float)) != hipSuccess) return fail(RIDC_E_NOMEM, "Q32");
      RIDC_HIP_TRY(hipMemcpy(t.q32, qf.data(), cnt * sizeof(float), hipMemcpyHostToDevice));
    } else {
      std::vector<u16> qb(2 * cnt);
      for (int64_t i = 0; i < cnt; ++i) {
        // round to nearest even BF16 of the FP32 value, then of the FP32 remainder
        auto to_bf = [](float f) -> u16 {
          uint32_t u = __builtin_bit_cast(uint32_t, f);
          u += 0x7fff + ((u >> 16) & 1);
          return (u16)(u >> 16);
        };
        auto from_bf = [](u16 b) -> float { return __builtin_bit_cast(float, (uint32_t)b << 16); };
        const float f = (float)q[i];
        const u16 hi = to_bf(f);
        const u16 lo = to_bf(f - from_bf(hi));
        qb[i] = hi;
        qb[cnt + i] = lo;
      }
      if (hipMalloc(&t.qbf, 2 * cnt * sizeof(u16)) != hipSuccess) return fail(RIDC_E_NOMEM, "Qbf");
      RIDC_HIP_TRY(hipMemcpy(t.qbf, qb.data(), 2 * cnt * sizeof(u16), hipMemcpyHostToDevice));
    }
  }
  *out = t;
  return RIDC_OK;
}

int prec_of(const ridc_problem* p) {
  return p->prec == RIDC_PREC_FP64 ? PREC_F64 : (p->prec == RIDC_PREC_FP32_REFINE ? PREC_F32 : PREC_BF16);
}

size_t level_ws_bytes(int64_t n, int prec) {
  const size_t nn = (size_t)n * n;
  if (prec == PREC_F64) return 2 * nn * sizeof(double);             // b64, x64 (intermediate)
  return 2 * nn * sizeof(double) + 2 * nn * sizeof(float);          // b64, x64, lo0, lo1
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Wide k-slices for the split-BF16 pass when the folded contraction is a multiple of twice the
// slice (measured: 31.9 -> 29.2 us per pass at 1024^2; the FP32 and FP64 passes gain nothing).
template <int PREC>
bool wide_slices(int64_t n) {
  return PREC == PREC_BF16 && folded(n) && (n / 2) % (2 * Tr<PREC>::BK) == 0;
}

// 64-column waves (tile bit kPassWide64) are possible when the fold cannot split a wave's
// columns between sums and differences (n/2 a multiple of 64, or no fold), for the FP32 and
// FP64 passes; the split-BF16 pass takes 64-wide k-slices unless tile bit kPassNarrowK asks for
// 32-wide ones.  Every shape issues the same MFMA sequence for every output element.
template <int PREC>
bool wide_waves(int64_t n, int tile) {
  return PREC != PREC_BF16 && (tile & kPassWide64) && (!folded(n) || n % 128 == 0);
}

// Prefolded operands: when n/2 is a multiple of the block tile (every block's output columns
// lie on one side of n/2) the passes exchange their intermediates as folded planes, written by
// the previous pass's epilogue, unless tile bit kPassPlainA asks for row-major intermediates
// folded while staging.  Both give bitwise the same results.
bool prefold(int64_t n, int tile) { return folded(n) && n % (2 * BT) == 0 && !(tile & kPassPlainA); }

// One transform pass.  AIN: the A operand is prefolded planes (1) or row-major (0); OUT_FOLD
// writes prefolded planes for the next pass.
template <int PREC, int OUT, int AIN>
void launch_pass(const Pass2D* d, const Lvl2D* lv, int count, int64_t nmax, int64_t sigma,
                 int tile, hipStream_t st) {
  const unsigned t = (unsigned)((nmax + BT - 1) / BT);
  const dim3 grid(t, t, count);
  if constexpr (AIN == 1) {
    const size_t planes = pass_lds_bytes<PREC, 1, 1>(1);
    if constexpr (PREC != PREC_BF16) {
      if (tile & kPassWide64) {
        hipLaunchKernelGGL((k_pass2d<PREC, OUT, 1, 1, 64, 1>), grid, dim3(pass_threads<64>()),
                           planes, st, d, lv, sigma);
        return;
      }
    }
    hipLaunchKernelGGL((k_pass2d<PREC, OUT, 1, 1, 32, 1>), grid, dim3(pass_threads<32>()), planes,
                       st, d, lv, sigma);
  } else {
    const size_t full = pass_lds_bytes<PREC, 1, 0>(0), fold = pass_lds_bytes<PREC, 1, 0>(1);
    const size_t wide = pass_lds_bytes<PREC, 2, 0>(1);
    if constexpr (PREC != PREC_BF16) {
      if (wide_waves<PREC>(nmax, tile)) {
        if constexpr (OUT != OUT_FOLD)
          if (!folded(nmax)) {
            hipLaunchKernelGGL((k_pass2d<PREC, OUT, 0, 1, 64, 0>), grid, dim3(pass_threads<64>()),
                               full, st, d, lv, sigma);
            return;
          }
        hipLaunchKernelGGL((k_pass2d<PREC, OUT, 1, 1, 64, 0>), grid, dim3(pass_threads<64>()),
                           fold, st, d, lv, sigma);
        return;
      }
    }
    if constexpr (OUT != OUT_FOLD)
      if (!folded(nmax)) {
        hipLaunchKernelGGL((k_pass2d<PREC, OUT, 0, 1, 32, 0>), grid, dim3(pass_threads<32>()),
                           full, st, d, lv, sigma);
        return;
      }
    if (!wide_slices<PREC>(nmax) || (tile & kPassNarrowK)) {
      hipLaunchKernelGGL((k_pass2d<PREC, OUT, 1, 1, 32, 0>), grid, dim3(pass_threads<32>()), fold,
                         st, d, lv, sigma);
    } else {
      if constexpr (PREC == PREC_BF16)
        hipLaunchKernelGGL((k_pass2d<PREC, OUT, 1, 2, 32, 0>), grid, dim3(pass_threads<32>()),
                           wide, st, d, lv, sigma);
    }
  }
}

// Allow a pass variant its LDS (host call, outside any stream capture).
template <int PREC, int OUT, int FOLD, int KX, int WC, int AIN>
hipError_t allow_one() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pass2d<PREC, OUT, FOLD, KX, WC, AIN>),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)pass_lds_bytes<PREC, KX, AIN>(FOLD));
}
// every variant launch_pass<PREC, OUT, AIN> can launch
template <int PREC, int OUT, int AIN>
hipError_t allow_lds() {
  hipError_t e = hipSuccess;
  auto add = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  if constexpr (AIN == 1) {
    add(allow_one<PREC, OUT, 1, 1, 32, 1>());
    if constexpr (PREC != PREC_BF16) add(allow_one<PREC, OUT, 1, 1, 64, 1>());
  } else {
    if constexpr (OUT != OUT_FOLD) add(allow_one<PREC, OUT, 0, 1, 32, 0>());
    add(allow_one<PREC, OUT, 1, 1, 32, 0>());
    if constexpr (PREC == PREC_BF16) {
      add(allow_one<PREC, OUT, 1, 2, 32, 0>());
    } else {
      if constexpr (OUT != OUT_FOLD) add(allow_one<PREC, OUT, 0, 1, 64, 0>());
      add(allow_one<PREC, OUT, 1, 1, 64, 0>());
    }
  }
  return e;
}
template <int PREC>
hipError_t allow_pass() {
  constexpr int OWN = PREC == PREC_F64 ? OUT_F64 : OUT_F32;
  hipError_t e = allow_lds<PREC, OWN, 0>();
  if (e == hipSuccess) e = allow_lds<PREC, OUT_FINAL, 0>();
  if (e == hipSuccess) e = allow_lds<PREC, OUT_FOLD, 0>();
  if (e == hipSuccess) e = allow_lds<PREC, OUT_FOLD, 1>();
  if (e == hipSuccess) e = allow_lds<PREC, OUT_FINAL, 1>();
  if constexpr (PREC != PREC_F64)
    if (e == hipSuccess) e = allow_lds<PREC, OUT_F32, 1>();
  return e;
}

hipError_t prepare_pass_kernels(int prec) {
  return prec == PREC_BF16  ? allow_pass<PREC_BF16>()
         : prec == PREC_F32 ? allow_pass<PREC_F32>()
                            : allow_pass<PREC_F64>();
}

}  // namespace

int plan2d_validate(const ridc_problem* p) {
  if (p->n % 32 != 0) return fail(RIDC_E_UNSUPPORTED, "2D n must be a multiple of 32");
  if (p->n > 16384) return fail(RIDC_E_UNSUPPORTED, "2D n above 16384");
  return RIDC_OK;
}

size_t plan2d_workspace_bytes(const ridc_problem* p) {
  const int P = p->order;
  const int prec = prec_of(p);
  size_t b = 0;
  b += align256(sizeof(Lvl2D) * P);
  const int npass = prec == PREC_F64 ? 4 : 8;
  b += align256(sizeof(Pass2D) * P * npass);
  b += align256(sizeof(double) * (size_t)p->n);                     // lam
  b += (size_t)P * align256(level_ws_bytes(p->n, prec));
  return b;
}

int plan2d_create(const ridc_problem* p, double h, double* const* ring, const int* R,
                  const double* W, const int64_t* woff, char* ws, size_t ws_bytes,
                  hipStream_t stream, Plan2D** out) {
  auto* pl = new Plan2D();
  pl->p = *p;
  pl->P = p->order;
  pl->prec = prec_of(p);
  pl->n = p->n;
  pl->h = h;
  pl->stream = stream;
  const int P = pl->P;
  const int64_t n = p->n, nn = n * n;
  Transform tf;
  int rc = get_transform(n, pl->prec, &tf);
  if (rc == RIDC_OK && prepare_pass_kernels(pl->prec) != hipSuccess)
    rc = fail(RIDC_E_HIP, "the transform kernels need more LDS than the device allows");
  if (rc != RIDC_OK) {
    delete pl;
    return rc;
  }
  pl->Q64 = tf.q64;
  pl->Q32 = tf.q32;
  pl->Qbf = tf.qbf;
  char* cur = ws;
  pl->d_levels = (Lvl2D*)cur;
  cur += align256(sizeof(Lvl2D) * P);
  pl->npass = pl->prec == PREC_F64 ? 4 : 8;
  pl->d_passes = (Pass2D*)cur;
  cur += align256(sizeof(Pass2D) * P * pl->npass);
  pl->lam = (double*)cur;
  cur += align256(sizeof(double) * n);
  // lam_k = dt nu (4/h^2) sin^2(pi (k+1) / (2(n+1)))
  {
    std::vector<double> lam(n);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int64_t k = 0; k < n; ++k) {
      const long double s = std::sin(pi * (long double)(k + 1) / (2.0L * (n + 1)));
      lam[k] = (double)((long double)p->dt * p->nu * 4.0L / ((long double)h * h) * s * s);
    }
    RIDC_HIP_TRY(hipMemcpy(pl->lam, lam.data(), n * sizeof(double), hipMemcpyHostToDevice));
  }
  pl->levels.assign(P, Lvl2D{});
  const size_t lws = align256(level_ws_bytes(n, pl->prec));
  for (int j = 0; j < P; ++j) {
    Lvl2D& L = pl->levels[j];
    L.own = ring[j];
    L.prev = j > 0 ? ring[j - 1] : nullptr;
    L.W = j > 0 ? W + woff[j] : nullptr;
    char* lw = cur + j * lws;
    L.b64 = (double*)lw;
    L.x64 = (double*)(lw + nn * sizeof(double));
    if (pl->prec != PREC_F64) {
      L.lo0 = lw + 2 * nn * sizeof(double);
      L.lo1 = lw + 2 * nn * sizeof(double) + nn * sizeof(float);
    }
    L.nt = 0;
    L.sigma0 = 0;
    L.n = (int32_t)n;
    L.j = j;
    L.R_own = R[j];
    L.R_prev = j > 0 ? R[j - 1] : 1;
    L.fe = p->fe_kind;
    L.prec = pl->prec;
    L.dt = p->dt;
    L.nu_h2 = p->nu / (h * h);
  }
  cur += P * lws;
  if ((size_t)(cur - ws) > ws_bytes) {
    delete pl;
    return fail(RIDC_E_NOMEM, "2D workspace layout overflow");
  }
  // pass tables: pass k, level j at passes[k * P + j]
  pl->passes.assign(pl->npass * P, Pass2D{});
  for (int j = 0; j < P; ++j) {
    Lvl2D& L = pl->levels[j];
    for (int k = 0; k < pl->npass; ++k) {
      Pass2D& E = pl->passes[k * P + j];
      E.level = j;
      E.lam = pl->lam;
      E.divide = (k % 4) == 1;
      if (pl->prec == PREC_F64) {
        E.Q = pl->Q64;
        const void* ins[4] = {L.b64, L.x64, L.b64, L.x64};
        void* outs[4] = {L.x64, L.b64, L.x64, nullptr};
        E.A = ins[k];
        E.C = outs[k];
      } else {
        E.Q = pl->prec == PREC_F32 ? (const void*)pl->Q32 : (const void*)pl->Qbf;
        const int kk = k % 4;
        const void* ins[4] = {L.lo0, L.lo1, L.lo0, L.lo1};
        void* outs[4] = {L.lo1, L.lo0, L.lo1, nullptr};
        E.A = ins[kk];
        E.C = outs[kk];
        if (k == 3) E.C = L.x64;             // first solve, kept in FP32 in this buffer
        if (k == 7) E.add = (const float*)L.x64;   // x = x1 + S~(rho)
      }
    }
  }
  RIDC_HIP_TRY(hipMemcpy(pl->d_passes, pl->passes.data(), sizeof(Pass2D) * pl->passes.size(),
                         hipMemcpyHostToDevice));
  {
    // the measured pass shape of this (n, precision), if the tuning table has one
    int tile = 0;
    if (tune_get_2d(p->n, p->prec, &tile)) (void)plan2d_set_tile(pl, tile);
    set_error("");
  }
  *out = pl;
  return RIDC_OK;
}

void plan2d_destroy(Plan2D* pl) { delete pl; }

int plan2d_tile(const Plan2D* pl) { return pl->tile; }

void plan2d_tile_candidates(const Plan2D* pl, std::vector<int>* out) {
  out->clear();
  out->push_back(0);
  if (pl->prec != PREC_BF16 && (!folded(pl->n) || pl->n % 128 == 0)) out->push_back(kPassWide64);
  if (pl->prec == PREC_BF16 && wide_slices<PREC_BF16>(pl->n)) out->push_back(kPassNarrowK);
  if (prefold(pl->n, 0)) {
    const size_t c = out->size();
    for (size_t i = 0; i < c; ++i) out->push_back((*out)[i] | kPassPlainA);
  }
}

int plan2d_set_tile(Plan2D* pl, int tile) {
  std::vector<int> c;
  plan2d_tile_candidates(pl, &c);
  if (std::find(c.begin(), c.end(), tile) == c.end())
    return fail(RIDC_E_INVAL, "launch shape not available for this side and precision");
  pl->tile = tile;
  return RIDC_OK;
}

int plan2d_arm(Plan2D* pl, int64_t nt, hipStream_t stream) {
  for (auto& L : pl->levels) {
    L.nt = nt;
    L.sigma0 = 0;
  }
  RIDC_HIP_TRY(hipMemcpyAsync(pl->d_levels, pl->levels.data(), sizeof(Lvl2D) * pl->levels.size(),
                              hipMemcpyHostToDevice, stream));
  return RIDC_OK;
}

namespace {

// The four passes of one solve (passes d[0 .. 3 cnt)): the last writes LAST.  With prefolded
// operands the first three write folded planes and the later three read them.
template <int PREC, int LAST>
void run_solve(const Lvl2D* lv, const Pass2D* d, int cnt, int64_t nmax, int64_t s, int tile,
               hipStream_t st) {
  constexpr int OWN = PREC == PREC_F64 ? OUT_F64 : OUT_F32;
  if (prefold(nmax, tile)) {
    launch_pass<PREC, OUT_FOLD, 0>(d + 0 * cnt, lv, cnt, nmax, s, tile, st);
    launch_pass<PREC, OUT_FOLD, 1>(d + 1 * cnt, lv, cnt, nmax, s, tile, st);
    launch_pass<PREC, OUT_FOLD, 1>(d + 2 * cnt, lv, cnt, nmax, s, tile, st);
    launch_pass<PREC, LAST, 1>(d + 3 * cnt, lv, cnt, nmax, s, tile, st);
  } else {
    launch_pass<PREC, OWN, 0>(d + 0 * cnt, lv, cnt, nmax, s, tile, st);
    launch_pass<PREC, OWN, 0>(d + 1 * cnt, lv, cnt, nmax, s, tile, st);
    launch_pass<PREC, OWN, 0>(d + 2 * cnt, lv, cnt, nmax, s, tile, st);
    launch_pass<PREC, LAST, 0>(d + 3 * cnt, lv, cnt, nmax, s, tile, st);
  }
}

// Every stage of one pipeline step for `cnt` (plan, level) entries of one precision: the
// right-hand side, the transform passes and (reduced precision) the residual, one launch each.
// passes is pass-major: passes[k * cnt + e].
void run_stages(int prec, const Lvl2D* lv, const Pass2D* d, int cnt, int64_t nmax, int64_t s,
                int tile, hipStream_t st) {
  launch_stencil(k_rhs2d, lv, cnt, nmax, s, st);
  if (prec == PREC_F64) {
    run_solve<PREC_F64, OUT_FINAL>(lv, d, cnt, nmax, s, tile, st);
  } else if (prec == PREC_F32) {
    run_solve<PREC_F32, OUT_F32>(lv, d, cnt, nmax, s, tile, st);
    launch_stencil(k_resid2d, lv, cnt, nmax, s, st);
    run_solve<PREC_F32, OUT_FINAL>(lv, d + 4 * cnt, cnt, nmax, s, tile, st);
  } else {
    run_solve<PREC_BF16, OUT_F32>(lv, d, cnt, nmax, s, tile, st);
    launch_stencil(k_resid2d, lv, cnt, nmax, s, st);
    run_solve<PREC_BF16, OUT_FINAL>(lv, d + 4 * cnt, cnt, nmax, s, tile, st);
  }
}

// Launch tables of grouped plans (one set per calling thread and device).  `done` follows the
// upload of the pinned staging copy (the host waits for it before rewriting the staging);
// `used` follows the last launch that read the device tables, and an upload on another stream
// waits for it on the device, so the tables are never rewritten under a running kernel.
struct Arena2D {
  int device = -1;
  Lvl2D* d_lv = nullptr;
  Pass2D* d_ps = nullptr;
  Lvl2D* h_lv = nullptr;
  Pass2D* h_ps = nullptr;
  size_t cap_lv = 0, cap_ps = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
  hipEvent_t used = nullptr;
  hipStream_t used_stream = nullptr;
  bool in_use = false;
};
thread_local Arena2D g_a2;

int arena2d_reserve(size_t nlv, size_t nps, hipStream_t stream) {
  int dev = 0;
  RIDC_HIP_TRY(hipGetDevice(&dev));
  if (g_a2.device != dev) {
    g_a2 = Arena2D{};
    g_a2.device = dev;
  }
  if (!g_a2.done) RIDC_HIP_TRY(hipEventCreateWithFlags(&g_a2.done, hipEventDisableTiming));
  if (!g_a2.used) RIDC_HIP_TRY(hipEventCreateWithFlags(&g_a2.used, hipEventDisableTiming));
  if (g_a2.pending) {
    RIDC_HIP_TRY(hipEventSynchronize(g_a2.done));
    g_a2.pending = false;
  }
  if (g_a2.in_use && g_a2.used_stream != stream)
    RIDC_HIP_TRY(hipStreamWaitEvent(stream, g_a2.used, 0));
  if (g_a2.in_use && (nlv > g_a2.cap_lv || nps > g_a2.cap_ps)) {
    RIDC_HIP_TRY(hipEventSynchronize(g_a2.used));   // a table is about to be freed
    g_a2.in_use = false;
  }
  if (nlv > g_a2.cap_lv) {
    if (g_a2.d_lv) (void)hipFree(g_a2.d_lv);
    if (g_a2.h_lv) (void)hipHostFree(g_a2.h_lv);
    g_a2.d_lv = nullptr;
    g_a2.h_lv = nullptr;
    const size_t cap = std::max(nlv, 2 * g_a2.cap_lv);
    if (hipMalloc(&g_a2.d_lv, cap * sizeof(Lvl2D)) != hipSuccess) return fail(RIDC_E_NOMEM, "2D level table");
    if (hipHostMalloc(&g_a2.h_lv, cap * sizeof(Lvl2D), hipHostMallocDefault) != hipSuccess)
      return fail(RIDC_E_NOMEM, "2D level staging");
    g_a2.cap_lv = cap;
  }
  if (nps > g_a2.cap_ps) {
    if (g_a2.d_ps) (void)hipFree(g_a2.d_ps);
    if (g_a2.h_ps) (void)hipHostFree(g_a2.h_ps);
    g_a2.d_ps = nullptr;
    g_a2.h_ps = nullptr;
    const size_t cap = std::max(nps, 2 * g_a2.cap_ps);
    if (hipMalloc(&g_a2.d_ps, cap * sizeof(Pass2D)) != hipSuccess) return fail(RIDC_E_NOMEM, "2D pass table");
    if (hipHostMalloc(&g_a2.h_ps, cap * sizeof(Pass2D), hipHostMallocDefault) != hipSuccess)
      return fail(RIDC_E_NOMEM, "2D pass staging");
    g_a2.cap_ps = cap;
  }
  return RIDC_OK;
}

}  // namespace

// Advance plans by `steps` pipeline steps.  A single plan uses its own tables.  Several plans
// are grouped by (precision, n): each group runs every stage of a step as one launch with one
// grid z-slice per (plan, level), with the same tile shapes as a single plan, so a plan's bits
// do not depend on its company.  Plan i's own step during launch step s is sigma_before[i] + s.
int plan2d_advance(Plan2D* const* pls, int count, const int64_t* sigma_before, int64_t steps,
                   hipStream_t stream) {
  if (count <= 0 || steps <= 0) return RIDC_OK;
  if (count == 1) {
    Plan2D* pl = pls[0];
    for (int64_t s = 1; s <= steps; ++s)
      run_stages(pl->prec, pl->d_levels, pl->d_passes, pl->P, pl->n, sigma_before[0] + s, pl->tile,
                 stream);
    RIDC_HIP_TRY(hipGetLastError());
    return RIDC_OK;
  }
  // groups keyed by (prec, n, launch shape), in first-seen order
  std::vector<std::pair<std::pair<int, int64_t>, std::vector<int>>> groups;
  size_t nlv = 0, nps = 0;
  for (int i = 0; i < count; ++i) {
    const auto key = std::make_pair(pls[i]->prec | (pls[i]->tile << 8), pls[i]->n);
    auto it = std::find_if(groups.begin(), groups.end(), [&](auto& g) { return g.first == key; });
    if (it == groups.end()) {
      groups.push_back({key, {}});
      it = groups.end() - 1;
    }
    it->second.push_back(i);
    nlv += pls[i]->P;
    nps += (size_t)pls[i]->P * pls[i]->npass;
  }
  int rc = arena2d_reserve(nlv, nps, stream);
  if (rc != RIDC_OK) return rc;
  struct G {
    int prec, cnt;
    int64_t n;
    size_t lv_off, ps_off;
    int tile;
  };
  std::vector<G> gs;
  size_t lo = 0, po = 0;
  for (auto& g : groups) {
    const int prec = g.first.first & 0xff;
    const int npass = prec == PREC_F64 ? 4 : 8;
    int cnt = 0;
    for (int i : g.second) cnt += pls[i]->P;
    G gg{prec, cnt, g.first.second, lo, po, g.first.first >> 8};
    int e = 0;
    for (int i : g.second) {
      Plan2D* pl = pls[i];
      for (int j = 0; j < pl->P; ++j) {
        Lvl2D L = pl->levels[j];
        L.sigma0 = -sigma_before[i];
        g_a2.h_lv[lo + e + j] = L;
        for (int k = 0; k < npass; ++k) {
          Pass2D E = pl->passes[k * pl->P + j];
          E.level = e + j;
          g_a2.h_ps[po + (size_t)k * cnt + e + j] = E;
        }
      }
      e += pl->P;
    }
    lo += cnt;
    po += (size_t)cnt * npass;
    gs.push_back(gg);
  }
  RIDC_HIP_TRY(hipMemcpyAsync(g_a2.d_lv, g_a2.h_lv, lo * sizeof(Lvl2D), hipMemcpyHostToDevice, stream));
  RIDC_HIP_TRY(hipMemcpyAsync(g_a2.d_ps, g_a2.h_ps, po * sizeof(Pass2D), hipMemcpyHostToDevice, stream));
  RIDC_HIP_TRY(hipEventRecord(g_a2.done, stream));
  g_a2.pending = true;
  for (int64_t s = 1; s <= steps; ++s)
    for (auto& g : gs)
      run_stages(g.prec, g_a2.d_lv + g.lv_off, g_a2.d_ps + g.ps_off, g.cnt, g.n, s, g.tile,
                 stream);
  RIDC_HIP_TRY(hipGetLastError());
  RIDC_HIP_TRY(hipEventRecord(g_a2.used, stream));
  g_a2.used_stream = stream;
  g_a2.in_use = true;
  return RIDC_OK;
}

int plan2d_time_pass(Plan2D* pl, int64_t sigma, int reps, hipStream_t stream, double* us) {
  const int P = pl->P;
  const int64_t n = pl->n;
  const int tile = pl->tile;
  const bool pf = prefold(n, tile);
  // inputs of the second pass of this step (the right-hand side and the first pass), then
  // `reps` back-to-back launches of the second pass, which only rewrites an intermediate
  launch_stencil(k_rhs2d, pl->d_levels, P, n, sigma, stream);
  auto pass = [&](int k) {
    const Pass2D* d = pl->d_passes + k * P;
    if (pl->prec == PREC_F64) {
      if (pf && k == 0) launch_pass<PREC_F64, OUT_FOLD, 0>(d, pl->d_levels, P, n, sigma, tile, stream);
      else if (pf) launch_pass<PREC_F64, OUT_FOLD, 1>(d, pl->d_levels, P, n, sigma, tile, stream);
      else launch_pass<PREC_F64, OUT_F64, 0>(d, pl->d_levels, P, n, sigma, tile, stream);
    } else if (pl->prec == PREC_F32) {
      if (pf && k == 0) launch_pass<PREC_F32, OUT_FOLD, 0>(d, pl->d_levels, P, n, sigma, tile, stream);
      else if (pf) launch_pass<PREC_F32, OUT_FOLD, 1>(d, pl->d_levels, P, n, sigma, tile, stream);
      else launch_pass<PREC_F32, OUT_F32, 0>(d, pl->d_levels, P, n, sigma, tile, stream);
    } else {
      if (pf && k == 0) launch_pass<PREC_BF16, OUT_FOLD, 0>(d, pl->d_levels, P, n, sigma, tile, stream);
      else if (pf) launch_pass<PREC_BF16, OUT_FOLD, 1>(d, pl->d_levels, P, n, sigma, tile, stream);
      else launch_pass<PREC_BF16, OUT_F32, 0>(d, pl->d_levels, P, n, sigma, tile, stream);
    }
  };
  pass(0);
  hipEvent_t a, b;
  RIDC_HIP_TRY(hipEventCreate(&a));
  RIDC_HIP_TRY(hipEventCreate(&b));
  pass(1);
  (void)hipEventRecord(a, stream);
  for (int r = 0; r < reps; ++r) pass(1);
  (void)hipEventRecord(b, stream);
  hipError_t e = hipEventSynchronize(b);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return fail(RIDC_E_HIP, std::string("pass timing: ") + hipGetErrorString(e));
  *us = 1e3 * (double)ms / reps;
  return RIDC_OK;
}

int plan2d_time_rhs(Plan2D* pl, int64_t sigma, int reps, hipStream_t stream, double* us,
                    double* bytes) {
  const int P = pl->P;
  const int64_t n = pl->n;
  // the right-hand side of this step, launched repeatedly (it rewrites the same values)
  launch_stencil(k_rhs2d, pl->d_levels, P, n, sigma, stream);
  hipEvent_t a, b;
  RIDC_HIP_TRY(hipEventCreate(&a));
  RIDC_HIP_TRY(hipEventCreate(&b));
  (void)hipEventRecord(a, stream);
  for (int r = 0; r < reps; ++r)
    launch_stencil(k_rhs2d, pl->d_levels, P, n, sigma, stream);
  (void)hipEventRecord(b, stream);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return fail(RIDC_E_HIP, std::string("rhs timing: ") + hipGetErrorString(e));
  *us = 1e3 * (double)ms / reps;
  // algorithmic bytes per point: level 0 reads its value (a 5-point stencil of one vector),
  // level j > 0 its value and j+1 window vectors; every level writes the FP64 right-hand side
  // and, in the mixed paths, its 4-byte low-precision copy
  const double lo = pl->prec == PREC_F64 ? 0.0 : 4.0;
  double per = 0.0;
  for (int j = 0; j < P; ++j) per += 8.0 * (j == 0 ? 1 : j + 2) + 8.0 + lo;
  *bytes = per * (double)n * (double)n;
  return RIDC_OK;
}

void plan2d_cost(const Plan2D* pl, double* bytes, double* flops) {
  const double n = (double)pl->n;
  const int passes = pl->prec == PREC_F64 ? 4 : 8;
  const double products = pl->prec == PREC_BF16 ? 3.0 : 1.0;
  // algorithmic flops of the transforms at steady state: P level solves of 4 (or 8) n^3 GEMMs
  *flops = 2.0 * n * n * n * passes * pl->P;
  (void)products;
  (void)bytes;
}

}  // namespace ridc
