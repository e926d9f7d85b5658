// 1D level-step kernel of the RIDC pipeline for gfx950.
//
// One launch advances every active (instance, level) work item of a batch by one pipeline step.
// A workgroup owns one work item, or one chunk of it, and fuses:
//   1. the right-hand side of the level's IMEX Euler step, computed straight from the level
//      rings: the predictor (section II, eq. imex_diffusion) or the corrector (section III-C,
//      eq. corr) with the (j+1)-node quadrature of f = f_E + f_I along level j-1;
//   2. the implicit solve (I - dt nu D2) x = rhs by parallel cyclic reduction in LDS;
//   3. the store of the new level value into the level's ring.
// Nothing but the new level value is written to HBM; f along the previous level is recomputed
// from that level's stored values (a 3-point stencil), so a step reads j+2 vectors for
// level j and writes one.
//
// Solve.  The matrix is tridiagonal with constant coefficients b = 1 + 2r, a = -r
// (r = dt nu / h^2).  Periodic grids give a cyclic system on m = n rows.  Dirichlet grids
// (zero ghosts) are solved as the odd extension to a cyclic system of m = 2n+2 rows (row 0 and
// row n+1 are the ghosts, rows n+2.. mirror rows n..1 with a sign flip), which reproduces the
// Dirichlet solution exactly.  Each PCR stage k updates every row with the same coefficient:
// d_i <- d_i - gamma_k (d_{i-s} + d_{i+s}), s = 2^k mod m; after the last stage x = d / divisor,
// taken as a product with the divisor's reciprocal.
// In "wrap" mode one workgroup holds the whole cycle and indexes it modulo m.  In "chunk" mode
// (used when the coupling falls below rounding after K stages) a workgroup computes B rows
// and carries a halo of 2^K - 1 rows on each side, recomputing the halo's right-hand side; the
// valid region shrinks by 2^k per stage.  Both modes perform the same operations on the same
// values for every output row, so results do not depend on the tiling.
#include "ridc_internal.h"

namespace ridc {

namespace {

// Global-memory views of descriptor pointers.  Pointers read from a launch table carry no
// address space, so the compiler would emit flat instructions, which also count against the LDS
// wait counter (every LDS wait would then wait for the outstanding global loads too).
typedef __attribute__((address_space(1))) double gdbl;
typedef __attribute__((address_space(1))) int gint;
template <typename X>
__device__ __forceinline__ __attribute__((address_space(1))) X* gp(X* p) {
  return (__attribute__((address_space(1))) X*)p;
}
template <typename X>
__device__ __forceinline__ const __attribute__((address_space(1))) X* gp(const X* p) {
  return (const __attribute__((address_space(1))) X*)p;
}

// One PCR update of a row: c - g (a + b), with one rounding of the product-sum (every path
// uses this so that all tilings give the same bits).
__device__ __forceinline__ double pcr_upd(double c, double a, double b, double g) {
  return __builtin_fma(-g, a + b, c);
}

// f_E at one point from its neighbours; ce is explicit_coeff(fe, a, h).
__device__ __forceinline__ double fe_eval(int fe, double ce, double um, double u0, double up) {
  if (fe == RIDC_FE_ADVECT_C2) return -ce * (up - um);
  if (fe == RIDC_FE_LOGISTIC) return u0 * (1.0 - u0);
  if (fe == RIDC_FE_ADVECT_UPWIND) return ce >= 0.0 ? -ce * (u0 - um) : -ce * (up - u0);
  if (fe == RIDC_FE_BURGERS) return -ce * (up * up - um * um);
  return 0.0;
}

// Per-workgroup view of one level step of level J: where the level's value and the previous
// level's window live this step, and the coefficients that fold eq. (corr) into one sum over the
// window:
//   rhs = u + dt f_E(u) + sum_i [ cf_i f_E(v_i) + cl_i L v_i ]
// with v_i = eta[J-1]_{s+i}, cf_i = dt (w_i - [s+i == n]), cl_i = dt (w_i - [s+i == n+1]).
// J is a template parameter so the window lives in registers.
template <int J>
struct Step {
  const gdbl* u;
  gdbl* out;
  const gdbl* v[J + 1];
  double cf[J + 1], cl[J + 1];
};

struct Geo {        // scalar problem data of a work item, copied out of the descriptor
  int n, M, fe;
  bool per;
  double dt, ce, nu_h2;
};

// The value v holds in lane - 1 (wave_shr:1) or lane + 1 (wave_shl:1) of the wavefront, moved
// as two 32-bit halves; lanes without a source receive 0.  All 64 lanes must be active.
__device__ __forceinline__ double from_lane_below(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_lane_above(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Right-hand sides of the cycle rows gbase + l, l in [0, count), written to d[l] by the waves of
// one workgroup (or level group): wave w of nw takes 62 consecutive rows per pass, its lane lam
// holding row base + lam - 1.  Each lane loads one value of each vector (coalesced, all loads in
// flight together) and takes its stencil neighbours from lanes lam -+ 1; lanes 0 and 63 only
// supply neighbours.  Cycle rows map to grid rows as: periodic g -> g; Dirichlet (the odd
// extension on M = 2n+2 rows) g in 1..n -> g - 1, mirror rows g >= n+2 -> M - g - 1 (the result
// negated, the neighbours' roles swapped), ghost rows 0 and n+1 hold zero -- which is also the
// value the zero-ghost stencil needs beyond either end.  Every row computes
//   u + dt f_E(u) + sum_i [cf_i f_E(v_i) + cl_i L v_i]
// at its grid row with the same operations in every tiling.  The pass loop is uniform per wave.
template <int J, bool PER>
__device__ __forceinline__ void rhs_rows_bc(const Geo& G, const Step<J>& S, int gbase, int count,
                                            double* __restrict__ d, int wave, int nw, int lane) {
  const int n = G.n, M = G.M;
  for (int base = wave * 62; base < count; base += nw * 62) {
    const int l = base + lane - 1;
    // lanes past `count` are unused except row `count` as a neighbour: clamp, so that every
    // cycle row lies in [gbase - 1, gbase + count], within (-M, 2M) for every caller
    int g = gbase + (l < count ? l : count);
    if (g < 0) g += M;
    else if (g >= M) g -= M;
    bool ghost = false, mir = false;
    int p = g;
    if constexpr (!PER) {
      ghost = g == 0 || g == n + 1;
      mir = g > n + 1;
      p = ghost ? 0 : (mir ? M - g - 1 : g - 1);
    }
    double u0 = S.u[p];
    double v0[J + 1];                       // the window of level J-1 (none for the predictor)
    if constexpr (J > 0) {
#pragma unroll
      for (int i = 0; i <= J; ++i) v0[i] = S.v[i][p];
#pragma unroll
      for (int i = 0; i <= J; ++i) v0[i] = ghost ? 0.0 : v0[i];
    }
    u0 = ghost ? 0.0 : u0;
    double um = from_lane_below(u0), up = from_lane_above(u0);
    if (mir) {
      const double t = um;
      um = up;
      up = t;
    }
    double acc = u0 + G.dt * fe_eval(G.fe, G.ce, um, u0, up);
#pragma unroll
    for (int i = 0; i < (J > 0 ? J + 1 : 0); ++i) {
      double vm = from_lane_below(v0[i]), vp = from_lane_above(v0[i]);
      if (mir) {
        const double t = vm;
        vm = vp;
        vp = t;
      }
      const double li = G.nu_h2 * ((vm + vp) - 2.0 * v0[i]);
      acc += S.cf[i] * fe_eval(G.fe, G.ce, vm, v0[i], vp) + S.cl[i] * li;
    }
    if (lane >= 1 && lane <= 62 && l < count) d[l] = ghost ? 0.0 : (mir ? -acc : acc);
  }
}

// periodic cycles have no ghost or mirror rows: their gather is compiled without them
template <int J>
__device__ __forceinline__ void rhs_rows(const Geo& G, const Step<J>& S, int gbase, int count,
                                         double* __restrict__ d, int wave, int nw, int lane) {
  if (G.per)
    rhs_rows_bc<J, true>(G, S, gbase, count, d, wave, nw, lane);
  else
    rhs_rows_bc<J, false>(G, S, gbase, count, d, wave, nw, lane);
}

// Everything one level step reads besides the rings: built from a descriptor table entry
// (batched launches) or from the kernel arguments (a single instance's launch).
struct View {
  gdbl* own;
  const gdbl* prev;
  const gdbl* W;
  const gdbl* gamma;
  const gint* shift;
  int R_own, R_prev, n, M, bc, fe, stages, wrap, B, H;
  double dt, ce, nu_h2, inv_divisor;
};

__device__ __forceinline__ void store_row(gdbl* p, double v, bool nt) {
  if (nt)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Geometry and this step's window of a level (shared by the per-step and the fused kernels).
template <int J>
__device__ __forceinline__ void make_step(const View& L, int64_t m, Geo& G, Step<J>& S) {
  G.n = L.n;
  G.M = L.M;
  G.fe = L.fe;
  G.per = L.bc == RIDC_BC_PERIODIC;
  G.dt = L.dt;
  G.ce = L.ce;
  G.nu_h2 = L.nu_h2;
  const int n = G.n;
  const int64_t nidx = m - 1;
  S.u = L.own + (nidx % L.R_own) * (int64_t)n;
  S.out = L.own + (m % L.R_own) * (int64_t)n;
  if constexpr (J > 0) {
    const int64_t s = m - J > 0 ? m - J : 0;          // window t_s..t_{s+J}
    const gdbl* w = L.W + (nidx - s) * (J + 1);       // row r = n - s
    const int R = L.R_prev;
    int slot = (int)(s % R);
#pragma unroll
    for (int i = 0; i <= J; ++i) {
      S.v[i] = L.prev + (int64_t)slot * n;
      slot = slot + 1 == R ? 0 : slot + 1;
      const int64_t node = s + i;
      const double wi = w[i];
      S.cf[i] = G.dt * (wi - (node == nidx ? 1.0 : 0.0));
      S.cl[i] = G.dt * (wi - (node == nidx + 1 ? 1.0 : 0.0));
    }
  }
}

template <int J, int T>
__device__ __forceinline__ void level_step(const View& L, int chunk, int64_t m, double* lds,
                                           bool nt_store) {
  Geo G;
  Step<J> S;
  make_step<J>(L, m, G, S);
  const int n = G.n, M = G.M;
  const bool per = G.per;
  const int stages = L.stages;
  const double inv_div = L.inv_divisor;
  const gdbl* __restrict__ gam = L.gamma;

  if (L.wrap) {
    const int ms = per ? n : n + 2;                   // stored rows of the cycle
    const gint* __restrict__ shift = L.shift;
    double* d0 = lds;
    double* d1 = lds + ms;
    rhs_rows<J>(G, S, 0, ms, d0, threadIdx.x >> 6, T / 64, threadIdx.x & 63);
    for (int l = threadIdx.x; l < ms; l += T) d1[l] = 0.0;
    __syncthreads();
    const int l0 = per ? 0 : 1, l1 = per ? n : n + 1;  // Dirichlet ghosts stay zero
    for (int k = 0; k < stages; ++k) {
      const int sh = shift[k];
      const double g = gam[k];
      for (int l = l0 + threadIdx.x; l < l1; l += T) {
        int ia = l - sh;
        if (ia < 0) ia += M;
        int ib = l + sh;
        if (ib >= M) ib -= M;
        double da, db;
        if (per) {
          da = d0[ia];
          db = d0[ib];
        } else {
          da = ia <= n + 1 ? d0[ia] : -d0[M - ia];
          db = ib <= n + 1 ? d0[ib] : -d0[M - ib];
        }
        d1[l] = pcr_upd(d0[l], da, db, g);
      }
      __syncthreads();
      double* t = d0;
      d0 = d1;
      d1 = t;
    }
    for (int l = l0 + threadIdx.x; l < l1; l += T)
      store_row(S.out + (per ? l : l - 1), d0[l] * inv_div, nt_store);
    return;
  }

  // chunk mode: rows [g0, g0 + B) of the cycle plus a halo of H rows each side
  const int B = L.B, H = L.H, E = B + 2 * H;
  const int g0 = (per ? 0 : 1) + chunk * B;
  double* d0 = lds;
  double* d1 = lds + E;
  // cycle rows g0 - H - 1 .. g0 + B + H lie in (-M, 2M): H < M and B + H <= n
  rhs_rows<J>(G, S, g0 - H, E, d0, threadIdx.x >> 6, T / 64, threadIdx.x & 63);
  __syncthreads();
  // stages in pairs: stage k+1 of row l needs stage k at l and l +- 2s, i.e. the inputs at
  // l + t s, |t| <= 3 -- one barrier per pair, the same operations as one stage at a time
  int k = 0;
  for (; k + 1 < stages; k += 2) {
    const int sh = 1 << k;
    const int reach = (1 << stages) - (4 << k);       // rows beyond the chunk still needed
    const int lo = H - reach, hi = H + B + reach;
    const double ga = gam[k], gb = gam[k + 1];
    for (int l = lo + threadIdx.x; l < hi; l += T) {
      const double m3 = d0[l - 3 * sh], m2 = d0[l - 2 * sh], m1 = d0[l - sh], c = d0[l];
      const double p1 = d0[l + sh], p2 = d0[l + 2 * sh], p3 = d0[l + 3 * sh];
      const double lm = pcr_upd(m2, m3, m1, ga);      // stage k at l - 2s
      const double lc = pcr_upd(c, m1, p1, ga);       // stage k at l
      const double lp = pcr_upd(p2, p1, p3, ga);      // stage k at l + 2s
      d1[l] = pcr_upd(lc, lm, lp, gb);
    }
    __syncthreads();
    double* t = d0;
    d0 = d1;
    d1 = t;
  }
  if (k < stages) {
    const int sh = 1 << k;
    const int reach = (1 << stages) - (2 << k);
    const int lo = H - reach, hi = H + B + reach;
    const double g = gam[k];
    for (int l = lo + threadIdx.x; l < hi; l += T) d1[l] = pcr_upd(d0[l], d0[l - sh], d0[l + sh], g);
    __syncthreads();
    double* t = d0;
    d0 = d1;
    d1 = t;
  }
  const int last = per ? n : n + 1;                   // one past the last physical row of g
  for (int l = H + threadIdx.x; l < H + B; l += T) {
    const int g = g0 - H + l;
    if (g < last) store_row(S.out + (per ? g : g - 1), d0[l] * inv_div, nt_store);
  }
}

// Level j of a work item runs level_step<j>.  A kernel instantiates the levels up to MJ only
// (the host picks MJ from the highest order in the launch), so that the register budget of an
// order-4 launch is that of the level-3 body and not of the largest level; 1024-thread kernels
// stop at kMaxJ1024 (128 registers per thread).
template <int T, int MJ>
__device__ __forceinline__ void dispatch_level(int j, const View& v, int chunk, int64_t m,
                                               double* lds, bool nt) {
  switch (j) {
    case 0: level_step<0, T>(v, chunk, m, lds, nt); break;
    case 1: if constexpr (MJ >= 1) level_step<1, T>(v, chunk, m, lds, nt); break;
    case 2: if constexpr (MJ >= 2) level_step<2, T>(v, chunk, m, lds, nt); break;
    case 3: if constexpr (MJ >= 3) level_step<3, T>(v, chunk, m, lds, nt); break;
    case 4: if constexpr (MJ >= 4) level_step<4, T>(v, chunk, m, lds, nt); break;
    case 5: if constexpr (MJ >= 5) level_step<5, T>(v, chunk, m, lds, nt); break;
    case 6: if constexpr (MJ >= 6) level_step<6, T>(v, chunk, m, lds, nt); break;
    case 7: if constexpr (MJ >= 7) level_step<7, T>(v, chunk, m, lds, nt); break;
    case 8: if constexpr (MJ >= 8) level_step<8, T>(v, chunk, m, lds, nt); break;
    case 9: if constexpr (MJ >= 9) level_step<9, T>(v, chunk, m, lds, nt); break;
    case 10: if constexpr (MJ >= 10) level_step<10, T>(v, chunk, m, lds, nt); break;
    case 11: if constexpr (MJ >= 11) level_step<11, T>(v, chunk, m, lds, nt); break;
    default: break;
  }
}

template <int T, int MJ>
__global__ __launch_bounds__(T) void k_step1d(const Lvl1D* __restrict__ items,
                                              const Blk1D* __restrict__ blocks, int64_t sigma) {
  extern __shared__ double lds[];
  const Blk1D bk = blocks[blockIdx.x];
  const Lvl1D* L = items + bk.item;
  const int j = L->j;
  const int64_t m = sigma - L->sigma0 - (int64_t)j * (j + 1) / 2;  // time index computed now
  if (m < 1 || m > L->nt) return;                                   // level idle this step
  View v{gp(L->own), gp(L->prev), gp(L->W), gp(L->gamma), gp(L->shift), L->R_own, L->R_prev,
         L->n, L->M, L->bc,
         L->fe, L->stages, L->wrap, L->B, L->H, L->dt, L->ce, L->nu_h2, L->inv_divisor};
  dispatch_level<T, MJ>(j, v, bk.chunk, m, lds, false);
}

// A single instance's step with every descriptor in the kernel arguments: block b handles level
// b / nchunks, chunk b % nchunks, so the first memory access of a block is its data.
template <int T, int MJ>
__global__ __launch_bounds__(T) void k_step1d_solo(const Solo1D a, int64_t sigma) {
  extern __shared__ double lds[];
  const int j = blockIdx.x / a.nchunks;
  const int chunk = blockIdx.x - j * a.nchunks;
  const int64_t m = sigma - (int64_t)j * (j + 1) / 2;
  if (m < 1 || m > a.nt) return;
  View v{gp(a.ring[j]), gp(j > 0 ? a.ring[j - 1] : nullptr), gp(a.W[j]), gp(a.gamma),
         gp(a.shift), a.R[j],
         j > 0 ? a.R[j - 1] : 1, a.n, a.M, a.bc, a.fe, a.stages, a.wrap, a.B, a.H, a.dt,
         a.ce, a.nu_h2, a.inv_divisor};
  dispatch_level<T, MJ>(j, v, chunk, m, lds, a.nt_store != 0);
}

// ---------------------------------------------------------------------------------------------
// Fused integration: one workgroup owns one instance for a range of pipeline steps.  The P levels
// run concurrently in P thread groups of G threads (whole waves); every group does the
// same PCR stages, so all groups share the workgroup barriers.  Each group solves its level's
// whole cycle in its own LDS region (the "wrap" tiling of the per-step kernel, with the same
// operations per row, so results are bitwise those of the per-step kernel).  The level rings
// stay in global memory, hot in this CU's caches; a barrier after the stores makes a step's
// values visible to the next step's loads.
// ---------------------------------------------------------------------------------------------
// Thread lt of a level group owns rows l0 + lt + r G, r < RPT (RHS rows: lt + r G of [0, ms)).
// Every phase first gathers what all of its rows need into registers, so the loads of a phase
// are in flight together, then computes, then writes.
template <int J>
__device__ __forceinline__ void fused_rhs(const View& L, int64_t m, double* d, int lt, int G) {
  Geo g;
  Step<J> S;
  make_step<J>(L, m, g, S);
  const int ms = g.per ? g.n : g.n + 2;
  rhs_rows<J>(g, S, 0, ms, d, lt >> 6, G / 64, lt & 63);
}

template <int MJ>
__device__ __forceinline__ void fused_rhs_any(int j, const View& v, int64_t m, double* d, int lt,
                                              int G) {
  // levels up to MJ are instantiated (the host sends orders up to MJ + 1)
  switch (j) {
    case 0: fused_rhs<0>(v, m, d, lt, G); break;
    case 1: if constexpr (MJ >= 1) fused_rhs<1>(v, m, d, lt, G); break;
    case 2: if constexpr (MJ >= 2) fused_rhs<2>(v, m, d, lt, G); break;
    case 3: if constexpr (MJ >= 3) fused_rhs<3>(v, m, d, lt, G); break;
    case 4: if constexpr (MJ >= 4) fused_rhs<4>(v, m, d, lt, G); break;
    default: if constexpr (MJ >= 5) fused_rhs<5>(v, m, d, lt, G); break;
  }
}

// Two LDS buffers per level, one barrier per stage.
template <int MJ>
__device__ __forceinline__ void fused_body(const Fused1D& F) {
  extern __shared__ double lds[];
  const int P = F.P;
  const int G = F.group;                     // threads per level group (blockDim.x / P, waves)
  const int j = threadIdx.x / G;             // this thread's level (j >= P: idle)
  const int lt = threadIdx.x - j * G;
  const bool mine = j < P;
  const int n = F.n, M = F.M;
  const bool per = F.bc == RIDC_BC_PERIODIC;
  const int ms = per ? n : n + 2;
  const int l0 = per ? 0 : 1, l1 = per ? n : n + 1;
  double* d0 = lds + (mine ? j : 0) * 2 * ms;
  double* d1 = d0 + ms;
  View v{};
  if (mine) {
    v = View{gp(F.ring[j]), gp(j > 0 ? F.ring[j - 1] : nullptr), gp(F.W[j]), gp(F.gamma),
             gp(F.shift), F.R[j],
             j > 0 ? F.R[j - 1] : 1, n, M, F.bc, F.fe, F.stages, 1, 0, 0, F.dt, F.ce, F.nu_h2,
             F.inv_divisor};
    // Dirichlet ghost rows (0 and n+1) must read zero in both buffers whatever their roles: a
    // level waiting for its start-up swaps the buffers without writing them
    for (int l = lt; l < ms; l += G) {
      d0[l] = 0.0;
      d1[l] = 0.0;
    }
  }
  const int stages = F.stages;
  for (int64_t sigma = F.sigma_first + 1; sigma <= F.sigma_last; ++sigma) {
    const int64_t m = sigma - F.sigma0 - (int64_t)j * (j + 1) / 2;
    const bool act = mine && m >= 1 && m <= F.nt;
    if (act) fused_rhs_any<MJ>(j, v, m, d0, lt, G);
    __syncthreads();
    for (int k = 0; k < stages; ++k) {
      const int sh = gp(F.shift)[k];
      const double g = gp(F.gamma)[k];
      if (act) {
        constexpr int RB = 4;                 // rows gathered together
#pragma unroll 1
        for (int base = l0 + lt; base < l1; base += RB * G) {
          double c[RB], a[RB], b[RB];
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            const int l = base + r * G;
            c[r] = a[r] = b[r] = 0.0;
            if (l < l1) {
              int ia = l - sh;
              if (ia < 0) ia += M;
              int ib = l + sh;
              if (ib >= M) ib -= M;
              c[r] = d0[l];
              if (per) {
                a[r] = d0[ia];
                b[r] = d0[ib];
              } else {
                a[r] = ia <= n + 1 ? d0[ia] : -d0[M - ia];
                b[r] = ib <= n + 1 ? d0[ib] : -d0[M - ib];
              }
            }
          }
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            const int l = base + r * G;
            if (l < l1) d1[l] = pcr_upd(c[r], a[r], b[r], g);
          }
        }
      }
      __syncthreads();
      double* t = d0;
      d0 = d1;
      d1 = t;
    }
    if (act) {
      gdbl* out = gp(F.ring[j]) + (m % F.R[j]) * (int64_t)n;
      for (int l = l0 + lt; l < l1; l += G) out[per ? l : l - 1] = d0[l] * F.inv_divisor;
    }
    __syncthreads();                         // this step's values before the next step reads
  }
}

template <int MJ, int FT>
__global__ __launch_bounds__(FT) void k_fused1d(const Fused1D* __restrict__ items) {
  fused_body<MJ>(items[blockIdx.x]);
}

// One instance, descriptor in the kernel arguments.
template <int MJ, int FT>
__global__ __launch_bounds__(FT) void k_fused1d_one(const Fused1D F) {
  fused_body<MJ>(F);
}


__global__ void k_nonfinite(const double* __restrict__ x, int64_t count, int* flag) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = x[i];
    if (!(v - v == 0.0)) bad = 1;      // NaN or Inf
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// Item blockIdx.y of a copy list, strided over blockIdx.x; flags non-finite values when asked.
__global__ void k_copy_items(const CopyItem* __restrict__ items) {
  const CopyItem it = items[blockIdx.y];
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < it.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = gp(it.src)[i];
    gp(it.dst)[i] = v;
    if (!(v - v == 0.0)) bad = 1;      // NaN or Inf
  }
  if (it.flag && __any(bad) && (threadIdx.x & 63) == 0) atomicOr(it.flag, 1);
}

}  // namespace

hipError_t launch_copy_items(const CopyItem* d_items, int count, int64_t max_n,
                             hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  int64_t bx = (max_n + 1023) / 1024;
  if (bx < 1) bx = 1;
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(k_copy_items, dim3((unsigned)bx, (unsigned)count), dim3(256), 0, stream,
                     d_items);
  return hipGetLastError();
}

size_t lds_bytes_1d(const Lvl1D& it) {
  if (it.wrap) {
    const int ms = it.bc == RIDC_BC_PERIODIC ? it.n : it.n + 2;
    return 2 * sizeof(double) * (size_t)ms;
  }
  return 2 * sizeof(double) * (size_t)(it.B + 2 * it.H);
}

namespace {

// Highest level index instantiated for a launch whose highest order is max_order: 3 (orders up
// to 4), kMaxJ1024 (orders up to kMaxJ1024 + 1) or kMaxOrder - 1; -1 if no kernel of `threads`
// threads covers it.
int level_bound(int max_order, int threads) {
  if (max_order <= 4) return 3;
  if (max_order <= kMaxJ1024 + 1) return kMaxJ1024;
  if (threads < 1024 && max_order <= kMaxOrder) return kMaxOrder - 1;
  return -1;
}

template <int T, int MJ>
hipError_t allow_lds_t(size_t lds_bytes) {
  static size_t allowed = 65536;
  if (lds_bytes > allowed) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step1d<T, MJ>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step1d_solo<T, MJ>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    allowed = lds_bytes;
  }
  return hipSuccess;
}

template <int T, int MJ>
hipError_t step_t(const Lvl1D* d_items, const Blk1D* d_blocks, const Solo1D* solo, int nblocks,
                  size_t lds_bytes, int64_t sigma, hipStream_t stream) {
  if (solo)
    hipLaunchKernelGGL((k_step1d_solo<T, MJ>), dim3(nblocks), dim3(T), lds_bytes, stream, *solo,
                       sigma);
  else
    hipLaunchKernelGGL((k_step1d<T, MJ>), dim3(nblocks), dim3(T), lds_bytes, stream, d_items,
                       d_blocks, sigma);
  return hipGetLastError();
}

// prepare (launch == false) or launch one step with T threads and the level bound of max_order
template <int T>
hipError_t step_threads(bool launch, int max_order, const Lvl1D* d_items, const Blk1D* d_blocks,
                        const Solo1D* solo, int nblocks, size_t lds, int64_t sigma,
                        hipStream_t stream) {
  switch (level_bound(max_order, T)) {
    case 3:
      return launch ? step_t<T, 3>(d_items, d_blocks, solo, nblocks, lds, sigma, stream)
                    : allow_lds_t<T, 3>(lds);
    case kMaxJ1024:
      return launch ? step_t<T, kMaxJ1024>(d_items, d_blocks, solo, nblocks, lds, sigma, stream)
                    : allow_lds_t<T, kMaxJ1024>(lds);
    case kMaxOrder - 1:
      if constexpr (T < 1024)
        return launch ? step_t<T, kMaxOrder - 1>(d_items, d_blocks, solo, nblocks, lds, sigma,
                                                 stream)
                      : allow_lds_t<T, kMaxOrder - 1>(lds);
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t step_any(bool launch, int threads, int max_order, const Lvl1D* d_items,
                    const Blk1D* d_blocks, const Solo1D* solo, int nblocks, size_t lds,
                    int64_t sigma, hipStream_t stream) {
  switch (threads) {
    case 64:
      return step_threads<64>(launch, max_order, d_items, d_blocks, solo, nblocks, lds, sigma,
                              stream);
    case 128:
      return step_threads<128>(launch, max_order, d_items, d_blocks, solo, nblocks, lds, sigma,
                               stream);
    case 256:
      return step_threads<256>(launch, max_order, d_items, d_blocks, solo, nblocks, lds, sigma,
                               stream);
    case 512:
      return step_threads<512>(launch, max_order, d_items, d_blocks, solo, nblocks, lds, sigma,
                               stream);
    case 1024:
      return step_threads<1024>(launch, max_order, d_items, d_blocks, solo, nblocks, lds, sigma,
                                stream);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t prepare_1d_step(int threads, int max_order, size_t lds_bytes) {
  return step_any(false, threads, max_order, nullptr, nullptr, nullptr, 0, lds_bytes, 0, nullptr);
}

hipError_t launch_1d_step(const Lvl1D* d_items, const Blk1D* d_blocks, int nblocks, int threads,
                          int max_order, size_t lds_bytes, int64_t sigma, hipStream_t stream) {
  if (nblocks <= 0) return hipSuccess;
  return step_any(true, threads, max_order, d_items, d_blocks, nullptr, nblocks, lds_bytes, sigma,
                  stream);
}

hipError_t launch_1d_solo(const Solo1D& a, int nblocks, int threads, int max_order,
                          size_t lds_bytes, int64_t sigma, hipStream_t stream) {
  if (nblocks <= 0) return hipSuccess;
  return step_any(true, threads, max_order, nullptr, nullptr, &a, nblocks, lds_bytes, sigma,
                  stream);
}

namespace {

template <int MJ, int FT>
hipError_t fused_launch(const Fused1D* d_items, const Fused1D* one, int count, size_t lds,
                        hipStream_t stream) {
  static size_t allowed_tab = 65536, allowed_one = 65536;
  if (one) {
    if (lds > allowed_one) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused1d_one<MJ, FT>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      allowed_one = lds;
    }
    hipLaunchKernelGGL((k_fused1d_one<MJ, FT>), dim3(1), dim3(FT), lds, stream, *one);
  } else {
    if (lds > allowed_tab) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused1d<MJ, FT>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      allowed_tab = lds;
    }
    hipLaunchKernelGGL((k_fused1d<MJ, FT>), dim3(count), dim3(FT), lds, stream, d_items);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fused_1d(const Fused1D* d_items, const Fused1D* one, int count, int max_order,
                           int threads, size_t lds_bytes, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (threads == 512) {
    if (max_order <= 4) return fused_launch<3, 512>(d_items, one, count, lds_bytes, stream);
    if (max_order <= kMaxJ1024 + 1)
      return fused_launch<kMaxJ1024, 512>(d_items, one, count, lds_bytes, stream);
  } else if (threads == 1024) {
    // orders 5 and 6 would spill at 1024 threads (128 registers): they take 512
    if (max_order <= 4) return fused_launch<3, 1024>(d_items, one, count, lds_bytes, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_nonfinite_check(const double* x, int64_t count, int* flag, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)blocks), dim3(256), 0, stream, x, count, flag);
  return hipGetLastError();
}

}  // namespace ridc
