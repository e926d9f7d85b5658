// 1D level step of ARK-based RIDC and of RIDC with a nonlinear stiff term, for gfx950.
//
// One workgroup advances one (instance, level) work item by one pipeline step: it computes the
// level's value at t_{n+1} from its value at t_n with the s stages of the level's IMEX pair
// (section II):
//   Y_i = y_n + I_i + dt sum_{l<i} (AS_il K^S_l + AN_il K^N_l) + dt AS_ii K^S_i,
//   K^S_i = f^S(Y_i) - f^S(eta(t_n + c_i dt)),  K^N_i = f^N(Y_i) - f^N(eta(t_n + c_i dt)),
// where, for a corrector (section III-A, the integral form of the error equation), eta is the
// previous level interpolated through its S stored nodes (the section III-C window widened to
// S nodes) and I_i = int_{t_n}^{t_n + c_i dt} f(eta); for the predictor I_i and the subtracted
// terms are zero.  Every pair is stiffly accurate, so y_{n+1} = Y_s.  Stage 0 is explicit with
// c_0 = 0 (Y_0 = y_n); every other stage solves y - tau f^S(y) = rhs, tau = dt AS_ii:
//  - f^S = nu Lap_h: one tridiagonal solve (I - tau nu D2) y = rhs;
//  - f^S = nu Lap_h + kappa g: Newton's method (section III-B), each iterate solving the
//    Jacobian system (I - tau (nu D2 + kappa diag g'(y))) delta = rhs - (y - tau f^S(y)) and
//    stopping when the update reaches rounding.
// The implicit stage derivative is taken from the stage equation, f^S(Y_i) = (Y_i - rhs)/tau.
// The new value and f = f^S + f^N of it (read by the next level's window) go to the level's
// rings.
//
// Layout.  Thread t of T owns the M consecutive rows g0 = t M .. g0 + M - 1 in registers; rows
// at or past n are padding (identity rows, value 0).  Stencil neighbours of loaded vectors come
// from global memory; those of computed values from the edge exchange in LDS.
//
// Tridiagonal solve (a partition method): each thread eliminates its block so that every row
// couples only to the block's first and last unknowns, leaving a tridiagonal system of two
// rows per thread, which parallel cyclic reduction solves in LDS (one barrier per stage, two
// LDS buffers); the interior rows follow by back substitution.  Periodic grids (cyclic
// systems) take the Sherman-Morrison correction: the cyclic matrix is a tridiagonal one plus
// a rank-one term, so one solve with two right-hand sides and a scalar combination give the
// cyclic solution.
#include "ridc_internal.h"

namespace ridc {

namespace {

// f_E at one point from its neighbours; ce is explicit_coeff(fe, a, h).
__device__ __forceinline__ double fe_eval(int fe, double ce, double um, double u0, double up) {
  if (fe == RIDC_FE_ADVECT_C2) return -ce * (up - um);
  if (fe == RIDC_FE_LOGISTIC) return u0 * (1.0 - u0);
  if (fe == RIDC_FE_ADVECT_UPWIND) return ce >= 0.0 ? -ce * (u0 - um) : -ce * (up - u0);
  if (fe == RIDC_FE_BURGERS) return -ce * (up * up - um * um);
  return 0.0;
}

// g and g' of the stiff reaction
__device__ __forceinline__ double react(int fs, double u) {
  if (fs == RIDC_FS_LOGISTIC) return u * (1.0 - u);
  if (fs == RIDC_FS_CUBIC) return u - u * u * u;
  return 0.0;
}
__device__ __forceinline__ double react_prime(int fs, double u) {
  if (fs == RIDC_FS_LOGISTIC) return 1.0 - 2.0 * u;
  if (fs == RIDC_FS_CUBIC) return 1.0 - 3.0 * u * u;
  return 0.0;
}

// Per-workgroup state: problem data, thread position and the LDS regions (each region has two
// buffers used alternately, so that one barrier per use keeps readers and writers apart).
// Buffer k of a region is base + (k & 1) * stride (pointer arithmetic, not an indexed array,
// so that the context stays in registers).
struct Ctx {
  int n, T, t, g0, fe, fs;
  double ce, nu_h2, kappa;
  double* pcr;     // PCR buffers: left coefficients (2T), right coefficients (2T), rhs (NR x 2T)
  double* ex;      // edge exchange: first rows (NR x T), last rows (NR x T), rows 0 and n-1
  double* red;     // workgroup reductions: 2 values per wave (32 doubles per buffer)
  int pstride, xstride;
  int pk, xk, rk;  // buffer toggles
};

// LDS doubles of a workgroup of T threads with NR right-hand sides (layout as in imex_step)
inline size_t lds_doubles(int NR, int T) {
  return 2 * (size_t)(2 * T) * (2 + NR) + 2 * (size_t)(NR * (2 * T + 2)) + 2 * 32;
}

// Publish this thread's first and last rows (and rows 0 and n-1 from their owners), then read
// the neighbours of the block: xl = row g0-1, xr = row g0+M (0 past either end), w0 = row 0,
// wn = row n-1.
template <int M, int NR>
__device__ __forceinline__ void exchange(Ctx& c, const double (&x)[NR][M], double (&xl)[NR],
                                         double (&xr)[NR], double (&w0)[NR], double (&wn)[NR]) {
  double* e = c.ex + (c.xk & 1) * c.xstride;
  c.xk++;
  const int T = c.T, t = c.t;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    e[r * T + t] = x[r][0];
    e[NR * T + r * T + t] = x[r][M - 1];
  }
  if (t == 0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) e[2 * NR * T + r] = x[r][0];
  }
#pragma unroll
  for (int i = 0; i < M; ++i)
    if (c.g0 + i == c.n - 1) {
#pragma unroll
      for (int r = 0; r < NR; ++r) e[2 * NR * T + NR + r] = x[r][i];
    }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    xl[r] = t > 0 ? e[NR * T + r * T + t - 1] : 0.0;
    xr[r] = t + 1 < T ? e[r * T + t + 1] : 0.0;
    w0[r] = e[2 * NR * T + r];
    wn[r] = e[2 * NR * T + NR + r];
  }
}

// Stencil neighbours of local row i of a register block x with block neighbours xl, xr;
// periodic grids wrap rows 0 and n-1 (w0, wn: their values).
template <int M, bool PER>
__device__ __forceinline__ void nbrs(const Ctx& c, const double (&x)[M], int i, double xl,
                                     double xr, double w0, double wn, double& um, double& up) {
  um = i > 0 ? x[i - 1] : xl;
  up = i < M - 1 ? x[i + 1] : xr;
  if (PER) {
    const int g = c.g0 + i;
    if (g == 0) um = wn;
    if (g == c.n - 1) up = w0;
  }
}

// Value of a global vector at row g in [-1, n]: zero ghosts (Dirichlet) or wrapped (periodic).
template <bool PER>
__device__ __forceinline__ double ld(const double* __restrict__ v, int g, int n) {
  if (g >= 0 && g < n) return v[g];
  if (PER) {
    if (g == -1) return v[n - 1];
    if (g == n) return v[0];
  }
  return 0.0;
}

// Rows g0-1 .. g0+M of a global vector (blocks away from both ends: plain loads).
template <int M, bool PER>
__device__ __forceinline__ void load_halo(const Ctx& c, const double* __restrict__ v,
                                          double (&out)[M + 2]) {
  if (c.g0 >= 1 && c.g0 + M < c.n) {
    const double* p = v + c.g0 - 1;
#pragma unroll
    for (int i = 0; i < M + 2; ++i) out[i] = p[i];
    return;
  }
#pragma unroll
  for (int i = 0; i < M + 2; ++i) out[i] = ld<PER>(v, c.g0 + i - 1, c.n);
}

// Rows g0 .. g0+M-1: 16-byte loads when the block is inside the grid and 16-byte aligned.
template <int M>
__device__ __forceinline__ void load_rows(const Ctx& c, const double* __restrict__ v,
                                          double (&out)[M]) {
  if (c.g0 + M <= c.n && (reinterpret_cast<uintptr_t>(v + c.g0) & 15) == 0) {
    const double2* p = reinterpret_cast<const double2*>(v + c.g0);
#pragma unroll
    for (int i = 0; i < M / 2; ++i) {
      const double2 q = p[i];
      out[2 * i] = q.x;
      out[2 * i + 1] = q.y;
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < M; ++i) out[i] = c.g0 + i < c.n ? v[c.g0 + i] : 0.0;
}

template <int M>
__device__ __forceinline__ void store_rows(const Ctx& c, double* __restrict__ v,
                                           const double (&x)[M]) {
  if (c.g0 + M <= c.n && (reinterpret_cast<uintptr_t>(v + c.g0) & 15) == 0) {
    double2* p = reinterpret_cast<double2*>(v + c.g0);
#pragma unroll
    for (int i = 0; i < M / 2; ++i) p[i] = make_double2(x[2 * i], x[2 * i + 1]);
    return;
  }
#pragma unroll
  for (int i = 0; i < M; ++i)
    if (c.g0 + i < c.n) v[c.g0 + i] = x[i];
}

// f^S = nu Lap_h u + kappa g(u) and f^N at one row.
__device__ __forceinline__ double fstiff(const Ctx& c, double um, double u0, double up) {
  return c.nu_h2 * (up - 2.0 * u0 + um) + c.kappa * react(c.fs, u0);
}

// Largest of two values over the workgroup (both non-negative).
__device__ __forceinline__ void wg_max2(Ctx& c, double& a, double& b) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a = fmax(a, __shfl_xor(a, off, 64));
    b = fmax(b, __shfl_xor(b, off, 64));
  }
  double* r = c.red + (c.rk & 1) * 32;
  c.rk++;
  const int wave = c.t >> 6, nw = c.T >> 6;
  if ((c.t & 63) == 0) {
    r[2 * wave] = a;
    r[2 * wave + 1] = b;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  for (int w = 0; w < nw; ++w) {
    a = fmax(a, r[2 * w]);
    b = fmax(b, r[2 * w + 1]);
  }
}

// Solve the tridiagonal system with off-diagonals -r (zero at Dirichlet ends; periodic: cyclic
// with corners -r) whose diagonal b_g and right-hand side d_g (NR = 1) this thread's rows get
// from rows(i, b, d).  x receives this thread's rows of the solution (padding rows: 0).
// Periodic (PER): d0 is the diagonal of row 0; the second right-hand side is the rank-one
// correction's vector.
template <int M, bool PER, typename Rows>
__device__ __forceinline__ void tri_solve(Ctx& c, double r, double d0, Rows rows,
                                          double (&x)[M]) {
  constexpr int NR = PER ? 2 : 1;
  const int n = c.n, g0 = c.g0;
  double A[M], C[M], D[NR][M];
  double a0n = 0.0, c0n = 0.0, D0n[NR];
  // forward: row 0 normalised; rows 1..M-1 to  A_i x_0 + x_i + C_i x_{i+1} = D_i
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const int g = g0 + i;
    const bool real = g < n;
    double b = 1.0, d[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) d[q] = 0.0;
    if (real) {
      double dd;
      rows(i, b, dd);
      d[0] = dd;
    }
    const double lo = (!real || g == 0) ? 0.0 : -r;
    const double up = (!real || g == n - 1) ? 0.0 : -r;
    if (PER) {
      if (g == 0) {
        b += d0;            // b - gamma, gamma = -d0
        d[NR - 1] = -d0;    // u_0 = gamma
      }
      if (g == n - 1) {
        b += r * r / d0;    // b - a_0 c_{n-1} / gamma
        d[NR - 1] = -r;     // u_{n-1} = c_{n-1}
      }
    }
    if (i == 0) {
      const double inv = 1.0 / b;
      a0n = lo * inv;
      c0n = up * inv;
#pragma unroll
      for (int q = 0; q < NR; ++q) D0n[q] = d[q] * inv;
    } else if (i == 1) {
      const double inv = 1.0 / b;
      A[1] = lo * inv;
      C[1] = up * inv;
#pragma unroll
      for (int q = 0; q < NR; ++q) D[q][1] = d[q] * inv;
    } else {
      const double inv = 1.0 / (b - lo * C[i - 1]);
      A[i] = -lo * A[i - 1] * inv;
      C[i] = up * inv;
#pragma unroll
      for (int q = 0; q < NR; ++q) D[q][i] = (d[q] - lo * D[q][i - 1]) * inv;
    }
  }
  // backward: rows M-2..1 to  A_i x_0 + x_i + C_i x_{M-1} = D_i
#pragma unroll
  for (int i = M - 3; i >= 1; --i) {
    A[i] -= C[i] * A[i + 1];
#pragma unroll
    for (int q = 0; q < NR; ++q) D[q][i] -= C[i] * D[q][i + 1];
    C[i] = -C[i] * C[i + 1];
  }
  // the two reduced rows of this block: (x_{-1}, x_0, x_{M-1}) and (x_0, x_{M-1}, x_M)
  double ra[2], rc[2], rd[NR][2];
  if (M >= 3) {
    const double inv = 1.0 / (1.0 - c0n * A[1]);
    ra[0] = a0n * inv;
    rc[0] = -c0n * C[1] * inv;
#pragma unroll
    for (int q = 0; q < NR; ++q) rd[q][0] = (D0n[q] - c0n * D[q][1]) * inv;
  } else {
    ra[0] = a0n;
    rc[0] = c0n;
#pragma unroll
    for (int q = 0; q < NR; ++q) rd[q][0] = D0n[q];
  }
  ra[1] = A[M - 1];
  rc[1] = C[M - 1];
#pragma unroll
  for (int q = 0; q < NR; ++q) rd[q][1] = D[q][M - 1];
  // parallel cyclic reduction of the 2T reduced rows (normalised: unit diagonal)
  const int T2 = 2 * c.T;
  for (int s = 1; s < T2; s <<= 1) {
    double* pa = c.pcr + (c.pk & 1) * c.pstride;
    double* pc = pa + T2;
    double* pd = pc + T2;
    c.pk++;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = 2 * c.t + h;
      pa[q] = ra[h];
      pc[q] = rc[h];
#pragma unroll
      for (int k = 0; k < NR; ++k) pd[k * T2 + q] = rd[k][h];
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = 2 * c.t + h;
      double am = 0.0, cm = 0.0, ap = 0.0, cp = 0.0, dm[NR], dp[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) dm[k] = dp[k] = 0.0;
      if (q - s >= 0) {
        am = pa[q - s];
        cm = pc[q - s];
#pragma unroll
        for (int k = 0; k < NR; ++k) dm[k] = pd[k * T2 + q - s];
      }
      if (q + s < T2) {
        ap = pa[q + s];
        cp = pc[q + s];
#pragma unroll
        for (int k = 0; k < NR; ++k) dp[k] = pd[k * T2 + q + s];
      }
      const double inv = 1.0 / (1.0 - ra[h] * cm - rc[h] * ap);
      const double a = ra[h], cc = rc[h];
      ra[h] = -a * am * inv;
      rc[h] = -cc * cp * inv;
#pragma unroll
      for (int k = 0; k < NR; ++k) rd[k][h] = (rd[k][h] - a * dm[k] - cc * dp[k]) * inv;
    }
  }
  // back substitution, in place
#pragma unroll
  for (int q = 0; q < NR; ++q) {
#pragma unroll
    for (int i = 1; i < M - 1; ++i) D[q][i] = D[q][i] - A[i] * rd[q][0] - C[i] * rd[q][1];
    D[q][0] = rd[q][0];
    D[q][M - 1] = rd[q][1];
  }
  if (PER) {
    // x = y - z (v.y) / (1 + v.z),  v = (1, 0, .., 0, r/d0)
    double xl[NR], xr[NR], w0[NR], wn[NR];
    exchange<M, NR>(c, D, xl, xr, w0, wn);
    const double v1 = r / d0;
    const double f = (w0[0] + v1 * wn[0]) / (1.0 + w0[NR - 1] + v1 * wn[NR - 1]);
#pragma unroll
    for (int i = 0; i < M; ++i) x[i] = D[0][i] - f * D[NR - 1][i];
  } else {
#pragma unroll
    for (int i = 0; i < M; ++i) x[i] = D[0][i];
  }
}

// Neighbours of a register block of values (one right-hand side).
template <int M>
struct Edges {
  double l, r, w0, wn;
};

template <int M, bool PER>
__device__ __forceinline__ Edges<M> edges(Ctx& c, const double (&x)[M]) {
  double xx[1][M];
#pragma unroll
  for (int i = 0; i < M; ++i) xx[0][i] = x[i];
  double xl[1], xr[1], w0[1], wn[1];
  exchange<M, 1>(c, xx, xl, xr, w0, wn);
  return Edges<M>{xl[0], xr[0], w0[0], wn[0]};
}

// Solve y - tau f^S(y) = rhs for this thread's rows (guess in y on entry).  Linear f^S: one
// solve and one step of iterative refinement with the FP64 residual, so that each stage is the
// exact solution of its linear system to rounding (section II).  Otherwise Newton's method
// with the stopping rule: the largest update is below 1e-15 max(1, max|y|), or below
// 1e-11 max(1, max|y|) and above half the previous one (rounding noise); after maxit iterates
// without stopping, y becomes NaN.  MEM: the right-hand side is read from rhs_mem (rows g0..)
// instead of registers, which keeps the largest blocks (16 rows per thread) out of scratch.
template <int M, bool PER, bool MEM>
__device__ __forceinline__ void stage_solve(Ctx& c, double tau, int maxit, const double (&rhs)[M],
                                            const double* __restrict__ rhs_mem, double (&y)[M]) {
  const double r = tau * c.nu_h2;
  const double b0 = 1.0 + 2.0 * r;
  auto rhs_at = [&](int i) { return MEM ? rhs_mem[c.g0 + i] : rhs[i]; };
  if (c.fs == RIDC_FS_DIFFUSION) {
    tri_solve<M, PER>(c, r, b0, [&](int i, double& b, double& d) { b = b0; d = rhs_at(i); }, y);
    const Edges<M> e = edges<M, PER>(c, y);
    double delta[M];
    tri_solve<M, PER>(
        c, r, b0,
        [&](int i, double& b, double& d) {
          double um, up;
          nbrs<M, PER>(c, y, i, e.l, e.r, e.w0, e.wn, um, up);
          d = rhs_at(i) - (y[i] - tau * c.nu_h2 * (up - 2.0 * y[i] + um));
          b = b0;
        },
        delta);
#pragma unroll
    for (int i = 0; i < M; ++i) y[i] += delta[i];
    return;
  }
  double last = __builtin_inf();
  bool done = false;
  for (int it = 0; it < maxit && !done; ++it) {
    const Edges<M> e = edges<M, PER>(c, y);
    double delta[M];
    tri_solve<M, PER>(
        c, r, b0,
        [&](int i, double& b, double& d) {
          double um, up;
          nbrs<M, PER>(c, y, i, e.l, e.r, e.w0, e.wn, um, up);
          d = rhs_at(i) - (y[i] - tau * fstiff(c, um, y[i], up));
          b = b0 - tau * c.kappa * react_prime(c.fs, y[i]);
        },
        delta);
    double dmax = 0.0, ymax = 0.0;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      y[i] += delta[i];
      if (c.g0 + i < c.n) {
        dmax = fmax(dmax, fabs(delta[i]));
        ymax = fmax(ymax, fabs(y[i]));
      }
    }
    wg_max2(c, dmax, ymax);
    const double scale = fmax(1.0, ymax);
    done = dmax <= 1e-15 * scale || (dmax <= 1e-11 * scale && dmax > 0.5 * last);
    last = dmax;
  }
  if (!done) {
#pragma unroll
    for (int i = 0; i < M; ++i) y[i] = __builtin_nan("");
  }
}

template <int M, bool PER>
__device__ void imex_step(const ImexLvl& L, int64_t sigma, bool init, double* lds) {
  constexpr int NR = PER ? 2 : 1;
  Ctx c;
  c.n = L.n;
  c.T = blockDim.x;
  c.t = threadIdx.x;
  c.g0 = c.t * M;
  c.fe = L.fe;
  c.fs = L.fs;
  c.ce = L.ce;
  c.nu_h2 = L.nu_h2;
  c.kappa = L.kappa;
  c.pstride = 2 * c.T * (2 + NR);
  c.xstride = NR * (2 * c.T + 2);
  c.pcr = lds;
  c.ex = lds + 2 * c.pstride;
  c.red = c.ex + 2 * c.xstride;
  c.pk = c.xk = c.rk = 0;
  const int n = c.n;
  if (init) {
    // f of the initial value (slot 0), read by the next level's window at node t_0
    if (!L.ownF) return;
    double u[M + 2];
    load_halo<M, PER>(c, L.own, u);
    double f[M];
#pragma unroll
    for (int i = 0; i < M; ++i)
      f[i] = fstiff(c, u[i], u[i + 1], u[i + 2]) + fe_eval(c.fe, c.ce, u[i], u[i + 1], u[i + 2]);
    store_rows<M>(c, L.ownF, f);
    return;
  }
  const int64_t m = sigma - L.sigma0 - L.delay;   // this step computes t_m from t_{m-1}
  if (m < 1 || m > L.nt) return;
  const int64_t tn = m - 1;
  const double dt = L.dt;
  const int s = L.s, S = L.S;
  const bool corr = L.prev != nullptr;
  const double* yn_p = L.own + (tn % L.R_own) * (int64_t)n;
  // corrector window: S nodes t_start .. t_{start+S-1}; t_n sits at position rpos
  int64_t start = 0;
  int rpos = 0;
  if (corr) {
    start = tn >= S - 2 ? tn + 2 - S : 0;
    rpos = (int)(tn - start);
  }
  double Y[M], rhs[M];
  for (int i = 0; i < s; ++i) {
    double* ss_p = L.ks + (int64_t)(2 * (s - 1)) * n;     // f^S(eta(t_n + c_i dt)), scratch
    double* sn_p = ss_p + n;                              // f^N(eta(t_n + c_i dt)), scratch
    // rhs = y_n + I_i + dt sum_{l<i} (AS K^S_l + AN K^N_l)
    load_rows<M>(c, yn_p, rhs);
    double guess[M];
    if (corr) {
      const double* w = L.wt + ((int64_t)rpos * s + i) * 2 * S;
      double e[M + 2], q[M];
#pragma unroll
      for (int k = 0; k < M + 2; ++k) e[k] = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) q[k] = 0.0;
      for (int k = 0; k < S; ++k) {
        const int64_t slot = ((start + k) % L.R_prev) * (int64_t)n;
        const double lk = w[k], qk = w[S + k];
        double v[M + 2];
        load_halo<M, PER>(c, L.prev + slot, v);
#pragma unroll
        for (int x = 0; x < M + 2; ++x) e[x] += lk * v[x];
        double fv[M];
        load_rows<M>(c, L.prevF + slot, fv);
#pragma unroll
        for (int x = 0; x < M; ++x) q[x] += qk * fv[x];
      }
      double ssv[M], snv[M];
#pragma unroll
      for (int x = 0; x < M; ++x) {
        ssv[x] = fstiff(c, e[x], e[x + 1], e[x + 2]);
        snv[x] = fe_eval(c.fe, c.ce, e[x], e[x + 1], e[x + 2]);
        rhs[x] = rhs[x] + dt * q[x];
        guess[x] = e[x + 1];
      }
      store_rows<M>(c, ss_p, ssv);
      store_rows<M>(c, sn_p, snv);
    } else {
#pragma unroll
      for (int x = 0; x < M; ++x) guess[x] = rhs[x];
    }
    for (int l = 0; l < i; ++l) {
      const double as = dt * L.AS[i][l], an = dt * L.AN[i][l];
      if (as == 0.0 && an == 0.0) continue;
      double kS[M], kN[M];
      load_rows<M>(c, L.ks + (int64_t)(2 * l) * n, kS);
      load_rows<M>(c, L.ks + (int64_t)(2 * l + 1) * n, kN);
#pragma unroll
      for (int x = 0; x < M; ++x) rhs[x] = rhs[x] + (as * kS[x] + an * kN[x]);
    }
    const double a = L.AS[i][i];
    double kS[M];   // f^S(Y_i), then K^S_i
    Edges<M> e;     // neighbours of this thread's block of Y_i
    if (a == 0.0) {
      // stage 0 (c_0 = 0): Y_0 = y_n
#pragma unroll
      for (int x = 0; x < M; ++x) Y[x] = rhs[x];
      e = edges<M, PER>(c, Y);
#pragma unroll
      for (int x = 0; x < M; ++x) {
        double um, up;
        nbrs<M, PER>(c, Y, x, e.l, e.r, e.w0, e.wn, um, up);
        kS[x] = fstiff(c, um, Y[x], up);
      }
    } else {
      const double tau = dt * a;
      if (corr) {
        double ssv[M];
        load_rows<M>(c, ss_p, ssv);
#pragma unroll
        for (int x = 0; x < M; ++x) rhs[x] = rhs[x] - tau * ssv[x];
      }
#pragma unroll
      for (int x = 0; x < M; ++x) Y[x] = guess[x];
      constexpr bool kMem = M >= 16;
      double* rhs_p = sn_p + n;                             // third scratch vector
      if (kMem) store_rows<M>(c, rhs_p, rhs);
      stage_solve<M, PER, kMem>(c, tau, L.maxit, rhs, rhs_p, Y);
      if (kMem) load_rows<M>(c, rhs_p, rhs);
      e = edges<M, PER>(c, Y);
#pragma unroll
      for (int x = 0; x < M; ++x) kS[x] = (Y[x] - rhs[x]) / tau;
    }
    if (i < s - 1) {
      double kN[M], ssv[M], snv[M];
      if (corr) {
        load_rows<M>(c, ss_p, ssv);
        load_rows<M>(c, sn_p, snv);
      } else {
#pragma unroll
        for (int x = 0; x < M; ++x) ssv[x] = snv[x] = 0.0;
      }
#pragma unroll
      for (int x = 0; x < M; ++x) {
        double um, up;
        nbrs<M, PER>(c, Y, x, e.l, e.r, e.w0, e.wn, um, up);
        kS[x] = kS[x] - ssv[x];
        kN[x] = fe_eval(c.fe, c.ce, um, Y[x], up) - snv[x];
      }
      store_rows<M>(c, L.ks + (int64_t)(2 * i) * n, kS);
      store_rows<M>(c, L.ks + (int64_t)(2 * i + 1) * n, kN);
    } else {
      const int64_t slot = (m % L.R_own) * (int64_t)n;
      store_rows<M>(c, L.own + slot, Y);
      if (L.ownF) {
        double f[M];
#pragma unroll
        for (int x = 0; x < M; ++x) {
          double um, up;
          nbrs<M, PER>(c, Y, x, e.l, e.r, e.w0, e.wn, um, up);
          f[x] = fstiff(c, um, Y[x], up) + fe_eval(c.fe, c.ce, um, Y[x], up);
        }
        store_rows<M>(c, L.ownF + slot, f);
      }
    }
  }
}

template <int M, bool PER>
__global__ __launch_bounds__(kImexMaxThreads) void k_imex1d(const ImexLvl* __restrict__ items,
                                                            int64_t sigma, int init) {
  extern __shared__ double lds[];
  imex_step<M, PER>(items[blockIdx.x], sigma, init != 0, lds);
}

template <int M, bool PER>
hipError_t launch_t(const ImexLvl* items, int count, int threads, int64_t sigma, bool init,
                    hipStream_t stream) {
  const size_t lds = sizeof(double) * lds_doubles(PER ? 2 : 1, threads);
  static size_t allowed = 65536;
  if (lds > allowed) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_imex1d<M, PER>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    allowed = lds;
  }
  hipLaunchKernelGGL((k_imex1d<M, PER>), dim3(count), dim3(threads), lds, stream, items, sigma,
                     init ? 1 : 0);
  return hipGetLastError();
}

template <bool PER>
hipError_t launch_m(int M, const ImexLvl* items, int count, int threads, int64_t sigma,
                    bool init, hipStream_t stream) {
  switch (M) {
    case 2: return launch_t<2, PER>(items, count, threads, sigma, init, stream);
    case 4: return launch_t<4, PER>(items, count, threads, sigma, init, stream);
    case 8: return launch_t<8, PER>(items, count, threads, sigma, init, stream);
    case 16: return launch_t<16, PER>(items, count, threads, sigma, init, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

void imex_shape(int64_t n, int* M, int* threads) {
  // the fewest rows per thread that keep the workgroup within 512 threads (measured: longer
  // per-thread blocks with fewer waves are slower at every size, the elimination chain and the
  // register pressure outweighing the PCR stages saved)
  int m = 2;
  while (m < kImexMaxRows && (n + m - 1) / m > kImexMaxThreads) m *= 2;
  const int64_t t = (n + m - 1) / m;
  *M = m;
  *threads = (int)((t + 63) / 64 * 64);
}

hipError_t launch_imex1d(const ImexLvl* d_items, int count, int M, int threads, bool periodic,
                         int64_t sigma, bool init, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (threads < 64 || threads > kImexMaxThreads || threads % 64) return hipErrorInvalidValue;
  return periodic ? launch_m<true>(M, d_items, count, threads, sigma, init, stream)
                  : launch_m<false>(M, d_items, count, threads, sigma, init, stream);
}

}  // namespace ridc
