// HIP kernels (gfx950) of the rAPDB hot path for convex QCQPs.
//
// Paper: "Restarted Accelerated Primal-Dual Algorithms with Adaptive Stepsizes for Nonlinear
// Conic Constrained Convex Optimization" (arXiv 2605.29291).  Section / equation references:
//   eq. (qcqp-coupling), §2.1 .... Phi, grad_x Phi = Q_0x+q_0+sum lambda_i (Q_ix+q_i)+A'v,
//                                   grad_y Phi = (Ax-b, g(x))
//   eq. (apdb-yx-y), §3.2 ......... APDB-yx updates and its test function E_k
//   Algorithm 1, §3 ............... APDB-xy updates and the test function E_k of
//                                   eq. (backtracking); backtracking loop, tau/gamma rule,
//                                   ergodic averages (both variants)
//   Remark (non-monotone), §3.1 ... c_nm = 1 step rule
//   Algorithm 2, §4.1 ............. fixed-frequency restarts
//   Theorem (metric subregularity), §4.3 ... residual r(x,v,lambda) behind the KKT stop test
//
// All reductions are fixed-order (wave butterflies, then waves in index order), never atomics,
// so every slot's arithmetic is bitwise independent of what else shares a launch.
#include "qcqp_device.h"

namespace qcqp {

// ---------------------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ double clipd(double v, double lo, double hi)
{
    // same comparison form as a plain projection: NaN passes through (and is caught later)
    return v < lo ? lo : (v > hi ? hi : v);
}

// Deterministic block sum of NV doubles; the result is valid in thread 0 only.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV])
{
    __shared__ double sh[NV][STEP_BS / 64];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[k][wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < STEP_BS / 64; ++w) s += sh[k][w];
            v[k] = s;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------------------
// projections onto the dual domain (called by every thread of a block; results visible to the
// whole block on return)

// w (k entries, LDS or global) onto the unit simplex: w <- max(w - theta, 0) with
// sum max(w - theta, 0) = 1.  theta by Michelot's iteration: start from the mean rule over all
// entries, then repeat theta <- (sum_{w_i > theta} w_i - 1) / #{w_i > theta} until the count
// stops changing (theta only grows, so at most k rounds; one fixed-order block sum each).
__device__ void simplex_block(double *w, int k)
{
    const int tid = threadIdx.x;
    __shared__ double s_th[2];
    double v[2] = {0.0, 0.0};
    for (int l = tid; l < k; l += STEP_BS) v[0] += w[l];
    block_sum<2>(v);
    if (tid == 0) s_th[0] = (v[0] - 1.0) / (double)k;
    __syncthreads();
    double theta = s_th[0], cnt = (double)k;
    __syncthreads();
    for (int round = 0; round <= k; ++round) {
        double u[2] = {0.0, 0.0};
        for (int l = tid; l < k; l += STEP_BS) {
            const double a = w[l];
            if (a > theta) {
                u[0] += a;
                u[1] += 1.0;
            }
        }
        block_sum<2>(u);
        if (tid == 0) {
            s_th[0] = (u[0] - 1.0) / u[1];
            s_th[1] = u[1];
        }
        __syncthreads();
        const double nt = s_th[0], nc = s_th[1];
        __syncthreads();
        theta = nt;
        if (nc == cnt) break;
        cnt = nc;
    }
    for (int l = tid; l < k; l += STEP_BS) {
        const double a = w[l];
        w[l] = a > theta ? a - theta : 0.0;
    }
    __syncthreads();
}

// z = (t, u) (k entries) onto the second-order cone Q^k = {||u|| <= t} by one thread: z inside,
// 0 inside the polar cone (||u|| <= -t), otherwise ((t + ||u||) / 2) (1, u / ||u||)
__device__ __forceinline__ void soc_serial(double *z, int k)
{
    const double t = z[0];
    double s = 0.0;
    for (int i = 1; i < k; ++i) s = fma(z[i], z[i], s);
    const double un = sqrt(s);
    if (un <= t) return;
    if (un <= -t) {
        for (int i = 0; i < k; ++i) z[i] = 0.0;
        return;
    }
    const double a = 0.5 * (t + un);
    z[0] = a;
    for (int i = 1; i < k; ++i) z[i] *= a / un;
}

// lambda (m entries, LDS or global) onto K*: R^m_+, the unit simplex, or
// R^{m0}_+ x Q^{k_1} x ... x Q^{k_r} (cones smaller than SOC_BLOCK_DIM one per thread, larger
// ones by the whole block with a fixed-order reduction)
__device__ void project_kstar_block(const Slot *S, double *lam)
{
    const int m = S->m, tid = threadIdx.x;
    if (S->lambda_set == LAMBDA_SIMPLEX) {
        simplex_block(lam, m);
        return;
    }
    const int m0 = S->lambda_set == LAMBDA_CONES ? S->m0 : m;
    for (int l = tid; l < m0; l += STEP_BS)
        if (lam[l] < 0.0) lam[l] = 0.0;
    if (S->lambda_set == LAMBDA_CONES) {
        const int nc = S->n_soc;
        const int32_t *off = S->soc_off, *dim = S->soc_off + nc;
        for (int c = tid; c < nc; c += STEP_BS)
            if (dim[c] < SOC_BLOCK_DIM) soc_serial(lam + off[c], dim[c]);
        __shared__ double s_soc[2];
        for (int bi = 0; bi < S->n_soc_big; ++bi) {
            const int c = S->soc_big[bi];
            double *z = lam + off[c];
            const int k = dim[c];
            double v[1] = {0.0};
            for (int i = 1 + tid; i < k; i += STEP_BS) v[0] = fma(z[i], z[i], v[0]);
            block_sum<1>(v);
            if (tid == 0) {
                const double t = z[0], un = sqrt(v[0]);
                double a = t, f = 1.0;
                if (!(un <= t)) {
                    if (un <= -t) {
                        a = 0.0;
                        f = 0.0;
                    } else {
                        a = 0.5 * (t + un);
                        f = a / un;
                    }
                }
                s_soc[0] = a;
                s_soc[1] = f;
            }
            __syncthreads();
            const double a = s_soc[0], f = s_soc[1];
            if (f != 1.0)
                for (int i = 1 + tid; i < k; i += STEP_BS) z[i] *= f;
            if (tid == 0) z[0] = a;
            __syncthreads();
        }
    }
    __syncthreads();
}

// y = (v, lambda) (ny entries) onto Y-hat = Y ∩ B (problem (R-min-max), §3.2): lambda onto K*
// (R^m_+, a product with second-order cones, or the simplex), then the ball ||y|| <= B
// (eq. (defcalB)) or ||v|| <= B_v, ||lambda|| <= B_lambda (the separable form): scaled back
// when outside, which is the exact projection for a closed convex cone intersected with a ball
// centred at 0.
__device__ void project_dual_block(const Slot *S, double *w)
{
    const int p = S->p, ny = S->ny, tid = threadIdx.x;
    project_kstar_block(S, w + p);
    const double B = S->ball, Bv = S->ball_v, Bl = S->ball_l;
    if (B > 0.0 || Bv > 0.0 || Bl > 0.0) {
        __shared__ double s_f[2];
        double v[2] = {0.0, 0.0};
        for (int l = tid; l < ny; l += STEP_BS) v[l < p ? 0 : 1] += w[l] * w[l];
        block_sum<2>(v);
        if (tid == 0) {
            double fv = 1.0, fl = 1.0;
            if (B > 0.0) {
                const double r = sqrt(v[0] + v[1]);
                if (r > B) fv = fl = B / r;
            }
            if (Bv > 0.0) {
                const double r = sqrt(v[0]);
                if (r > Bv) fv = Bv / r;
            }
            if (Bl > 0.0) {
                const double r = sqrt(v[1]);
                if (r > Bl) fl = Bl / r;
            }
            s_f[0] = fv;
            s_f[1] = fl;
        }
        __syncthreads();
        const double fv = s_f[0], fl = s_f[1];
        if (fv != 1.0 || fl != 1.0)
            for (int l = tid; l < ny; l += STEP_BS) w[l] *= (l < p ? fv : fl);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// step kernel: dual step then primal step for B candidate step sizes (eq. (apdb-yx-y)):
//   sigma = gamma tau, theta = sigma_{k-1}/sigma, s = (1+theta) G^k - theta G^{k-1},
//   y+ = Pi_{Y-hat}(y + sigma s)   (lambda in K* or the simplex, v free, optional ball),
//   x+ = Pi_X(x - tau grad_x Phi(x^k, y+)),  grad from the cached U^k = [Q_i x^k].
// Also the KKT partials of the iterate (x^k, y^k).

template <int B>
__device__ __forceinline__ void step_yx(Slot *__restrict__ S, const int bx)
{
    if (S->variant != VAR_YX || S->status != ST_RUNNING || S->mode != MODE_TRIAL) return;
    if (bx >= S->nblk_step) return;
    const int n = S->n, m = S->m, p = S->p, ny = S->ny;
    extern __shared__ double sm[];
    double *ycur = sm;
    double *ynew = sm + ny;
    __shared__ double s_acc[STEP_WAVES - 1][B + 1][STEP_COLS];
    double tau_b[B], sig_b[B], th_b[B];
    {
        double t = S->tau;
        const double gam = S->gam, sp = S->sig_prev, eta = S->eta;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            tau_b[b] = t;
            sig_b[b] = gam * t;
            th_b[b] = sp / sig_b[b];
            t *= eta;
        }
    }
    // block = STEP_COLS columns; wave w sums matrices i = 1 + w, 1 + w + STEP_WAVES, ... in
    // batches of SB.  The values the primal step needs and the first batch of U_i + q_i are
    // loaded before the dual step and its projection, so their round trip overlaps them.
    constexpr int SB = 8;
    const int lane = threadIdx.x % STEP_COLS, wave = threadIdx.x / STEP_COLS;
    const int j = bx * STEP_COLS + lane;
    const double *U = S->U, *q = S->q;
    double xj = 0.0, lo = 0.0, hi = 0.0, u0 = 0.0;
    if (wave == 0 && j < n) {
        xj = S->x[j];
        lo = S->lb[j];
        hi = S->ub[j];
        u0 = U[j] + q[j];
    }
    double t[SB];
    auto load_batch = [&](int i0) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int ii = i0 + u * STEP_WAVES;
            const size_t o = (size_t)(ii <= m ? ii : 0) * n + j;
            t[u] = (ii <= m && j < n) ? U[o] + q[o] : 0.0;
        }
    };
    load_batch(1 + wave);
    const double *G = S->G, *Gp = S->Gp, *y = S->y;
    for (int l = threadIdx.x; l < ny; l += STEP_BS) {
        const double yl = y[l], gl = G[l], gpl = Gp[l];
        ycur[l] = yl;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const double s = (1.0 + th_b[b]) * gl - th_b[b] * gpl;
            ynew[b * ny + l] = yl + sig_b[b] * s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < B; ++b) project_dual_block(S, ynew + b * ny);
    if (bx == 0) {
        for (int l = threadIdx.x; l < ny; l += STEP_BS) {
#pragma unroll
            for (int b = 0; b < B; ++b) S->yc[b][l] = ynew[b * ny + l];
        }
    }
    double acc[B], kk = 0.0;
#pragma unroll
    for (int b = 0; b < B; ++b) acc[b] = 0.0;
    if (j < n) {
        // ascending i; the next batch is loaded before the current one is summed
        for (int i = 1 + wave; i <= m; i += SB * STEP_WAVES) {
            double c[SB];
#pragma unroll
            for (int u = 0; u < SB; ++u) c[u] = t[u];
            if (i + SB * STEP_WAVES <= m) load_batch(i + SB * STEP_WAVES);
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int ii = i + u * STEP_WAVES;
                if (ii <= m) {
#pragma unroll
                    for (int b = 0; b < B; ++b) acc[b] = fma(ynew[b * ny + p + ii - 1], c[u], acc[b]);
                    kk = fma(ycur[p + ii - 1], c[u], kk);
                }
            }
        }
    }
    if (wave > 0) {
#pragma unroll
        for (int b = 0; b < B; ++b) s_acc[wave - 1][b][lane] = acc[b];
        s_acc[wave - 1][B][lane] = kk;
    }
    __syncthreads();
    double part[NPART];
#pragma unroll
    for (int f = 0; f < NPART; ++f) part[f] = 0.0;
    if (wave == 0 && j < n) {
        // fixed-order combine of the wave partial sums, then the objective and equality terms
#pragma unroll
        for (int w = 1; w < STEP_WAVES; ++w) {
#pragma unroll
            for (int b = 0; b < B; ++b) acc[b] += s_acc[w - 1][b][lane];
            kk += s_acc[w - 1][B][lane];
        }
        double av = 0.0;
        double g[B];
#pragma unroll
        for (int b = 0; b < B; ++b) g[b] = u0 + acc[b];
        for (int l = 0; l < p; ++l) {
            const double a = S->A[(size_t)l * n + j];
#pragma unroll
            for (int b = 0; b < B; ++b) g[b] = fma(ynew[b * ny + l], a, g[b]);
            av = fma(ycur[l], a, av);
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const double xn = clipd(xj - tau_b[b] * g[b], lo, hi);
            S->xc[b][j] = xn;
            const double d = xn - xj;
            part[4 + b] = d * d;
        }
        const double gk = u0 + kk + av;
        const double r = xj - clipd(xj - gk, lo, hi);
        part[0] = r * r;
        part[1] = u0 * u0;
        part[2] = kk * kk;
        part[3] = av * av;
    }
    block_sum<NPART>(part);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int f = 0; f < NPART; ++f) S->part[(size_t)bx * NPART + f] = part[f];
    }
}

template <int B>
__global__ void __launch_bounds__(STEP_BS) k_step(Slot *__restrict__ slots,
                                                  const int *__restrict__ live)
{
    step_yx<B>(slots + (live ? live[blockIdx.y] : (int)blockIdx.y), (int)blockIdx.x);
}

// ---------------------------------------------------------------------------------------
// APDB-xy step kernel (Algorithm 1): the primal step comes first, with momentum on grad_x Phi:
//   sigma = gamma tau, theta = sigma_{k-1}/sigma,
//   s = (1+theta) grad_x Phi(x^k,y^k) - theta grad_x Phi(x^{k-1},y^{k-1}),
//   x+ = Pi_X(x - tau s),
// for B candidate step sizes.  grad_x Phi(x^k,y^k) is recomputed from the cached U^k (it is the
// gradient the KKT residual of the iterate needs anyway) and kept in gxk; gxp holds the one of
// the previous iterate, except at the first iteration of an epoch, where x^{-1} = x^0.

template <int B>
__device__ __forceinline__ void step_xy(Slot *__restrict__ S, const int bx)
{
    if (S->variant != VAR_XY || S->status != ST_RUNNING || S->mode != MODE_TRIAL) return;
    if (bx >= S->nblk_step) return;
    const int n = S->n, m = S->m, p = S->p, ny = S->ny;
    extern __shared__ double sm[];
    double *ycur = sm;
    __shared__ double s_acc[STEP_WAVES - 1][STEP_COLS];
    double tau_b[B], th_b[B];
    {
        double t = S->tau;
        const double gam = S->gam, sp = S->sig_prev, eta = S->eta;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            tau_b[b] = t;
            th_b[b] = sp / (gam * t);
            t *= eta;
        }
    }
    // wave w sums matrices i = 1 + w, 1 + w + STEP_WAVES, ... in batches of SB; the first batch
    // is loaded before the barrier that publishes y
    constexpr int SB = 8;
    const int lane = threadIdx.x % STEP_COLS, wave = threadIdx.x / STEP_COLS;
    const int j = bx * STEP_COLS + lane;
    const double *U = S->U, *q = S->q;
    double t[SB];
    auto load_batch = [&](int i0) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int ii = i0 + u * STEP_WAVES;
            const size_t o = (size_t)(ii <= m ? ii : 0) * n + j;
            t[u] = (ii <= m && j < n) ? U[o] + q[o] : 0.0;
        }
    };
    load_batch(1 + wave);
    // the per-column values of the primal step, loaded now too
    const bool first = S->ke == 0;
    double xj = 0.0, lo = 0.0, hi = 0.0, u0 = 0.0, gxp = 0.0;
    if (wave == 0 && j < n) {
        xj = S->x[j];
        lo = S->lb[j];
        hi = S->ub[j];
        u0 = U[j] + q[j];
        if (!first) gxp = S->gxp[j];
    }
    const double *y = S->y;
    for (int l = threadIdx.x; l < ny; l += STEP_BS) ycur[l] = y[l];
    __syncthreads();
    double kk = 0.0;
    if (j < n) {
        for (int i = 1 + wave; i <= m; i += SB * STEP_WAVES) {
            double c[SB];
#pragma unroll
            for (int u = 0; u < SB; ++u) c[u] = t[u];
            if (i + SB * STEP_WAVES <= m) load_batch(i + SB * STEP_WAVES);
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int ii = i + u * STEP_WAVES;
                if (ii <= m) kk = fma(ycur[p + ii - 1], c[u], kk);
            }
        }
    }
    if (wave > 0) s_acc[wave - 1][lane] = kk;
    __syncthreads();
    double part[NPART];
#pragma unroll
    for (int f = 0; f < NPART; ++f) part[f] = 0.0;
    if (wave == 0 && j < n) {
#pragma unroll
        for (int w = 1; w < STEP_WAVES; ++w) kk += s_acc[w - 1][lane];
        double av = 0.0;
        for (int l = 0; l < p; ++l) av = fma(ycur[l], S->A[(size_t)l * n + j], av);
        const double gk = u0 + kk + av;          // grad_x Phi(x^k, y^k)
        const double gp = first ? gk : gxp;      // grad_x Phi(x^{k-1}, y^{k-1})
        S->gxk[j] = gk;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const double sdir = (1.0 + th_b[b]) * gk - th_b[b] * gp;
            const double xn = clipd(xj - tau_b[b] * sdir, lo, hi);
            S->xc[b][j] = xn;
            const double d = xn - xj;
            part[4 + b] = d * d;
        }
        const double r = xj - clipd(xj - gk, lo, hi);
        part[0] = r * r;
        part[1] = u0 * u0;
        part[2] = kk * kk;
        part[3] = av * av;
    }
    block_sum<NPART>(part);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int f = 0; f < NPART; ++f) S->part[(size_t)bx * NPART + f] = part[f];
    }
}

template <int B>
__global__ void __launch_bounds__(STEP_BS) k_step_xy(Slot *__restrict__ slots,
                                                     const int *__restrict__ live)
{
    step_xy<B>(slots + (live ? live[blockIdx.y] : (int)blockIdx.y), (int)blockIdx.x);
}

// ---------------------------------------------------------------------------------------
// epilogue: one block per (matrix i or equality row l, slot).
//   anchor:      G_i = 1/2 x'U_i + q_i'x + c_i            (g_i, and f for i = 0)
//   direct:      e_i = d'(U+_i - U_i),  G+_i = 1/2 x+'U+_i + q_i'x+ + c_i
//   incremental: e_i = d'W_i,  G+_i - G_i = d'U_i + 1/2 e_i + q_i'd  (Q_i symmetric), and
//                U+_i = U_i + W_i
// G arrays are laid out (Ax-b [p], g [m], f [1]).

template <int B>
__device__ __forceinline__ void epi_rows(Slot *__restrict__ S, const int bx)
{
    if (S->status != ST_RUNNING) return;
    const int n = S->n, m = S->m, p = S->p, ny = S->ny;
    const int row = bx;
    if (row > m + p) return;
    const bool anchor = S->mode == MODE_ANCHOR;
    const bool inc = S->incremental != 0;
    const double *x = S->x;
    const int tid = threadIdx.x;
    // identity part of the objective: row 0 becomes (Q_0 + rho I) x (or (Q_0 + rho I) d), set in
    // place so every later reader of U_0 / W_0 sees it; without Q_0 the pass never writes row 0
    const double rho = row == 0 ? S->q0_shift : 0.0;
    const double keep0 = S->has_q0 ? 1.0 : 0.0;
    if (row <= m) {
        const int gi = row == 0 ? ny : p + row - 1;
        // G_i of the iterate, for the stores at the end, is loaded with the first loads
        const double g_old = (!anchor && tid == 0) ? S->G[gi] : 0.0;
        const double *q = S->q + (size_t)row * n;
        const double ci = S->c[row];
        const size_t off = (size_t)row * n;
        // The column loops below issue the loads of EU strided iterations before using them
        // (each thread still sums its columns in ascending order), with the candidate
        // pointers held in registers: loads no longer wait on stores through other pointers.
        constexpr int EU = 4;
        if (anchor) {
            double *u = S->Uc[0] + off;
            double v[2] = {0.0, 0.0};
            int j = tid;
            for (; j + (EU - 1) * STEP_BS < n; j += EU * STEP_BS) {
                double xj[EU], uj[EU], qj[EU];
#pragma unroll
                for (int k = 0; k < EU; ++k) {
                    xj[k] = x[j + k * STEP_BS];
                    uj[k] = u[j + k * STEP_BS];
                    qj[k] = q[j + k * STEP_BS];
                }
#pragma unroll
                for (int k = 0; k < EU; ++k) {
                    if (rho != 0.0) {
                        uj[k] = fma(rho, xj[k], keep0 * uj[k]);
                        u[j + k * STEP_BS] = uj[k];
                    }
                    v[0] = fma(xj[k], uj[k], v[0]);
                    v[1] = fma(qj[k], xj[k], v[1]);
                }
            }
            for (; j < n; j += STEP_BS) {
                const double xj = x[j];
                double uj = u[j];
                if (rho != 0.0) {
                    uj = fma(rho, xj, keep0 * uj);
                    u[j] = uj;
                }
                v[0] = fma(xj, uj, v[0]);
                v[1] = fma(q[j], xj, v[1]);
            }
            block_sum<2>(v);
            if (tid == 0) S->Gc[0][gi] = 0.5 * v[0] + v[1] + ci;
        } else if (inc) {
            const double *u = S->U + off;
            const double *xcb[B];
            double *wb[B], *ucb[B];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                xcb[b] = S->xc[b];
                wb[b] = S->W[b] + off;
                ucb[b] = S->Uc[b] + off;
            }
            double v[3 * B];
#pragma unroll
            for (int k = 0; k < 3 * B; ++k) v[k] = 0.0;
            auto col = [&](int jj, double xj, double uj, double qj, const double (&xn)[B], const double (&wl)[B]) {
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const double d = xn[b] - xj;
                    double wv = wl[b];
                    if (rho != 0.0) {
                        wv = fma(rho, d, keep0 * wv);
                        wb[b][jj] = wv;
                    }
                    v[3 * b + 0] = fma(d, wv, v[3 * b + 0]);
                    v[3 * b + 1] = fma(d, uj, v[3 * b + 1]);
                    v[3 * b + 2] = fma(qj, d, v[3 * b + 2]);
                    ucb[b][jj] = uj + wv;
                }
            };
            int j = tid;
            for (; j + (EU - 1) * STEP_BS < n; j += EU * STEP_BS) {
                double xj[EU], uj[EU], qj[EU], xn[EU][B], wl[EU][B];
#pragma unroll
                for (int k = 0; k < EU; ++k) {
                    const int jj = j + k * STEP_BS;
                    xj[k] = x[jj];
                    uj[k] = u[jj];
                    qj[k] = q[jj];
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        xn[k][b] = xcb[b][jj];
                        wl[k][b] = wb[b][jj];
                    }
                }
#pragma unroll
                for (int k = 0; k < EU; ++k) col(j + k * STEP_BS, xj[k], uj[k], qj[k], xn[k], wl[k]);
            }
            for (; j < n; j += STEP_BS) {
                double xn[B], wl[B];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    xn[b] = xcb[b][j];
                    wl[b] = wb[b][j];
                }
                col(j, x[j], u[j], q[j], xn, wl);
            }
            block_sum<3 * B>(v);
            if (tid == 0) {
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const double e = v[3 * b];
                    const double dg = v[3 * b + 1] + 0.5 * e + v[3 * b + 2];
                    S->e[b * (m + 1) + row] = e;
                    S->dG[b][gi] = dg;
                    S->Gc[b][gi] = g_old + dg;
                }
            }
        } else {
            const double *u = S->U + off;
            const double *xcb[B];
            double *ucb[B];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                xcb[b] = S->xc[b];
                ucb[b] = S->Uc[b] + off;
            }
            double v[3 * B];
#pragma unroll
            for (int k = 0; k < 3 * B; ++k) v[k] = 0.0;
            auto col = [&](int jj, double xj, double uj, double qj, const double (&xn)[B], const double (&ul)[B]) {
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    double un = ul[b];
                    if (rho != 0.0) {
                        un = fma(rho, xn[b], keep0 * un);
                        ucb[b][jj] = un;
                    }
                    v[3 * b + 0] = fma(xn[b] - xj, un - uj, v[3 * b + 0]);
                    v[3 * b + 1] = fma(xn[b], un, v[3 * b + 1]);
                    v[3 * b + 2] = fma(qj, xn[b], v[3 * b + 2]);
                }
            };
            int j = tid;
            for (; j + (EU - 1) * STEP_BS < n; j += EU * STEP_BS) {
                double xj[EU], uj[EU], qj[EU], xn[EU][B], ul[EU][B];
#pragma unroll
                for (int k = 0; k < EU; ++k) {
                    const int jj = j + k * STEP_BS;
                    xj[k] = x[jj];
                    uj[k] = u[jj];
                    qj[k] = q[jj];
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        xn[k][b] = xcb[b][jj];
                        ul[k][b] = ucb[b][jj];
                    }
                }
#pragma unroll
                for (int k = 0; k < EU; ++k) col(j + k * STEP_BS, xj[k], uj[k], qj[k], xn[k], ul[k]);
            }
            for (; j < n; j += STEP_BS) {
                double xn[B], ul[B];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    xn[b] = xcb[b][j];
                    ul[b] = ucb[b][j];
                }
                col(j, x[j], u[j], q[j], xn, ul);
            }
            block_sum<3 * B>(v);
            if (tid == 0) {
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const double gn = 0.5 * v[3 * b + 1] + v[3 * b + 2] + ci;
                    S->e[b * (m + 1) + row] = v[3 * b];
                    S->Gc[b][gi] = gn;
                    S->dG[b][gi] = gn - g_old;
                }
            }
        }
    } else {
        const int l = row - (m + 1);
        const double *a = S->A + (size_t)l * n;
        const double bl = S->b[l];
        const double g_old = (!anchor && tid == 0) ? S->G[l] : 0.0;
        if (anchor) {
            double v[1] = {0.0};
            for (int j = tid; j < n; j += STEP_BS) v[0] = fma(a[j], x[j], v[0]);
            block_sum<1>(v);
            if (tid == 0) S->Gc[0][l] = v[0] - bl;
        } else {
            double v[B];
#pragma unroll
            for (int b = 0; b < B; ++b) v[b] = 0.0;
            for (int j = tid; j < n; j += STEP_BS) {
                const double aj = a[j];
#pragma unroll
                for (int b = 0; b < B; ++b) v[b] = fma(aj, inc ? S->xc[b][j] - x[j] : S->xc[b][j], v[b]);
            }
            block_sum<B>(v);
            if (tid == 0) {
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    if (inc) {
                        S->dG[b][l] = v[b];
                        S->Gc[b][l] = g_old + v[b];
                    } else {
                        S->Gc[b][l] = v[b] - bl;
                        S->dG[b][l] = (v[b] - bl) - g_old;
                    }
                }
            }
        }
    }
}

template <int B>
__global__ void __launch_bounds__(STEP_BS) k_epi(Slot *__restrict__ slots,
                                                 const int *__restrict__ live)
{
    epi_rows<B>(slots + (live ? live[blockIdx.y] : (int)blockIdx.y), (int)blockIdx.x);
}

// ---------------------------------------------------------------------------------------
// APDB-xy post kernel (Algorithm 1), after the pass and the epilogue have given
// U+ = [Q_i x+] and grad_y Phi(x+) = (Ax+ - b, g(x+)) of every candidate:
//   y+ = Pi_{Y-hat}(y + sigma grad_y Phi(x+))   (as in the yx step kernel),
// and, per column j, the two gradient differences of the test function E_k:
//   a_j = [grad_x Phi(x+,y+) - grad_x Phi(x+,y)]_j = sum_i (l+_i - l_i)(Q_i x+ + q_i)_j + [A'(v+ - v)]_j
//   c_j = [grad_x Phi(x+,y) - grad_x Phi(x,y)]_j  = (Q_0 d)_j + sum_i l_i (Q_i d)_j ,  d = x+ - x,
// with Q_i d = U+_i - U_i (direct pass) or the pass output W_i itself (incremental pass).
// Per block: |a|^2 and |c|^2 of its columns, per candidate.

template <int B>
__device__ __forceinline__ void post_xy(Slot *__restrict__ S, const int bx)
{
    if (S->variant != VAR_XY || S->status != ST_RUNNING || S->mode != MODE_TRIAL) return;
    if (bx >= S->nblk_step) return;
    const int n = S->n, m = S->m, p = S->p, ny = S->ny;
    extern __shared__ double sm[];
    double *ycur = sm;
    double *ynew = sm + ny;
    __shared__ double s_acc[STEP_WAVES - 1][2 * B][STEP_COLS];
    double sig_b[B];
    {
        double t = S->tau;
        const double gam = S->gam, eta = S->eta;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            sig_b[b] = gam * t;
            t *= eta;
        }
    }
    const double *y = S->y;
    for (int l = threadIdx.x; l < ny; l += STEP_BS) {
        const double yl = y[l];
        ycur[l] = yl;
#pragma unroll
        for (int b = 0; b < B; ++b) ynew[b * ny + l] = yl + sig_b[b] * S->Gc[b][l];
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < B; ++b) project_dual_block(S, ynew + b * ny);
    if (bx == 0) {
        for (int l = threadIdx.x; l < ny; l += STEP_BS) {
#pragma unroll
            for (int b = 0; b < B; ++b) S->yc[b][l] = ynew[b * ny + l];
        }
    }
    const int lane = threadIdx.x % STEP_COLS, wave = threadIdx.x / STEP_COLS;
    const int j = bx * STEP_COLS + lane;
    const bool inc = S->incremental != 0;
    const double *U = S->U, *q = S->q;
    double a[B], c[B];
#pragma unroll
    for (int b = 0; b < B; ++b) a[b] = c[b] = 0.0;
    if (j < n) {
        const double *ucb[B], *wb[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            ucb[b] = S->Uc[b];
            wb[b] = inc ? S->W[b] : S->Uc[b];
        }
        auto mat = [&](int i, double u, double qv, const double (&un)[B], const double (&wv)[B]) {
            const double lam = ycur[p + i - 1];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const double du = inc ? wv[b] : un[b] - u;
                a[b] = fma(ynew[b * ny + p + i - 1] - lam, un[b] + qv, a[b]);
                c[b] = fma(lam, du, c[b]);
            }
        };
        int i = 1 + wave;
        // 4 matrices per step, loads first; the sums keep the ascending order of i
        for (; i + 3 * STEP_WAVES <= m; i += 4 * STEP_WAVES) {
            double u[4], qv[4], un[4][B], wv[4][B];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const size_t o = (size_t)(i + k * STEP_WAVES) * n + j;
                u[k] = U[o];
                qv[k] = q[o];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    un[k][b] = ucb[b][o];
                    wv[k][b] = wb[b][o];
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) mat(i + k * STEP_WAVES, u[k], qv[k], un[k], wv[k]);
        }
        for (; i <= m; i += STEP_WAVES) {
            const size_t o = (size_t)i * n + j;
            double un[B], wv[B];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                un[b] = ucb[b][o];
                wv[b] = wb[b][o];
            }
            mat(i, U[o], q[o], un, wv);
        }
    }
    if (wave > 0) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            s_acc[wave - 1][2 * b][lane] = a[b];
            s_acc[wave - 1][2 * b + 1][lane] = c[b];
        }
    }
    __syncthreads();
    double part[2 * B];
#pragma unroll
    for (int f = 0; f < 2 * B; ++f) part[f] = 0.0;
    if (wave == 0 && j < n) {
#pragma unroll
        for (int w = 1; w < STEP_WAVES; ++w) {
#pragma unroll
            for (int b = 0; b < B; ++b) {
                a[b] += s_acc[w - 1][2 * b][lane];
                c[b] += s_acc[w - 1][2 * b + 1][lane];
            }
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const double c0 = inc ? S->W[b][j] : S->Uc[b][j] - U[j];
            const double cb = c0 + c[b];
            double ab = a[b];
            for (int l = 0; l < p; ++l)
                ab = fma(ynew[b * ny + l] - ycur[l], S->A[(size_t)l * n + j], ab);
            part[2 * b] = ab * ab;
            part[2 * b + 1] = cb * cb;
        }
    }
    block_sum<2 * B>(part);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int f = 0; f < 2 * B; ++f) S->part2[(size_t)bx * NPART2 + f] = part[f];
    }
}

template <int B>
__global__ void __launch_bounds__(STEP_BS) k_post_xy(Slot *__restrict__ slots,
                                                     const int *__restrict__ live)
{
    post_xy<B>(slots + (live ? live[blockIdx.y] : (int)blockIdx.y), (int)blockIdx.x);
}

// ---------------------------------------------------------------------------------------
// control kernel (one block per slot, FP64)

__device__ __forceinline__ void swap_ptr(double *&a, double *&b)
{
    double *t = a;
    a = b;
    b = t;
}

// New epoch of Algorithm 2: rs = 1 restarts at the last iterate, rs = 2 at the ergodic
// average; the routine's first line resets tau, gamma, the momentum (x^{-1} = x^0) and the
// averages.  A re-anchor (exact direct pass at the restart point) follows when the point moved
// or when trial products are formed incrementally.  Called by all threads of one block.
__device__ void restart_epoch(Slot *S, int rs)
{
    const int n = S->n, ny = S->ny, tid = threadIdx.x;
    if (rs == 2) {
        const double invT = 1.0 / S->T;
        double *x = S->x, *y = S->y;
        const double *cx = S->cx, *cy = S->cy;
        for (int j = tid; j < n; j += STEP_BS) x[j] = cx[j] * invT;
        for (int l = tid; l < ny; l += STEP_BS) y[l] = cy[l] * invT;
    }
    __syncthreads();
    double *cx = S->cx, *cy = S->cy;
    for (int j = tid; j < n; j += STEP_BS) cx[j] = 0.0;
    for (int l = tid; l < ny; l += STEP_BS) cy[l] = 0.0;
    const bool anchor = (rs == 2) || S->incremental;
    if (!anchor) {
        const double *G = S->G;
        double *Gp = S->Gp;
        for (int l = tid; l <= ny; l += STEP_BS) Gp[l] = G[l];
    }
    __syncthreads();
    if (tid == 0) {
        S->tau = S->tau_bar;
        S->tau_prev = S->tau_bar;
        S->sig_prev = S->gamma0 * S->tau_bar;
        S->gam = S->gamma0;
        // alpha_0, beta_0 from tau_{-1}, sigma_{-1}
        S->alpha_k = S->c_alpha / (S->variant == VAR_XY ? S->tau_prev : S->sig_prev);
        S->beta_k = S->gamma0 * S->c_beta / S->sig_prev;
        S->T = 0.0;
        S->ke = 0;
        S->restarts += 1;
        if (anchor) {
            S->mode = MODE_ANCHOR;
            S->anchor_keep_gp = 0;
        }
    }
}

// The slot fields the control phase's thread 0 reads, loaded in one batch (see ctrl_slot).
struct CtlState {
    double cnorm, bnorm, f_star, tol, tau, gam, sig_prev, eta, sig0, c_alpha, gamma0, c_beta, delta;
    double alpha_k, beta_k, T, mu, tau_prev, fval;
    int64_t k, ke, max_iter, passes, trials, iter_trials, restart_every, ada_first, ada_every;
    int32_t stop_rule, m0, n_soc, fresh, c_nm, restart, restart_from_avg, variant, dtype, incremental;
    double *x, *U, *y, *G, *Gp, *gxp, *gxk;
    double *xc[MAXB], *Uc[MAXB], *yc[MAXB], *Gc[MAXB];
    double fc[MAXB];   // f at each candidate: Gc[b][ny]

    template <int B>
    __device__ __forceinline__ void load(const Slot *__restrict__ S)
    {
        cnorm = S->cnorm; bnorm = S->bnorm; f_star = S->f_star; tol = S->tol;
        tau = S->tau; gam = S->gam; sig_prev = S->sig_prev; eta = S->eta; sig0 = S->sig0;
        c_alpha = S->c_alpha; gamma0 = S->gamma0; c_beta = S->c_beta; delta = S->delta;
        alpha_k = S->alpha_k; beta_k = S->beta_k; T = S->T; mu = S->mu; tau_prev = S->tau_prev;
        k = S->k; ke = S->ke; max_iter = S->max_iter; passes = S->passes; trials = S->trials;
        iter_trials = S->iter_trials; restart_every = S->restart_every; ada_first = S->ada_first;
        ada_every = S->ada_every;
        stop_rule = S->stop_rule; m0 = S->m0; n_soc = S->n_soc; fresh = S->fresh; c_nm = S->c_nm;
        restart = S->restart; restart_from_avg = S->restart_from_avg; variant = S->variant;
        dtype = S->dtype; incremental = S->incremental;
        x = S->x; U = S->U; y = S->y; G = S->G; Gp = S->Gp; gxp = S->gxp; gxk = S->gxk;
        const int ny = S->ny;
        fval = G[ny];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            xc[b] = S->xc[b];
            Uc[b] = S->Uc[b];
            yc[b] = S->yc[b];
            Gc[b] = S->Gc[b];
            fc[b] = Gc[b][ny];
        }
    }
};

template <int B>
__device__ __forceinline__ void ctrl_slot(Slot *__restrict__ S)
{
    const int status = S->status;
    const int mode = S->mode;
    __syncthreads();
    if (status != ST_RUNNING) return;
    const int n = S->n, m = S->m, p = S->p, ny = S->ny;
    const int tid = threadIdx.x;
    __shared__ int s_dec;       // accepted candidate, -1 none, -2 stop
    __shared__ int s_restart;   // 0 none, 1 restart at last iterate, 2 from the average
    __shared__ double s_t;

    if (mode == MODE_ANCHOR) {
        // install [Q_i x] and G(x) of the anchor point; x^{-1} = x^0 (epoch start)
        if (tid == 0) {
            swap_ptr(S->U, S->Uc[0]);
            swap_ptr(S->G, S->Gc[0]);
        }
        __syncthreads();
        const double *G = S->G;
        double *Gp = S->Gp;
        if (!S->anchor_keep_gp)
            for (int l = tid; l <= ny; l += STEP_BS) Gp[l] = G[l];
        __syncthreads();
        if (tid == 0) {
            S->f = G[ny];
            S->mode = MODE_TRIAL;
            S->passes += 1;
            S->fresh = 1;
            S->anchor_keep_gp = 0;
        }
        return;
    }

    // Everything thread 0 reads for the decision and the bookkeeping is loaded now, before the
    // reductions: none of it is written before thread 0's own stores below, and the loads then
    // overlap the reductions instead of following them as two more round trips.  Every thread
    // takes the candidates' x and y pointers for the ergodic sums.
    const double *xcp[B], *ycp[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        xcp[b] = S->xc[b];
        ycp[b] = S->yc[b];
    }
    double *const cxp = S->cx, *const cyp = S->cy;
    CtlState cs;
    if (tid == 0) cs.load<B>(S);

    // ---- 1+2. one fixed-order block reduction of everything the decision needs:
    //   step partials (KKT pieces of the iterate, ||d_b||^2), ||min(lambda,-g)||^2,
    //   ||([g]+, Ax-b)||^2, and per candidate 1/2 d'Q(lambda+)d terms, ||dG||^2, ||dy||^2 ----
    // lambda on the simplex or on cones: the lambda-part of the KKT residual is the natural
    // residual lambda - Pi_K*(lambda + g(x)), and with cones the infeasibility is
    // dist(g, -K) = ||Pi_K*(g)||; the projected points are staged in LDS (wsm, wsm + m)
    extern __shared__ double wsm[];
    const bool simplex = S->lambda_set == LAMBDA_SIMPLEX;
    const bool cones = S->lambda_set == LAMBDA_CONES;
    if (simplex || cones) {
        for (int l = tid; l < m; l += STEP_BS) {
            wsm[l] = S->y[p + l] + S->G[p + l];
            if (cones) wsm[m + l] = S->G[p + l];
        }
        __syncthreads();
        project_kstar_block(S, wsm);
        if (cones) project_kstar_block(S, wsm + m);
    }
    constexpr int NR = NPART + 3 + 3 * B;   // ..., per-candidate triples, summed violation
    double r[NR];
#pragma unroll
    for (int f = 0; f < NR; ++f) r[f] = 0.0;
    double mx = 0.0;
    {
        const double *part = S->part;
        const int nblk = S->nblk_step;
        for (int blk = tid; blk < nblk; blk += STEP_BS) {
#pragma unroll
            for (int f = 0; f < NPART; ++f) r[f] += part[(size_t)blk * NPART + f];
        }
        const double *G = S->G, *y = S->y;
        for (int l = tid; l < ny; l += STEP_BS) {
            const double gl = G[l];
            if (l < p) {
                r[NPART + 1] += gl * gl;
                r[NR - 1] += fabs(gl);
                mx = fmax(mx, fabs(gl));
            } else if (simplex) {
                const double d = y[l] - wsm[l - p];
                r[NPART] += d * d;
            } else if (cones) {
                const double d = y[l] - wsm[l - p];
                const double gp = wsm[m + l - p];
                r[NPART] += d * d;
                r[NPART + 1] += gp * gp;
                if (l - p < S->m0) {
                    r[NR - 1] += gp;
                    mx = fmax(mx, gp);
                }
            } else {
                const double lam = y[l];
                const double mn = lam < -gl ? lam : -gl;
                r[NPART] += mn * mn;
                if (gl > 0.0) {
                    r[NPART + 1] += gl * gl;
                    r[NR - 1] += gl;
                    mx = fmax(mx, gl);
                }
            }
        }
        if (cones) {
            // one violation dist(g_c, -Q) = ||Pi_Q(g_c)|| per cone
            const int nc = S->n_soc;
            const int32_t *off = S->soc_off, *dim = S->soc_off + nc;
            for (int c = tid; c < nc; c += STEP_BS) {
                double sq = 0.0;
                const double *z = wsm + m + off[c];
                for (int i = 0; i < dim[c]; ++i) sq = fma(z[i], z[i], sq);
                const double v = sqrt(sq);
                r[NR - 1] += v;
                mx = fmax(mx, v);
            }
        }
        const bool xy = S->variant == VAR_XY;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const double *yc = S->yc[b];
            double *t = r + NPART + 2 + 3 * b;
            if (xy) {
                // xy: |a_b|^2 and |c_b|^2 from the post kernel's block partials
                const double *p2 = S->part2;
                for (int blk = tid; blk < nblk; blk += STEP_BS) {
                    t[0] += p2[(size_t)blk * NPART2 + 2 * b];
                    t[1] += p2[(size_t)blk * NPART2 + 2 * b + 1];
                }
            } else {
                // yx: sum_i w_i d'(Q_i d) with w = (1, lambda+), and |dG|^2
                const double *e = S->e + b * (m + 1);
                const double *dg = S->dG[b];
                for (int i = tid; i <= m; i += STEP_BS) {
                    const double wgt = (i == 0) ? 1.0 : yc[p + i - 1];
                    t[0] = fma(wgt, e[i], t[0]);
                }
                for (int l = tid; l < ny; l += STEP_BS) t[1] = fma(dg[l], dg[l], t[1]);
            }
            for (int l = tid; l < ny; l += STEP_BS) {
                const double dy = yc[l] - y[l];
                t[2] = fma(dy, dy, t[2]);
            }
        }
    }
    // the block maximum of the violations: per-wave shuffles, then one value per wave
    __shared__ double s_mx[STEP_BS / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((tid & 63) == 0) s_mx[tid >> 6] = mx;
    block_sum<NR>(r);              // includes the barrier that publishes s_mx
    double tot[NPART], kv[3], tq[3 * B];
#pragma unroll
    for (int f = 0; f < NPART; ++f) tot[f] = r[f];
    kv[0] = r[NPART];
    kv[1] = r[NPART + 1];
    kv[2] = 0.0;
#pragma unroll
    for (int k2 = 0; k2 < 3 * B; ++k2) tq[k2] = r[NPART + 2 + k2];
    if (tid == 0) {
        double mm = 0.0;
        for (int w = 0; w < STEP_BS / 64; ++w) mm = fmax(mm, s_mx[w]);
        kv[2] = mm;
    }

    if (tid == 0) {
        const auto cnorm = cs.cnorm, bnorm = cs.bnorm, f_star = cs.f_star, tol = cs.tol;
        const auto stop_rule = cs.stop_rule, m0 = cs.m0, n_soc = cs.n_soc, fresh = cs.fresh;
        const auto kk = cs.k, ke = cs.ke, max_iter = cs.max_iter, passes = cs.passes;
        const auto trials = cs.trials, iter_trials = cs.iter_trials;
        const auto tau = cs.tau, gam = cs.gam, sp = cs.sig_prev, eta = cs.eta, sig0 = cs.sig0;
        const auto c_alpha = cs.c_alpha, gamma0 = cs.gamma0, c_beta = cs.c_beta, delta = cs.delta;
        const auto alpha_k = cs.alpha_k, beta_k = cs.beta_k;
        const bool xy = cs.variant == VAR_XY;
        const double fval = cs.fval;
        const double rel_dual = sqrt(tot[0]) / (1.0 + sqrt(tot[1]) + sqrt(tot[2]) + sqrt(tot[3]));
        const double rel_comp = sqrt(kv[0]) / (1.0 + cnorm);
        const double rel_pri = sqrt(kv[1]) / (1.0 + cnorm + bnorm);
        double rk = fmax(rel_dual, fmax(rel_pri, rel_comp));
        if (isnan(rel_dual) || isnan(rel_pri) || isnan(rel_comp)) rk = NAN;
        S->kkt[0] = rk;
        S->kkt[1] = rel_dual;
        S->kkt[2] = rel_pri;
        S->kkt[3] = rel_comp;
        S->maxviol = kv[2];
        // stop rule: the relative KKT residual, or the criterion of the experiments of §5.1
        // (relative suboptimality against f_star and the mean constraint violation)
        double crit = rk;
        if (stop_rule == 1) {
            const int cnt = p + (simplex ? 0 : (cones ? m0 + n_soc : m));
            const double fs = f_star;
            const double sub = fabs(fval - fs) / (1.0 + fabs(fs));
            const double mv = cnt > 0 ? r[NR - 1] / (double)cnt : 0.0;
            crit = sub > mv ? sub : mv;
            if (isnan(sub) || isnan(mv)) crit = NAN;
        }
        S->crit = crit;
        int dec = -1;
        S->passes = passes + 1;         // this group's pass was streamed, whatever follows
        if (isnan(rk) || isnan(crit)) {
            S->status = ST_NUMERICAL;
            dec = -2;
        } else if (crit <= tol) {
            if (fresh) {
                S->status = ST_CONVERGED;
            } else {
                // the cached U carries FP32 / incremental rounding: confirm the stop test on
                // exact FP64 values first (refresh anchor, the epoch continues)
                S->mode = MODE_ANCHOR;
                S->anchor_keep_gp = 1;
            }
            dec = -2;
        } else if (kk >= max_iter) {
            S->status = ST_MAX_ITER;
            dec = -2;
        }
        if (dec == -1) {
            double t = tau;
            for (int b = 0; b < B; ++b) {
                const double sig = gam * t;
                const double th = sp / sig;
                const double dd = tot[4 + b], dy2 = tq[3 * b + 2];
                const double Dp = 0.5 * dd, Dd = 0.5 * dy2;
                double E;
                if (xy) {
                    // Algorithm 1: alpha_{k+1} = c_a / tau_k, beta_{k+1} = gamma_0 c_b / sigma_k;
                    // E_k of eq. (backtracking) with the two gradient differences of k_post_xy
                    const double alpha_next = c_alpha / t;
                    const double beta_next = gamma0 * c_beta / sig;
                    E = tq[3 * b] / (2.0 * alpha_next) - Dd / sig + tq[3 * b + 1] / (2.0 * beta_next) -
                        (1.0 / t - th * (alpha_k + beta_k)) * Dp;
                } else {
                    const double alpha_next = c_alpha / sig;        // alpha_{k+1} = c_a / sigma_k
                    const double quad = 0.5 * tq[3 * b];              // 1/2 d'Q(lambda+)d
                    E = quad - Dp / t + tq[3 * b + 1] / (2.0 * alpha_next) -
                        (1.0 / sig - th * alpha_k) * Dd;
                }
                const double rhs = -(delta / t) * Dp - (delta / sig) * Dd;
                if (E <= rhs) {
                    dec = b;
                    break;
                }
                if (isnan(E) || isnan(rhs)) {
                    dec = -3;
                    break;
                }
                t *= eta;
            }
            if (dec == -3) {
                S->status = ST_NUMERICAL;
                dec = -2;
            } else if (dec == -1) {
                // all candidates rejected: tau <- eta^B tau, next group retries
                S->tau = t;
                S->trials = trials + B;
                S->iter_trials = iter_trials + B;
                if (iter_trials + B > 400 || !(t > 1e-300)) {
                    S->status = ST_NUMERICAL;
                    dec = -2;
                }
            }
        }
        s_dec = dec;
        if (dec >= 0) {
            double t = tau;
            for (int b = 0; b < dec; ++b) t *= eta;
            const double sig = gam * t;
            const double s0 = ke == 0 ? sig : sig0;
            if (ke == 0) S->sig0 = sig;
            s_t = sig / s0;                                          // t_k = sigma_k / sigma_0
        }
    }
    __syncthreads();
    const int dec = s_dec;
    if (dec < 0) return;

    // ---- 3. accepted candidate `dec`: ergodic sums (Algorithm 1) ----
    {
        const double tk = s_t;
        const double *xn = xcp[0], *yn = ycp[0];
#pragma unroll
        for (int b = 1; b < B; ++b) {
            if (dec == b) {
                xn = xcp[b];
                yn = ycp[b];
            }
        }
        for (int j = tid; j < n; j += STEP_BS) cxp[j] = fma(tk, xn[j], cxp[j]);
        for (int l = tid; l < ny; l += STEP_BS) cyp[l] = fma(tk, yn[l], cyp[l]);
    }
    __syncthreads();
    if (tid == 0) {
        const auto tau = cs.tau, eta = cs.eta, gam = cs.gam, T = cs.T, mu = cs.mu;
        const auto c_nm = cs.c_nm;
        const auto tau_prev = cs.tau_prev;
        const auto c_alpha = cs.c_alpha, gamma0 = cs.gamma0, c_beta = cs.c_beta;
        const auto trials = cs.trials, kk = cs.k, ke = cs.ke;
        const auto restart = cs.restart;
        const auto restart_every = cs.restart_every;
        const auto ada_first = cs.ada_first, ada_every = cs.ada_every;
        const auto restart_from_avg = cs.restart_from_avg;
        const bool xy = cs.variant == VAR_XY;
        const bool exact = cs.dtype == DT_F64 && !cs.incremental;
        double *xn = cs.xc[0], *Un = cs.Uc[0], *yn = cs.yc[0], *Gn = cs.Gc[0];
        double fn = cs.fc[0];
#pragma unroll
        for (int b = 1; b < B; ++b) {
            if (dec == b) {
                xn = cs.xc[b];
                Un = cs.Uc[b];
                yn = cs.yc[b];
                Gn = cs.Gc[b];
                fn = cs.fc[b];
            }
        }
        double *const x = cs.x, *const U = cs.U, *const y = cs.y;
        double *const Gp = cs.Gp, *const G = cs.G;
        double *const gxp = cs.gxp, *const gxk = cs.gxk;
        double t = tau;
        for (int b = 0; b < dec; ++b) t *= eta;
        const double sig = gam * t;
        const double Tn = T + s_t;
        S->T = Tn;
        S->trials = trials + dec + 1;
        S->iter_trials = 0;
        // step-size rule, Algorithm 1 (non-monotone form with c_nm = 1)
        const double gam_next = gam * (1.0 + mu * t);
        const double tau_next = t * sqrt(gam / gam_next * (1.0 + c_nm * t / tau_prev));
        // shift the state: (x, U, y) <- candidate, G^{k-1} <- G^k, G^k <- candidate
        S->x = xn;
        S->xc[dec] = x;
        S->U = Un;
        S->Uc[dec] = U;
        S->y = yn;
        S->yc[dec] = y;
        S->Gp = G;
        S->G = Gn;
        S->Gc[dec] = Gp;
        S->f = fn;
        S->fresh = exact ? 1 : 0;
        if (xy) {
            // grad_x Phi(x^k, y^k) becomes the previous iterate's; the next step kernel
            // recomputes the new one from U
            S->gxp = gxk;
            S->gxk = gxp;
            S->alpha_k = c_alpha / t;
            S->beta_k = gamma0 * c_beta / sig;
        } else {
            S->alpha_k = c_alpha / sig;
        }
        S->sig_prev = sig;
        S->tau_prev = t;
        S->tau = tau_next;
        S->gam = gam_next;
        const auto k1 = kk + 1, ke1 = ke + 1;
        S->k = k1;
        S->ke = ke1;
        int rs = 0;
        if (restart == 1 && ke1 >= restart_every) rs = 1;
        if (restart == 2 && (k1 == ada_first || (k1 > ada_first && (k1 % ada_every) == 0)))
            S->status = ST_GAP_PENDING;
        if (rs && restart_from_avg && Tn > 0.0) rs = 2;
        s_restart = rs;
    }
    __syncthreads();
    const int rs = s_restart;
    if (rs == 0) return;

    // ---- 4. restart (Algorithm 2) ----
    restart_epoch(S, rs);
}

template <int B>
__global__ void __launch_bounds__(STEP_BS) k_ctrl(Slot *__restrict__ slots,
                                                  const int *__restrict__ live)
{
    ctrl_slot<B>(slots + (live ? live[blockIdx.x] : (int)blockIdx.x));
}

// ---------------------------------------------------------------------------------------
// start: clip x^0 into X, project y^0 onto Y-hat, clear the averages; the first group is an
// anchor pass.

__global__ void __launch_bounds__(STEP_BS) k_start(Slot *__restrict__ S)
{
    const int n = S->n, ny = S->ny;
    for (int j = threadIdx.x; j < n; j += STEP_BS) {
        S->x[j] = clipd(S->x[j], S->lb[j], S->ub[j]);
        S->cx[j] = 0.0;
    }
    for (int l = threadIdx.x; l < ny; l += STEP_BS) S->cy[l] = 0.0;
    __syncthreads();
    project_dual_block(S, S->y);
}

// ---------------------------------------------------------------------------------------
// standalone evaluations: gradient and KKT residual at an arbitrary (x, y), given U = [Q_i x]

__global__ void __launch_bounds__(STEP_BS) k_grad(const Slot *__restrict__ S,
                                                  const double *__restrict__ U,
                                                  const double *__restrict__ y,
                                                  double *__restrict__ out)
{
    const int n = S->n, m = S->m, p = S->p;
    const int j = blockIdx.x * STEP_BS + threadIdx.x;
    if (j >= n) return;
    double g = U[j] + S->q[j];
    for (int i = 1; i <= m; ++i)
        g = fma(y[p + i - 1], U[(size_t)i * n + j] + S->q[(size_t)i * n + j], g);
    for (int l = 0; l < p; ++l) g = fma(y[l], S->A[(size_t)l * n + j], g);
    out[j] = g;
}

__global__ void __launch_bounds__(STEP_BS) k_kkt_part(const Slot *__restrict__ S,
                                                      const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      const double *__restrict__ U,
                                                      double *__restrict__ part)
{
    const int n = S->n, m = S->m, p = S->p;
    const int j = blockIdx.x * STEP_BS + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (j < n) {
        const double u0 = U[j] + S->q[j];
        double kk = 0.0, av = 0.0;
        for (int i = 1; i <= m; ++i)
            kk = fma(y[p + i - 1], U[(size_t)i * n + j] + S->q[(size_t)i * n + j], kk);
        for (int l = 0; l < p; ++l) av = fma(y[l], S->A[(size_t)l * n + j], av);
        const double gk = u0 + kk + av;
        const double r = x[j] - clipd(x[j] - gk, S->lb[j], S->ub[j]);
        v[0] = r * r;
        v[1] = u0 * u0;
        v[2] = kk * kk;
        v[3] = av * av;
    }
    block_sum<4>(v);
    if (threadIdx.x == 0) {
        for (int f = 0; f < 4; ++f) part[(size_t)blockIdx.x * 4 + f] = v[f];
    }
}

__global__ void __launch_bounds__(STEP_BS) k_kkt_fin(const Slot *__restrict__ S, int nblk,
                                                     const double *__restrict__ y,
                                                     const double *__restrict__ G,
                                                     const double *__restrict__ part,
                                                     double *__restrict__ out6)
{
    const int ny = S->ny, p = S->p, m = S->m;
    const int tid = threadIdx.x;
    double tot[4] = {0.0, 0.0, 0.0, 0.0};
    for (int blk = tid; blk < nblk; blk += STEP_BS)
        for (int f = 0; f < 4; ++f) tot[f] += part[(size_t)blk * 4 + f];
    block_sum<4>(tot);
    extern __shared__ double wsm[];
    const bool simplex = S->lambda_set == LAMBDA_SIMPLEX;
    const bool cones = S->lambda_set == LAMBDA_CONES;
    if (simplex || cones) {
        for (int l = tid; l < m; l += STEP_BS) {
            wsm[l] = y[p + l] + G[p + l];
            if (cones) wsm[m + l] = G[p + l];
        }
        __syncthreads();
        project_kstar_block(S, wsm);
        if (cones) project_kstar_block(S, wsm + m);
    }
    double kv[2] = {0.0, 0.0};
    double mx = 0.0;
    if (cones) {
        const int nc = S->n_soc;
        const int32_t *off = S->soc_off, *dim = S->soc_off + nc;
        for (int c = tid; c < nc; c += STEP_BS) {
            double sq = 0.0;
            const double *z = wsm + m + off[c];
            for (int i = 0; i < dim[c]; ++i) sq = fma(z[i], z[i], sq);
            mx = fmax(mx, sqrt(sq));
        }
    }
    for (int l = tid; l < ny; l += STEP_BS) {
        const double gl = G[l];
        if (l < p) {
            kv[1] += gl * gl;
            mx = fmax(mx, fabs(gl));
        } else if (simplex) {
            const double d = y[l] - wsm[l - p];
            kv[0] += d * d;
        } else if (cones) {
            const double d = y[l] - wsm[l - p];
            const double gp = wsm[m + l - p];
            kv[0] += d * d;
            kv[1] += gp * gp;
            if (l - p < S->m0) mx = fmax(mx, gp);
        } else {
            const double lam = y[l];
            const double mn = lam < -gl ? lam : -gl;
            kv[0] += mn * mn;
            if (gl > 0.0) {
                kv[1] += gl * gl;
                mx = fmax(mx, gl);
            }
        }
    }
    __shared__ double s_mx[STEP_BS];
    s_mx[tid] = mx;
    block_sum<2>(kv);
    if (tid == 0) {
        double mm = 0.0;
        for (int t = 0; t < STEP_BS; ++t) mm = fmax(mm, s_mx[t]);
        const double rel_dual = sqrt(tot[0]) / (1.0 + sqrt(tot[1]) + sqrt(tot[2]) + sqrt(tot[3]));
        const double rel_comp = sqrt(kv[0]) / (1.0 + S->cnorm);
        const double rel_pri = sqrt(kv[1]) / (1.0 + S->cnorm + S->bnorm);
        double rk = fmax(rel_dual, fmax(rel_pri, rel_comp));
        if (isnan(rel_dual) || isnan(rel_pri) || isnan(rel_comp)) rk = NAN;
        out6[0] = rk;
        out6[1] = rel_dual;
        out6[2] = rel_pri;
        out6[3] = rel_comp;
        out6[4] = G[ny];
        out6[5] = mm;
    }
}

// ---------------------------------------------------------------------------------------
// storage conversion, once at creation: src (dtype, ld_src) -> dst (dtype, ld_dst), the
// padding columns n..ld_dst-1 set to zero.  FP64 -> 16/32 bit rounds to nearest even in one
// step: a round-to-odd FP32 intermediate (truncate, then set the sticky bit when inexact)
// followed by the hardware's nearest-even FP32 -> 16-bit conversion.

__device__ __forceinline__ double load_any(const void *p, int dt, size_t i)
{
    switch (dt) {
    case DT_F64: return reinterpret_cast<const double *>(p)[i];
    case DT_F32: return (double)reinterpret_cast<const float *>(p)[i];
    case DT_BF16: return (double)__uint_as_float((uint32_t)reinterpret_cast<const uint16_t *>(p)[i] << 16);
    default: return (double)(float)__builtin_bit_cast(_Float16, reinterpret_cast<const uint16_t *>(p)[i]);
    }
}

__device__ __forceinline__ float round_to_odd_f32(double v)
{
    float f = __double2float_rz(v);
    if ((double)f != v && !isnan(v)) {
        uint32_t bits = __float_as_uint(f) | 1u;
        f = __uint_as_float(bits);
    }
    return f;
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // NaN stays NaN
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

__global__ void k_convert(const void *__restrict__ src, int sdt, int64_t lds,
                          void *__restrict__ dst, int ddt, int64_t ldd, int64_t rows, int64_t n)
{
    const int64_t total = rows * ldd;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = idx / ldd, j = idx - r * ldd;
        double v = 0.0;
        if (j < n) v = load_any(src, sdt, (size_t)(r * lds + j));
        switch (ddt) {
        case DT_F64: reinterpret_cast<double *>(dst)[idx] = v; break;
        case DT_F32: reinterpret_cast<float *>(dst)[idx] = (float)v; break;
        case DT_BF16:
            if (sdt == DT_BF16)
                reinterpret_cast<uint16_t *>(dst)[idx] =
                    j < n ? reinterpret_cast<const uint16_t *>(src)[r * lds + j] : (uint16_t)0;
            else
                reinterpret_cast<uint16_t *>(dst)[idx] = f32_to_bf16_rne(round_to_odd_f32(v));
            break;
        default: {
            _Float16 h;
            if (sdt == DT_F16) {
                h = j < n ? __builtin_bit_cast(_Float16, reinterpret_cast<const uint16_t *>(src)[r * lds + j])
                          : (_Float16)0.0f;
            } else {
                h = (_Float16)round_to_odd_f32(v);
            }
            reinterpret_cast<uint16_t *>(dst)[idx] = __builtin_bit_cast(uint16_t, h);
        }
        }
    }
}

// Symmetry and finiteness of the stored stack (the problem class has symmetric Q_i, and the
// packed pass reads only upper triangles).  Block (I, J), I <= J, of matrix `mat` compares the
// 64 x 64 tile (I, J) with the transpose of tile (J, I), staged in LDS; both tiles are read as
// 16-byte vectors (stored rows are 16-byte aligned and padded with zeros).  It folds into
// res[3 mat ..] the maximum |Q_rc - Q_cr|, the maximum |Q_rc| and a non-finite flag.  The two
// maxima are non-negative doubles, whose bit patterns order like their values, so unsigned
// atomic maxima over the bits give the same result in any block order.
constexpr int SC_T = 64;

__device__ __forceinline__ double vec_elem(const uint4 &v, int dt, int e)
{
    if (dt == DT_F64) {
        const unsigned lo = e == 0 ? v.x : v.z, hi = e == 0 ? v.y : v.w;
        return __hiloint2double((int)hi, (int)lo);
    }
    const unsigned w = dt == DT_F32 ? (e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w)
                                    : ((e >> 1) == 0 ? v.x : (e >> 1) == 1 ? v.y : (e >> 1) == 2 ? v.z : v.w);
    if (dt == DT_F32) return (double)__uint_as_float(w);
    const uint16_t h = (e & 1) ? (uint16_t)(w >> 16) : (uint16_t)(w & 0xffffu);
    if (dt == DT_BF16) return (double)__uint_as_float((uint32_t)h << 16);
    return (double)(float)__builtin_bit_cast(_Float16, h);
}

__global__ void __launch_bounds__(256) k_sym_check(const void *__restrict__ Q, int dt, int64_t ld, int n,
                                                   int ntile, int nq, unsigned long long *__restrict__ res)
{
    __shared__ double tb[SC_T][SC_T + 1];
    __shared__ double red[2][256 / 64];
    __shared__ int s_bad;
    const int I = blockIdx.x / ntile, J = blockIdx.x - I * ntile;
    if (I > J) return;
    const int es = dt == DT_F64 ? 8 : (dt == DT_F32 ? 4 : 2);
    const int V = 16 / es;                    // elements per 16-byte vector
    const int vpr = SC_T / V;                 // vectors per tile row
    const int nvec = SC_T * vpr;
    const size_t mat_bytes = (size_t)n * ld * es;
    for (int mat = blockIdx.y; mat < nq; mat += gridDim.y) {
        const char *base = (const char *)Q + mat * mat_bytes;
        if (threadIdx.x == 0) s_bad = 0;
        // tb[r][c] = Q[J*T + r][I*T + c]
        for (int k = threadIdx.x; k < nvec; k += 256) {
            const int r = k / vpr, c0 = (k - r * vpr) * V;
            const int row = J * SC_T + r, col = I * SC_T + c0;
            uint4 v = {0u, 0u, 0u, 0u};
            if (row < n && col < ld) v = *(const uint4 *)(base + ((size_t)row * ld + col) * es);
            for (int e = 0; e < V; ++e) tb[r][c0 + e] = vec_elem(v, dt, e);
        }
        __syncthreads();
        double dmax = 0.0, amax = 0.0;
        bool bad = false;
        for (int k = threadIdx.x; k < nvec; k += 256) {
            const int r = k / vpr, c0 = (k - r * vpr) * V;
            const int row = I * SC_T + r, col = J * SC_T + c0;
            if (row < n && col < ld) {
                const uint4 v = *(const uint4 *)(base + ((size_t)row * ld + col) * es);
                for (int e = 0; e < V; ++e) {
                    const double a = vec_elem(v, dt, e);
                    const double b = tb[c0 + e][r];          // Q[col + e][row]
                    bad |= !isfinite(a) || !isfinite(b);
                    dmax = fmax(dmax, fabs(a - b));
                    amax = fmax(amax, fmax(fabs(a), fabs(b)));
                }
            }
        }
        if (bad) s_bad = 1;
        for (int o = 32; o > 0; o >>= 1) {
            dmax = fmax(dmax, __shfl_xor(dmax, o));
            amax = fmax(amax, __shfl_xor(amax, o));
        }
        if ((threadIdx.x & 63) == 0) {
            red[0][threadIdx.x >> 6] = dmax;
            red[1][threadIdx.x >> 6] = amax;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double d = red[0][0], a = red[1][0];
            for (int w = 1; w < 256 / 64; ++w) {
                d = fmax(d, red[0][w]);
                a = fmax(a, red[1][w]);
            }
            atomicMax(res + 3 * mat, (unsigned long long)__builtin_bit_cast(uint64_t, d));
            atomicMax(res + 3 * mat + 1, (unsigned long long)__builtin_bit_cast(uint64_t, a));
            if (s_bad) atomicMax(res + 3 * mat + 2, 1ull);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// smoothed duality gap G_xi(z) (Definition in §4; Euclidean evaluation of the Remark in §4.2)
//   y-part: Py = <G, y'-y> - xi ||y'-y||^2,  y' = Pi_Y(y + G/(2 xi))          (closed form)
//   x-part: Px = -min_{x+D in X} grad'D + 1/2 D'(Q(lambda) + 2 xi I)D         (box QP)
// The box QP runs accelerated projected gradient with gradient restart, step 1/L, L the
// Gershgorin bound of H = Q(lambda) + 2 xi I, until L ||D+ - Z|| <= tol (1 + ||grad||).
// ctl layout: [0] t, [1] beta, [2] restart, [3] done, [4] iters, [5] L, [6] gnorm, [7] tol,
//             [9] Py, [10] Px; words 32..33 hold the inner loop's grid barrier

__global__ void __launch_bounds__(STEP_BS) k_gap_py(const Slot *__restrict__ S,
                                                    const double *__restrict__ y,
                                                    const double *__restrict__ G, double xi,
                                                    double *__restrict__ ctl)
{
    // maximiser y' = Pi_{Y-hat}(y + grad_y Phi / (2 xi)), staged in LDS
    extern __shared__ double yp[];
    const int ny = S->ny;
    for (int l = threadIdx.x; l < ny; l += STEP_BS) yp[l] = y[l] + G[l] / (2.0 * xi);
    __syncthreads();
    project_dual_block(S, yp);
    double v[1] = {0.0};
    for (int l = threadIdx.x; l < ny; l += STEP_BS) {
        const double d = yp[l] - y[l];
        v[0] += G[l] * d - xi * d * d;
    }
    block_sum<1>(v);
    if (threadIdx.x == 0) ctl[9] = v[0];
}

// H = Q(lambda) + 2 xi I (row r per block), Q(lambda) = Q_0 + rho I + sum lambda_i Q_i,
// rowabs[r] = sum_j |H_rj|; matrices with a zero multiplier are skipped (they contribute nothing)
__global__ void __launch_bounds__(STEP_BS) k_form_h(const Slot *__restrict__ S,
                                                    const double *__restrict__ y, double xi,
                                                    double *__restrict__ H, int ldh,
                                                    double *__restrict__ rowabs)
{
    const int n = S->n, m = S->m, p = S->p, r = blockIdx.x;
    const size_t ld = (size_t)S->ld;
    const int dt = S->dtype;
    const int32_t *qmap = S->qmap;
    double v[1] = {0.0};
    for (int j = n + threadIdx.x; j < ldh; j += STEP_BS) H[(size_t)r * ldh + j] = 0.0;   // padding
    for (int j = threadIdx.x; j < n; j += STEP_BS) {
        double h = 0.0;
        if (qmap[0] >= 0) h = load_any(S->Q, dt, ((size_t)qmap[0] * n + r) * ld + j);
        for (int i = 1; i <= m; ++i) {
            const double w = y[p + i - 1];
            const int si = qmap[i];
            if (w == 0.0 || si < 0) continue;
            h += w * load_any(S->Q, dt, ((size_t)si * n + r) * ld + j);
        }
        if (j == r) h += 2.0 * xi + S->q0_shift;
        H[(size_t)r * ldh + j] = h;
        v[0] += fabs(h);
    }
    block_sum<1>(v);
    if (threadIdx.x == 0) rowabs[r] = v[0];
}

__global__ void __launch_bounds__(STEP_BS) k_gap_init(int n, const double *__restrict__ grad,
                                                      const double *__restrict__ rowabs,
                                                      double tol, double *__restrict__ ctl)
{
    double v[1] = {0.0};
    double mx = 0.0;
    for (int j = threadIdx.x; j < n; j += STEP_BS) {
        v[0] += grad[j] * grad[j];
        mx = fmax(mx, rowabs[j]);
    }
    __shared__ double s_mx[STEP_BS];
    s_mx[threadIdx.x] = mx;
    block_sum<1>(v);
    if (threadIdx.x == 0) {
        double mm = 0.0;
        for (int t = 0; t < STEP_BS; ++t) mm = fmax(mm, s_mx[t]);
        ctl[0] = 1.0;
        ctl[1] = 0.0;
        ctl[2] = 0.0;
        ctl[3] = 0.0;
        ctl[4] = 0.0;
        ctl[5] = mm;
        ctl[6] = sqrt(v[0]);
        ctl[7] = tol;
        ctl[8] = 0.0;
    }
}

// Px = -(grad'D + 1/2 D'(H D))
__global__ void __launch_bounds__(STEP_BS) k_gap_px(int n, const double *__restrict__ grad,
                                                    const double *__restrict__ D,
                                                    const double *__restrict__ HD,
                                                    double *__restrict__ ctl)
{
    double v[1] = {0.0};
    for (int j = threadIdx.x; j < n; j += STEP_BS) v[0] += grad[j] * D[j] + 0.5 * D[j] * HD[j];
    block_sum<1>(v);
    if (threadIdx.x == 0) ctl[10] = -v[0];
}

// ---- the box QP in one cooperative launch -------------------------------------------------
// Every block owns rows r = 4 b + w + 4 G k of H (one wave per row at a time) and the same
// entries of Z, D and Dn.  An iteration is: (A) (H Z)_r, the projected step Dn_r and the two
// partial sums of the rows owned, per block; grid barrier; (B) every block sums all blocks'
// partials in the same fixed order, so all take the same momentum, restart and stop decision,
// then applies Z, D to its rows; grid barrier.  The stop decision is therefore uniform and every
// block leaves the loop at the same iteration (at the latest after max_inner iterations).
// The barrier counts arrivals with agent-scope atomics (release on arrival, acquire on the
// generation word) and gives up after a bounded spin, flagging bar->err, so a launch cannot hang.

constexpr int FISTA_BS = 256;
constexpr int FISTA_ROWS = 4;
constexpr long long BAR_SPIN_LIMIT = 1ll << 25;   // ~2 s of 64-cycle sleeps

__device__ __forceinline__ bool grid_barrier(GridBar *bar, unsigned nblocks, unsigned &gen)
{
    __shared__ int s_ok;
    __syncthreads();       // the block's writes of this phase are ordered before thread 0's arrival
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned g = gen;
        // release: the block's writes become visible at device scope before the arrival counts
        const unsigned arrived = __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&bar->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar->gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // spin on coherent relaxed loads (no cache invalidation per probe)
            long long spins = 0;
            while (__hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > BAR_SPIN_LIMIT) {
                    ok = 0;
                    __hip_atomic_store(&bar->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        // acquire once: the other blocks' writes are read afresh by this block
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        gen = g + 1u;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

__global__ void __launch_bounds__(FISTA_BS) k_fista_coop(const Slot *__restrict__ S, int n,
                                                         const double *__restrict__ x,
                                                         const double *__restrict__ grad,
                                                         const double *__restrict__ H, int ldh,
                                                         double *Z, double *D, double *Dn,
                                                         double *part, double *ctl, int64_t max_inner,
                                                         GridBar *bar)
{
    __shared__ double s_dec[3];   // t, beta, flags (restart + 2 done)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned G = gridDim.x;
    const int rstep = (int)G * (FISTA_BS / 64);
    unsigned gen = __hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double t = ctl[0], beta = ctl[1];
    const double L = ctl[5], gn = ctl[6], tol = ctl[7];
    double iters = ctl[4];
    bool done = ctl[3] != 0.0 || iters >= (double)max_inner;
    while (!done) {
        // (A) rows owned: (H Z)_r, projected step, partial sums
        double v[2] = {0.0, 0.0};
        for (int r = (int)blockIdx.x * (FISTA_BS / 64) + wave; r < n; r += rstep) {
            const double *h = H + (size_t)r * ldh;
            double acc = 0.0;
            for (int j = 2 * lane; j < n; j += 128) {      // ldh and Z are padded with zeros
                acc = fma(h[j], Z[j], acc);
                acc = fma(h[j + 1], Z[j + 1], acc);
            }
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (lane == 0) {
                const double zr = Z[r], xr = x[r];
                const double dn = clipd(zr - (grad[r] + acc) / L, S->lb[r] - xr, S->ub[r] - xr);
                Dn[r] = dn;
                const double a = dn - zr;
                v[0] += a * a;
                v[1] += (zr - dn) * (dn - D[r]);
            }
        }
        block_sum<2>(v);
        if (threadIdx.x == 0) {
            part[2 * blockIdx.x] = v[0];
            part[2 * blockIdx.x + 1] = v[1];
        }
        if (!grid_barrier(bar, G, gen)) return;
        // (B) every block: the same fixed-order total, the same decision
        double u[2] = {0.0, 0.0};
        for (int b = threadIdx.x; b < (int)G; b += FISTA_BS) {
            u[0] += part[2 * b];
            u[1] += part[2 * b + 1];
        }
        block_sum<2>(u);
        if (threadIdx.x == 0) {
            double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
            double fl = 0.0;
            if (u[1] > 0.0) {          // gradient restart
                tn = 1.0;
                fl = 1.0;
            } else {
                beta = (t - 1.0) / tn;
            }
            iters += 1.0;
            if (L * sqrt(u[0]) <= tol * (1.0 + gn) || iters >= (double)max_inner) fl += 2.0;
            s_dec[0] = tn;
            s_dec[1] = beta;
            s_dec[2] = fl;
        }
        __syncthreads();
        t = s_dec[0];
        beta = s_dec[1];
        const bool rst = ((int)s_dec[2] & 1) != 0;
        done = ((int)s_dec[2] & 2) != 0;
        for (int r = (int)blockIdx.x * (FISTA_BS / 64) + wave; r < n; r += rstep) {
            if (lane == 0) {
                const double dn = Dn[r];
                Z[r] = rst ? dn : dn + beta * (dn - D[r]);
                D[r] = dn;
            }
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctl[0] = t;
            ctl[1] = beta;
            ctl[2] = rst ? 1.0 : 0.0;
            ctl[3] = done ? 1.0 : 0.0;
            ctl[4] = iters;
        }
        if (!grid_barrier(bar, G, gen)) return;
    }
}

// The same loop with Z and D held by every block in LDS (n small enough): phase B then has
// every block update all of Z and D itself from the step Dn that all blocks wrote in phase A,
// so one grid barrier per iteration suffices.  Dn and the partial sums alternate between two
// buffers by iteration parity: a block that runs ahead writes the other buffer, which every
// slower block has finished reading (it passed the previous barrier).  Block 0 writes the
// final D back to global memory.
__global__ void __launch_bounds__(FISTA_BS) k_fista_coop_lds(const Slot *__restrict__ S, int n,
                                                             const double *__restrict__ x,
                                                             const double *__restrict__ grad,
                                                             const double *__restrict__ H, int ldh,
                                                             double *D, double *Dn2, int nstride,
                                                             double *part2, double *ctl,
                                                             int64_t max_inner, GridBar *bar)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int nw = (n + 1) & ~1;
    double *Zs = reinterpret_cast<double *>(smem);
    double *Ds = Zs + nw;
    __shared__ double s_dec[3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned G = gridDim.x;
    const int rstep = (int)G * (FISTA_BS / 64);
    for (int j = threadIdx.x; j < nw; j += FISTA_BS) {
        Zs[j] = 0.0;
        Ds[j] = 0.0;
    }
    unsigned gen = __hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double t = ctl[0], beta = ctl[1];
    const double L = ctl[5], gn = ctl[6], tol = ctl[7];
    double iters = ctl[4];
    bool done = ctl[3] != 0.0 || iters >= (double)max_inner;
    __syncthreads();
    int par = 0;
    while (!done) {
        double *Dn = Dn2 + (size_t)par * nstride;
        double *part = part2 + (size_t)par * GAP_MAX_BLOCKS;   // G <= GAP_MAX_BLOCKS / 2
        // (A) rows owned: (H Z)_r from the block's own Z, projected step, partial sums
        double v[2] = {0.0, 0.0};
        for (int r = (int)blockIdx.x * (FISTA_BS / 64) + wave; r < n; r += rstep) {
            // 16-byte loads, four in flight per lane (ldh is padded with zeros, Zs[n] = 0)
            const double2 *h2 = reinterpret_cast<const double2 *>(H + (size_t)r * ldh);
            const double2 *z2 = reinterpret_cast<const double2 *>(Zs);
            const int nv = nw >> 1;
            double acc = 0.0;
            int jv = lane;
            for (; jv + 192 < nv; jv += 256) {
                const double2 a0 = h2[jv], a1 = h2[jv + 64], a2 = h2[jv + 128], a3 = h2[jv + 192];
                const double2 b0 = z2[jv], b1 = z2[jv + 64], b2 = z2[jv + 128], b3 = z2[jv + 192];
                acc = fma(a0.x, b0.x, acc);
                acc = fma(a0.y, b0.y, acc);
                acc = fma(a1.x, b1.x, acc);
                acc = fma(a1.y, b1.y, acc);
                acc = fma(a2.x, b2.x, acc);
                acc = fma(a2.y, b2.y, acc);
                acc = fma(a3.x, b3.x, acc);
                acc = fma(a3.y, b3.y, acc);
            }
            for (; jv < nv; jv += 64) {
                const double2 a = h2[jv], b = z2[jv];
                acc = fma(a.x, b.x, acc);
                acc = fma(a.y, b.y, acc);
            }
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (lane == 0) {
                const double zr = Zs[r], xr = x[r];
                const double dn = clipd(zr - (grad[r] + acc) / L, S->lb[r] - xr, S->ub[r] - xr);
                Dn[r] = dn;
                const double a = dn - zr;
                v[0] += a * a;
                v[1] += (zr - dn) * (dn - Ds[r]);
            }
        }
        block_sum<2>(v);
        if (threadIdx.x == 0) {
            part[2 * blockIdx.x] = v[0];
            part[2 * blockIdx.x + 1] = v[1];
        }
        if (!grid_barrier(bar, G, gen)) return;
        // (B) every block: the same fixed-order totals and decision, then all of Z and D
        double u[2] = {0.0, 0.0};
        for (int b = threadIdx.x; b < (int)G; b += FISTA_BS) {
            u[0] += part[2 * b];
            u[1] += part[2 * b + 1];
        }
        block_sum<2>(u);
        if (threadIdx.x == 0) {
            double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
            double fl = 0.0;
            if (u[1] > 0.0) {          // gradient restart
                tn = 1.0;
                fl = 1.0;
            } else {
                beta = (t - 1.0) / tn;
            }
            iters += 1.0;
            if (L * sqrt(u[0]) <= tol * (1.0 + gn) || iters >= (double)max_inner) fl += 2.0;
            s_dec[0] = tn;
            s_dec[1] = beta;
            s_dec[2] = fl;
        }
        __syncthreads();
        t = s_dec[0];
        beta = s_dec[1];
        const bool rst = ((int)s_dec[2] & 1) != 0;
        done = ((int)s_dec[2] & 2) != 0;
        for (int j = threadIdx.x; j < n; j += FISTA_BS) {
            const double dn = Dn[j];
            Zs[j] = rst ? dn : dn + beta * (dn - Ds[j]);
            Ds[j] = dn;
        }
        __syncthreads();
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctl[0] = t;
            ctl[1] = beta;
            ctl[2] = rst ? 1.0 : 0.0;
            ctl[3] = done ? 1.0 : 0.0;
            ctl[4] = iters;
        }
        par ^= 1;
    }
    if (blockIdx.x == 0)
        for (int j = threadIdx.x; j < n; j += FISTA_BS) D[j] = Ds[j];
}

hipError_t launch_fista_coop(hipStream_t s, const Slot *slot, int n, const double *x,
                             const double *grad, const double *H, int ldh, double *Z, double *D,
                             double *Dn, double *part, double *ctl, int64_t max_inner, GridBar *bar,
                             int max_blocks, int max_lds, int nstride)
{
    // a block per 4 x FISTA_ROWS rows (each wave about FISTA_ROWS rows of H per iteration):
    // fewer blocks make the barrier cheaper
    int G = (n + FISTA_BS / 64 * FISTA_ROWS - 1) / (FISTA_BS / 64 * FISTA_ROWS);
    if (G > max_blocks) G = max_blocks;
    if (G > GAP_MAX_BLOCKS / 2) G = GAP_MAX_BLOCKS / 2;
    if (G < 1) G = 1;
    const size_t lds = (size_t)2 * ((n + 1) & ~1) * sizeof(double);
    if (lds + 1024 <= (size_t)max_lds) {
        // Dn in two buffers nstride apart; the partials in the two halves of `part`
        double *Dn2 = Dn;
        (void)Z;
        void *args[] = {(void *)&slot, (void *)&n, (void *)&x, (void *)&grad, (void *)&H, (void *)&ldh,
                        (void *)&D, (void *)&Dn2, (void *)&nstride, (void *)&part, (void *)&ctl,
                        (void *)&max_inner, (void *)&bar};
        return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_fista_coop_lds), dim3(G),
                                          dim3(FISTA_BS), args, lds, s);
    }
    void *args[] = {(void *)&slot, (void *)&n, (void *)&x, (void *)&grad, (void *)&H, (void *)&ldh,
                    (void *)&Z, (void *)&D, (void *)&Dn, (void *)&part, (void *)&ctl,
                    (void *)&max_inner, (void *)&bar};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_fista_coop), dim3(G), dim3(FISTA_BS),
                                      args, 0, s);
}

hipError_t prepare_fista_coop(int max_lds)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fista_coop_lds),
                               hipFuncAttributeMaxDynamicSharedMemorySize, max_lds - 1024);
}

// decision of eq. (ada_restart) with G_xi = Py + Px from the device
__global__ void __launch_bounds__(STEP_BS) k_restart_decision_dev(Slot *__restrict__ S,
                                                                  const double *__restrict__ ctl)
{
    __shared__ int s_rs;
    if (threadIdx.x == 0) {
        s_rs = 0;
        if (reinterpret_cast<const GridBar *>(ctl + 32)->err) {
            S->status = ST_NUMERICAL;   // the inner loop's barrier gave up: no decision on partial values
            s_rs = -1;
        }
    }
    __syncthreads();
    if (s_rs == -1) return;
    if (threadIdx.x == 0) {
        const double gap = ctl[9] + ctl[10];
        S->gap_evals += 1;
        S->last_gap = gap;
        int rs = 0;
        if (S->k == S->ada_first) {
            S->Gref = gap;
        } else if (gap <= S->q_restart * S->Gref) {
            S->Gref = gap;
            rs = (S->restart_from_avg && S->T > 0.0) ? 2 : 1;
        }
        S->status = ST_RUNNING;
        s_rs = rs;
    }
    __syncthreads();
    if (s_rs) restart_epoch(S, s_rs);
}

hipError_t launch_restart_decision_dev(hipStream_t s, Slot *slot, const double *ctl)
{
    k_restart_decision_dev<<<1, STEP_BS, 0, s>>>(slot, ctl);
    return hipGetLastError();
}

hipError_t launch_gap_setup(hipStream_t s, const Slot *slot, int n, int ny, const double *y,
                            const double *G, const double *grad, double xi, double *H, int ldh,
                            double *rowabs, double tol, double *ctl)
{
    k_gap_py<<<1, STEP_BS, (size_t)(ny > 0 ? ny : 1) * sizeof(double), s>>>(slot, y, G, xi, ctl);
    k_form_h<<<n, STEP_BS, 0, s>>>(slot, y, xi, H, ldh, rowabs);
    k_gap_init<<<1, STEP_BS, 0, s>>>(n, grad, rowabs, tol, ctl);
    return hipGetLastError();
}

hipError_t launch_gap_finish(hipStream_t s, int n, const double *grad, const double *H, int ldh,
                             int nw, const double *D, double *HD, double *ctl)
{
    hipError_t e = launch_hmv(s, H, n, ldh, D, nw, HD, ctl, 1);
    if (e != hipSuccess) return e;
    k_gap_px<<<1, STEP_BS, 0, s>>>(n, grad, D, HD, ctl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// launch wrappers

template <int B>
static hipError_t group_b(hipStream_t s, Slot *slots, const int *live, int nslots, const Tile *tiles, int ntiles,
                          const int *starts,
                          int dtype, int variants, int max_nblk_step, int max_ny, int max_nw, int max_epi,
                          int pass_grid, int nt, hipEvent_t ev0, hipEvent_t ev1, const SymPass *sym,
                          const Sym16Launch *s16)
{
    const size_t step_lds = (size_t)(B + 1) * (size_t)(max_ny > 0 ? max_ny : 1) * sizeof(double);
    const dim3 vgrid(max_nblk_step, nslots);
    if (variants & HAS_YX) k_step<B><<<vgrid, STEP_BS, step_lds, s>>>(slots, live);
    if (variants & HAS_XY) k_step_xy<B><<<vgrid, STEP_BS, step_lds, s>>>(slots, live);
    if (ev0) (void)hipEventRecord(ev0, s);
    (void)launch_pass_only(s, slots, tiles, ntiles, starts, B, dtype, max_nw, pass_grid, nt, sym, s16);
    if (ev1) (void)hipEventRecord(ev1, s);
    k_epi<B><<<dim3(max_epi, nslots), STEP_BS, 0, s>>>(slots, live);
    if (variants & HAS_XY) k_post_xy<B><<<vgrid, STEP_BS, step_lds, s>>>(slots, live);
    k_ctrl<B><<<nslots, STEP_BS, (size_t)(max_ny > 0 ? 2 * max_ny : 1) * sizeof(double), s>>>(slots, live);
    return hipGetLastError();
}

hipError_t launch_group(hipStream_t s, Slot *slots, const int *live, int nslots, const Tile *tiles,
                        int ntiles, const int *starts, int B, int dtype, int variants,
                        int max_nblk_step, int max_ny, int max_nw, int max_epi, int pass_grid,
                        int nt, hipEvent_t ev0, hipEvent_t ev1, const SymPass *sym,
                        const Sym16Launch *s16)
{
    switch (B) {
    case 1: return group_b<1>(s, slots, live, nslots, tiles, ntiles, starts, dtype, variants, max_nblk_step, max_ny, max_nw, max_epi, pass_grid, nt, ev0, ev1, sym, s16);
    case 2: return group_b<2>(s, slots, live, nslots, tiles, ntiles, starts, dtype, variants, max_nblk_step, max_ny, max_nw, max_epi, pass_grid, nt, ev0, ev1, sym, s16);
    case 3: return group_b<3>(s, slots, live, nslots, tiles, ntiles, starts, dtype, variants, max_nblk_step, max_ny, max_nw, max_epi, pass_grid, nt, ev0, ev1, sym, s16);
    default: return group_b<4>(s, slots, live, nslots, tiles, ntiles, starts, dtype, variants, max_nblk_step, max_ny, max_nw, max_epi, pass_grid, nt, ev0, ev1, sym, s16);
    }
}

hipError_t launch_epi_anchor(hipStream_t s, Slot *slots, const int *live, int nslots, int max_epi)
{
    // k_epi<1> handles the anchor mode for any B (it only touches candidate 0)
    k_epi<1><<<dim3(max_epi, nslots), STEP_BS, 0, s>>>(slots, live);
    return hipGetLastError();
}

hipError_t launch_grad(hipStream_t s, const Slot *slot, int n, const double *U, const double *y,
                       double *out)
{
    k_grad<<<(n + STEP_BS - 1) / STEP_BS, STEP_BS, 0, s>>>(slot, U, y, out);
    return hipGetLastError();
}

hipError_t launch_kkt(hipStream_t s, const Slot *slot, int n, int ny, const double *x,
                      const double *y, const double *U, const double *G, double *part,
                      double *out6)
{
    const int nblk = (n + STEP_BS - 1) / STEP_BS;
    k_kkt_part<<<nblk, STEP_BS, 0, s>>>(slot, x, y, U, part);
    k_kkt_fin<<<1, STEP_BS, (size_t)(ny > 0 ? 2 * ny : 1) * sizeof(double), s>>>(slot, nblk, y, G, part, out6);
    return hipGetLastError();
}

hipError_t launch_convert(hipStream_t s, const void *src, int src_dtype, int64_t ld_src,
                          void *dst, int dst_dtype, int64_t ld_dst, int64_t rows, int64_t n)
{
    const int64_t total = rows * ld_dst;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    k_convert<<<(unsigned)blocks, 256, 0, s>>>(src, src_dtype, ld_src, dst, dst_dtype, ld_dst, rows, n);
    return hipGetLastError();
}

hipError_t launch_sym_check(hipStream_t s, const void *Q, int dtype, int64_t ld, int n, int nq,
                            unsigned long long *res)
{
    const int ntile = (n + SC_T - 1) / SC_T;
    const dim3 grid((unsigned)((int64_t)ntile * ntile), (unsigned)(nq < 65535 ? nq : 65535));
    k_sym_check<<<grid, 256, 0, s>>>(Q, dtype, ld, n, ntile, nq, res);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_fill(double *__restrict__ v, int64_t n, double value)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) v[i] = value;
}

hipError_t launch_fill(hipStream_t s, double *v, int64_t n, double value)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    k_fill<<<(unsigned)blocks, 256, 0, s>>>(v, n, value);
    return hipGetLastError();
}

// lam = ||z|| (fixed-order block sum), v = z / lam
__global__ void __launch_bounds__(STEP_BS) k_pow_normalize(const double *__restrict__ z, int n,
                                                           double *__restrict__ v, double *__restrict__ lam)
{
    double acc[1] = {0.0};
    for (int j = threadIdx.x; j < n; j += STEP_BS) acc[0] += z[j] * z[j];
    block_sum<1>(acc);
    __shared__ double s_l;
    if (threadIdx.x == 0) {
        s_l = sqrt(acc[0]);
        lam[0] = s_l;
    }
    __syncthreads();
    const double l = s_l;
    if (l > 0.0)
        for (int j = threadIdx.x; j < n; j += STEP_BS) v[j] = z[j] / l;
}

hipError_t launch_pow_normalize(hipStream_t s, const double *z, int n, double *v, double *lam)
{
    k_pow_normalize<<<1, STEP_BS, 0, s>>>(z, n, v, lam);
    return hipGetLastError();
}

hipError_t launch_start(hipStream_t s, Slot *slot)
{
    k_start<<<1, STEP_BS, 0, s>>>(slot);
    return hipGetLastError();
}


}  // namespace qcqp
