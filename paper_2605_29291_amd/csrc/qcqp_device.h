// Device-side data layout shared by the HIP kernels and the host runtime of the rAPDB library.
//
// One "slot" is one resident QCQP solve.  A trial group (one backtracking test for every
// running slot) is four launches on one stream (five when a slot runs APDB-xy):
//   k_step  : APDB-yx (eq. (apdb-yx-y), §3.2): dual step + cone projection, then primal step +
//             box projection, for spec_trials candidate step sizes tau * eta^b;
//   k_step_xy: APDB-xy (Algorithm 1): primal step with momentum on grad_x Phi + box projection;
//             both compute the KKT partials of the iterate;
//   k_pass  : the Q-stack pass -- one streamed GEMV over the stacked ((m+1) n) x n matrix per
//             slot, all candidates at once, x (or the step d) staged in LDS;
//   k_epi   : per-matrix dot products (g_i, f, d'(Q_i d)) with fixed-order block reductions;
//   k_post_xy: APDB-xy only: dual step at the new x and the gradient differences of its E_k;
//   k_ctrl  : FP64 test E_k <= rhs per candidate in order, acceptance, step-size/momentum/
//             averaging bookkeeping (Algorithm 1), fixed restarts (Algorithm 2), KKT stop.
// The host never reads per-trial data: it enqueues groups and polls a status word.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qcqp {

constexpr int MAXB = 4;            // max speculative candidates per pass
constexpr int NPART = 4 + MAXB;    // step-kernel partials per block: rx2, s0, s1, s2, dd[b]
constexpr int NPART2 = 2 * MAXB;   // xy post-kernel partials per block: |a_b|^2, |c_b|^2
constexpr int STEP_BS = 256;       // threads per block of the vector kernels
constexpr int STEP_COLS = 64;      // columns per step-kernel block (one per lane of a wave)
constexpr int STEP_WAVES = STEP_BS / STEP_COLS;   // waves splitting the matrices of a column
constexpr int PASS_BS = 256;       // threads per block of the pass kernel

enum SlotStatus : int32_t {
    ST_RUNNING = 0,
    ST_CONVERGED = 1,
    ST_MAX_ITER = 2,
    ST_NUMERICAL = 3,
    ST_GAP_PENDING = 4,   // adaptive restart: host evaluates G_xi, then resumes the slot
    ST_IDLE = 5
};

enum SlotMode : int32_t {
    MODE_TRIAL = 0,       // candidates -> pass -> test
    MODE_ANCHOR = 1       // direct FP64-accumulated pass at x (start / restart)
};

enum StoreType : int32_t { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_F16 = 3 };

enum Variant : int32_t { VAR_YX = 0, VAR_XY = 1 };

enum LambdaSet : int32_t { LAMBDA_NONNEG = 0, LAMBDA_SIMPLEX = 1, LAMBDA_CONES = 2 };

// second-order cones of at least this dimension are projected by a whole block, smaller ones by
// one thread each
constexpr int SOC_BLOCK_DIM = 128;

// bit mask of the variants present among the slots of a launch
constexpr int HAS_YX = 1, HAS_XY = 2;

struct Slot {
    // ---- constants (set at admission) ----
    int32_t n, m, p, ny;          // ny = p + m
    int32_t nq, has_q0;           // stored matrices nq = m + has_q0
    int32_t ld, dtype;            // row stride (elements) and storage type of Q
    int32_t c_nm, restart, restart_from_avg, incremental;
    int32_t B, nblk_step, nw, variant;   // nw = n rounded up to the pass vector width
    int32_t lambda_set;           // dual domain of lambda: R^m_+ or the unit simplex
    int32_t stop_rule;            // 0: relative KKT <= tol; 1: the §5.1 criterion against f_star
    double q0_shift;              // rho: the objective's Hessian is Q_0 + rho I
    double ball, ball_v, ball_l;  // dual ball radii (0 = none): ||y||, ||v||, ||lambda||
    int32_t n_soc, m0;            // cones: count, and the R_+ entries of lambda before them
    int32_t n_soc_big, pad2;      // cones of dimension >= SOC_BLOCK_DIM
    const int32_t *soc_off;       // n_soc start offsets within lambda, then n_soc dimensions
    const int32_t *soc_big;       // indices of the large cones
    const int32_t *qmap;          // m+1: position of Q_i among the stored matrices, -1 if absent
    int64_t restart_every, ada_first, ada_every, max_iter;
    double eta, tau_bar, gamma0, mu, c_alpha, c_beta, delta, tol, q_restart;
    double cnorm, bnorm;          // ||c_{1..m}||, ||b||  (KKT scales)
    double f_star;                // optimal value for stop rule 1
    const void *Q;
    const double *q, *c, *A, *b, *lb, *ub;
    // ---- buffers (pointers swapped by k_ctrl on acceptance) ----
    double *x, *xc[MAXB];         // iterate x^k and candidates x^{k+1}(tau_b)
    double *U, *Uc[MAXB];         // [Q_i x] of the iterate / of the candidates, (m+1) x n
    double *W[MAXB];              // incremental pass outputs [Q_i d_b]
    double *y, *yc[MAXB];         // y^k = (v, lambda) and candidates, ny
    double *G, *Gc[MAXB], *Gp;    // (Ax-b, g(x), f(x)), ny + 1; Gp = value at x^{k-1}
    double *dG[MAXB];             // incremental: exact difference Gc - G, ny + 1
    double *e;                    // MAXB x (m+1): d_b'(Q_i d_b)
    double *cx, *cy;              // weighted sums for the ergodic average
    double *part;                 // nblk_step x NPART step partials
    double *gxk, *gxp;            // xy: grad_x Phi at (x^k, y^k) and at (x^{k-1}, y^{k-1}), n
    double *part2;                // xy: nblk_step x NPART2 post-kernel partials
    // ---- mutable scalars ----
    double tau, tau_prev, sig_prev, gam, sig0, alpha_k, beta_k, T;
    double kkt[4];                // rel_kkt, rel_dual, rel_pri, rel_comp of the iterate
    double crit;                  // the stop rule's value at the iterate
    double f, maxviol;
    double Gref, last_gap;
    int64_t k, ke, trials, passes, restarts, gap_evals, iter_trials;
    int32_t status, mode;
    int32_t fresh;            // 1 when U and G are exact FP64 values at x (no incremental drift)
    int32_t anchor_keep_gp;   // 1: the pending anchor refreshes U/G only (no epoch start)
};

struct Tile {
    int32_t slot;
    int32_t row0;    // first stored row (0 .. nq*n); a tile lies within one stored matrix
    int32_t nrows;
    int32_t lpr;     // lanes per row: 16, 32 or 64
    int32_t uoff;    // output row of stored row r is uoff + r: (i - s) n for Q_i stored s-th
};

// ---- launch wrappers (kernels.hip) ----
// one trial group for the slots listed in live[0..nslots) (live = NULL: slots 0..nslots-1);
// variants = HAS_YX | HAS_XY mask
// tiles[starts[b] .. starts[b+1]) go to pass block b (starts: min(pass_grid, ntiles) + 1 entries,
// or NULL for equal tile counts per block)
// Packed symmetric stack (options.sym_pass): for every stored matrix s, the tiles (I, J), I <= J,
// of SYM_T x SYM_T FP64 values (row-major inside a tile, zero beyond n), row of tiles by row of
// tiles.  One 64-lane block per tile yields the row products Q_IJ w_J and, for I < J, the
// column products Q_IJ' w_I; a second kernel adds them per output row in a fixed order.
constexpr int SYM_T = 128;
constexpr int SYM_TILE_STRIDE = SYM_T * SYM_T;   // doubles from one packed tile to the next
// With 16-bit storage (dt = DT_BF16 / DT_F16) the tiles are SYM16_T x SYM16_T stored elements
// (P16) and the per-tile results FP32 (ws16); only the trial passes of the incremental mode use
// them (W_b = Q d_b), the anchors stream the row-major stack.
constexpr int SYM16_T = 256;
constexpr int SYM16_TILE = SYM16_T * SYM16_T;    // elements from one packed 16-bit tile to the next
struct SymPass {
    const double *P;         // nq * ntt packed tiles (FP64 storage)
    double *ws;              // per tile: row results [B][SYM_T], then column results [B][SYM_T]
    const int32_t *ubase;    // output row of the first row of stored matrix s: (matrix index) n
    int32_t n, NT, ntt, nq;  // NT = ceil(n / tile side) tiles per side, ntt = NT (NT + 1) / 2
    int32_t B;               // candidate slots of the workspace
    int32_t dt;              // storage type of the packed tiles
    const uint16_t *P16;     // 16-bit storage: nq * ntt packed tiles
    float *ws16;             // 16-bit storage: per tile [2][B][SYM16_T] (rows, then columns)
};
hipError_t launch_sym_pack(hipStream_t s, const double *Q, int64_t ld, const SymPass &sp, double *P);
// Launch description of the 16-bit packed trial passes of one or more slots
struct Sym16Launch {
    int32_t dt, B;           // storage type (DT_BF16 / DT_F16) and candidates
    const SymPass *descs;    // device, indexed by slot: each packed slot's tiles and results
    const int2 *work;        // device: (slot, tile) per block of the tile kernel; NULL: slot 0,
                             // tile = block
    int32_t nwork;
    const int2 *work_r;      // device: (slot, s NT + I) per block of the row sums; NULL: slot 0
    int32_t nwork_r;
    // a batch's packed slots' row-major tiles (streamed for their anchors only); NULL: the
    // launch's tiles all belong to the packed slot of a single solve
    const Tile *tiles;
    int32_t ntiles, grid;
    const int *starts;
};
// *inexact |= 1 when a diagonal entry's half is not exact in the storage type
hipError_t launch_sym_pack16(hipStream_t s, const void *Q, int64_t ld, int dt, const SymPass &sp, void *P,
                             unsigned *inexact);

// one trial group; sym != NULL streams the packed FP64 symmetric stack instead of the tiles;
// s16 != NULL adds the 16-bit packed trial passes it describes
hipError_t launch_group(hipStream_t s, Slot *slots, const int *live, int nslots, const Tile *tiles,
                        int ntiles, const int *starts, int B, int dtype, int variants,
                        int max_nblk_step, int max_ny, int max_nw, int max_epi, int pass_grid,
                        int nt, hipEvent_t ev0, hipEvent_t ev1, const SymPass *sym = nullptr,
                        const Sym16Launch *s16 = nullptr);
hipError_t launch_pass_only(hipStream_t s, Slot *slots, const Tile *tiles, int ntiles,
                            const int *starts, int B, int dtype, int max_nw, int pass_grid, int nt,
                            const SymPass *sym = nullptr, const Sym16Launch *s16 = nullptr);
// pass grid: resident blocks per CU of k_pass for this configuration
int pass_blocks_per_cu(int B, int dtype, int max_nw);
size_t pass_lds_bytes(int B, int dtype, int max_nw);
// rows one lane group of the trial pass streams at a time for this storage type
int pass_rows_per_step(int dtype);
hipError_t launch_epi_anchor(hipStream_t s, Slot *slots, const int *live, int nslots, int max_epi);
hipError_t launch_matvec1(hipStream_t s, const void *Q, int dtype, int n, int ld, int row_base,
                          const double *v, int nw, double *z);
hipError_t launch_grad(hipStream_t s, const Slot *slot, int n, const double *U, const double *y,
                       double *out);
hipError_t launch_kkt(hipStream_t s, const Slot *slot, int n, int ny, const double *x,
                      const double *y, const double *U, const double *G, double *part,
                      double *out6);
hipError_t launch_convert(hipStream_t s, const void *src, int src_dtype, int64_t ld_src,
                          void *dst, int dst_dtype, int64_t ld_dst, int64_t rows, int64_t n);
// res: 3 zeroed words per stored matrix {max |Q_rc - Q_cr|, max |Q_rc|} as double bits, non-finite flag
hipError_t launch_sym_check(hipStream_t s, const void *Q, int dtype, int64_t ld, int n, int nq,
                            unsigned long long *res);
// Grid barrier of the cooperative G_xi inner loop (device memory, zero-initialised count)
struct GridBar {
    unsigned count;   // blocks arrived at the current barrier
    unsigned gen;     // barriers completed
    unsigned err;     // set when a wait exceeded its spin limit
    unsigned pad;
};
// Partial sums of the G_xi inner loop: at most this many blocks
constexpr int GAP_MAX_BLOCKS = 1024;
// the G_xi box QP by accelerated projected gradient to convergence in one cooperative launch
// (at most max_blocks blocks); ctl as for launch_gap_setup; bar->count must be 0.  Z, D, Dn:
// n-vectors (Z, D zero); with Z and D in LDS (when 2n doubles fit max_lds) Dn and the n doubles
// nstride after it are the two step buffers, and `part` holds 2 GAP_MAX_BLOCKS doubles
hipError_t launch_fista_coop(hipStream_t s, const Slot *slot, int n, const double *x,
                             const double *grad, const double *H, int ldh, double *Z, double *D,
                             double *Dn, double *part, double *ctl, int64_t max_inner, GridBar *bar,
                             int max_blocks, int max_lds, int nstride);
hipError_t prepare_fista_coop(int max_lds);
// adaptive restart decision with G_xi = ctl[9] + ctl[10] read on the device; the first
// evaluation of a run (k = ada_first) only records the reference
hipError_t launch_restart_decision_dev(hipStream_t s, Slot *slot, const double *ctl);
// v[0..n) = value
hipError_t launch_fill(hipStream_t s, double *v, int64_t n, double value);
// one power-iteration normalisation: lam[0] = ||z||, v = z / ||z|| (v unchanged when z = 0)
hipError_t launch_pow_normalize(hipStream_t s, const double *z, int n, double *v, double *lam);
hipError_t launch_start(hipStream_t s, Slot *slot);
hipError_t launch_gap_setup(hipStream_t s, const Slot *slot, int n, int ny, const double *y,
                            const double *G, const double *grad, double xi, double *H, int ldh,
                            double *rowabs, double tol, double *ctl);
hipError_t launch_gap_finish(hipStream_t s, int n, const double *grad, const double *H, int ldh,
                             int nw, const double *D, double *HD, double *ctl);
hipError_t launch_hmv(hipStream_t s, const double *H, int n, int ldh, const double *v, int nw,
                      double *z, const double *ctl, int force);
hipError_t prepare_kernels(int max_lds_bytes);

}  // namespace qcqp
