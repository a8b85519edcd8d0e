// Q-stack pass kernels (gfx950): the streamed GEMV over the stack of constraint matrices that
// every backtracking trial of APDB-yx (§3.2) evaluates -- U_i = Q_i w for i = 0..m with w the
// trial point, the step or the iterate -- plus the single-matrix products it shares code with
// (power iteration for the default step, H v inside the smoothed-gap box QP).
//
// Paper: "Restarted Accelerated Primal-Dual Algorithms with Adaptive Stepsizes for Nonlinear
// Conic Constrained Convex Optimization" (arXiv 2605.29291), eq. (qcqp-coupling) in §2.1.
#include "qcqp_device.h"

#include <type_traits>

namespace qcqp {

// ---------------------------------------------------------------------------------------
// storage types: one 16-byte vector load per lane per chunk.  Loads go through the global
// address space (the stack pointer is read from the slot, so the compiler cannot infer it);
// NT selects non-temporal loads for stacks that cannot stay cache-resident across passes.

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 g_u32x4;

template <bool NT>
__device__ __forceinline__ u32x4 ld16(const void *base, size_t byte_off)
{
    const g_u32x4 *p = (const g_u32x4 *)((const char *)base + byte_off);
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <int DT> struct Store;

template <> struct Store<DT_F64> {
    static constexpr int V = 2;
    static constexpr int ES = 8;
    using acc_t = double;
    __device__ static __forceinline__ double get(const u32x4 &v, int e)
    {
        const unsigned lo = e == 0 ? v.x : v.z, hi = e == 0 ? v.y : v.w;
        return __hiloint2double((int)hi, (int)lo);
    }
};

template <> struct Store<DT_F32> {
    static constexpr int V = 4;
    static constexpr int ES = 4;
    using acc_t = float;
    __device__ static __forceinline__ float get(const u32x4 &v, int e)
    {
        return __uint_as_float(e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w)));
    }
};

template <> struct Store<DT_BF16> {
    static constexpr int V = 8;
    static constexpr int ES = 2;
    using acc_t = float;
    __device__ static __forceinline__ float get(const u32x4 &v, int e)
    {
        const uint32_t w = (e >> 1) == 0 ? v.x : ((e >> 1) == 1 ? v.y : ((e >> 1) == 2 ? v.z : v.w));
        const uint32_t bits = (e & 1) ? (w & 0xffff0000u) : (w << 16);
        return __uint_as_float(bits);   // bf16 -> fp32 is exact
    }
};

template <> struct Store<DT_F16> {
    static constexpr int V = 8;
    static constexpr int ES = 2;
    using acc_t = float;
    __device__ static __forceinline__ float get(const u32x4 &v, int e)
    {
        const uint32_t w = (e >> 1) == 0 ? v.x : ((e >> 1) == 1 ? v.y : ((e >> 1) == 2 ? v.z : v.w));
        const uint16_t h = (e & 1) ? (uint16_t)(w >> 16) : (uint16_t)(w & 0xffffu);
        return (float)__builtin_bit_cast(_Float16, h);   // fp16 -> fp32 is exact
    }
};

// ---------------------------------------------------------------------------------------
// Q-stack pass: out_b[uoff + r] = sum_j Q[r, j] * w_b[j] for the stored rows r of a tile.
// LPR lanes share one row: each lane streams 16-byte vectors of the row (coalesced across
// the group), UNR loads in flight, multiply-adds against w held in LDS, then a butterfly
// reduction over the LPR lanes in FP64.  With FP32 accumulation each lane sums at most
// n / LPR products in FP32 before the FP64 combine.

// Rows per group step (R) and 16-byte loads per batch (UNR) for the trial passes: R rows share
// each w value read from LDS, which cuts LDS traffic by R for the 16/32-bit types (whose w
// reads are 2-4 LDS bytes per streamed byte).  For FP64, R = 2 keeps 16 loads per lane in
// flight, which large n needs: the staged trial points then fill the LDS with one block per CU
// (n = 10000: 5.6 -> 6.35 TB/s measured, no loss at n = 2000 or 4000).
template <int DT> struct PassShape {
    static constexpr int R = DT == DT_F64 ? 2 : 4;
    static constexpr int UNR = DT == DT_F64 ? 8 : 4;
};

template <int DT, typename AT, int B, int LPR, bool NT, int R, int UNR>
__device__ __forceinline__ void pass_rows(const void *__restrict__ Q, int n, size_t ld, int row0,
                                          int nrows, const AT *__restrict__ w, int nw,
                                          double *const (&outs)[B], int uoff)
{
    using T = Store<DT>;
    constexpr int V = T::V;
    constexpr int ES = T::ES;
    constexpr int NG = PASS_BS / LPR;
    constexpr int STRIDE = LPR * V;
    const int lane = threadIdx.x & (LPR - 1);
    const int grp = threadIdx.x / LPR;
    const int rend = row0 + nrows;
    for (int r = row0 + grp * R; r < rend; r += NG * R) {
        size_t base[R];
        bool live[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            live[i] = r + i < rend;
            base[i] = (size_t)(live[i] ? r + i : r) * ld * ES;
        }
        AT acc[R][B];
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int b = 0; b < B; ++b) acc[i][b] = AT(0);
        // batches of R x UNR independent 16-byte loads; the last batch is predicated per lane
        for (int col = lane * V; col < n; col += UNR * STRIDE) {
            u32x4 v[R][UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int c = col + u * STRIDE;
#pragma unroll
                for (int i = 0; i < R; ++i)
                    v[i][u] = (c < n && live[i]) ? ld16<NT>(Q, base[i] + (size_t)c * ES)
                                                 : u32x4{0u, 0u, 0u, 0u};
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int c = col + u * STRIDE;
                if (c < n) {
#pragma unroll
                    for (int e = 0; e < V; ++e) {
                        AT wv[B];
#pragma unroll
                        for (int b = 0; b < B; ++b) wv[b] = w[b * nw + c + e];
#pragma unroll
                        for (int i = 0; i < R; ++i) {
                            const AT qv = (AT)T::get(v[i][u], e);
#pragma unroll
                            for (int b = 0; b < B; ++b) acc[i][b] = fma(qv, wv[b], acc[i][b]);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            double sv[B];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                sv[b] = (double)acc[i][b];
#pragma unroll
                for (int off = LPR / 2; off > 0; off >>= 1) sv[b] += __shfl_xor(sv[b], off, LPR);
            }
            if (lane == 0 && live[i]) {
#pragma unroll
                for (int b = 0; b < B; ++b) outs[b][uoff + r + i] = sv[b];
            }
        }
    }
}

template <int DT, typename AT, int B, bool NT = false, int R = 1, int UNR = 8>
__device__ __forceinline__ void pass_rows_lpr(int lpr, const void *Q, int n, size_t ld, int row0,
                                              int nrows, const AT *w, int nw,
                                              double *const (&outs)[B], int uoff)
{
    if (lpr == 64) pass_rows<DT, AT, B, 64, NT, R, UNR>(Q, n, ld, row0, nrows, w, nw, outs, uoff);
    else if (lpr == 32) pass_rows<DT, AT, B, 32, NT, R, UNR>(Q, n, ld, row0, nrows, w, nw, outs, uoff);
    else if (lpr == 16) pass_rows<DT, AT, B, 16, NT, R, UNR>(Q, n, ld, row0, nrows, w, nw, outs, uoff);
    else pass_rows<DT, AT, B, 8, NT, R, UNR>(Q, n, ld, row0, nrows, w, nw, outs, uoff);
}

// Block b of the pass grid streams the contiguous tile range [starts[b], starts[b+1]), ranges
// of nearly equal bytes; w is staged into LDS when the block starts and again only when the
// tile's slot changes (tiles are grouped by slot).
// anchor_only: streams only for slots in anchor mode (their trial passes run on the packed
// 16-bit stack)
template <int DT, int B, bool NT>
__global__ void __launch_bounds__(PASS_BS) k_pass(Slot *__restrict__ slots,
                                                  const Tile *__restrict__ tiles, int ntiles,
                                                  const int *__restrict__ starts, int anchor_only)
{
    extern __shared__ __align__(16) unsigned char smem[];
    using AT = typename Store<DT>::acc_t;
    const int G = gridDim.x;
    // block b streams tiles [starts[b], starts[b+1]): ranges of nearly equal bytes (or of equal
    // tile counts when no table is given)
    const int t0 = starts ? starts[blockIdx.x] : (int)(((int64_t)blockIdx.x * ntiles) / G);
    const int t1 = starts ? starts[blockIdx.x + 1] : (int)(((int64_t)(blockIdx.x + 1) * ntiles) / G);
    int cur = -1;
    bool active = false, anchor = false, inc = false;
    int n = 0, nw = 0;
    size_t ld = 0;
    const void *Q = nullptr;
    double *outs[B];
#pragma unroll
    for (int b = 0; b < B; ++b) outs[b] = nullptr;
    // the next tile's descriptor is loaded while the current tile streams
    Tile tn = t0 < t1 ? tiles[t0] : Tile{};
    for (int ti = t0; ti < t1; ++ti) {
        const Tile t = tn;
        if (ti + 1 < t1) tn = tiles[ti + 1];
        if (t.slot != cur) {
            __syncthreads();   // every wave is done with the previous slot's w
            cur = t.slot;
            Slot *S = slots + cur;
            active = S->status == ST_RUNNING && (!anchor_only || S->mode == MODE_ANCHOR);
            if (active) {
                anchor = S->mode == MODE_ANCHOR;
                inc = S->incremental != 0;
                n = S->n;
                nw = S->nw;
                ld = (size_t)S->ld;
                Q = S->Q;
                const double *x = S->x;
                // staging loads are batched (SU per thread and vector in flight): every block
                // stages at once when the grid starts, and for large n the one-load-per-round-trip
                // loop held the stream back by up to 14 us
                constexpr int SU = 4;
                if (anchor) {
                    double *w = reinterpret_cast<double *>(smem);
                    for (int j0 = threadIdx.x; j0 < nw; j0 += SU * PASS_BS) {
                        double xv[SU];
#pragma unroll
                        for (int u = 0; u < SU; ++u) {
                            const int j = j0 + u * PASS_BS;
                            xv[u] = j < n ? x[j] : 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < SU; ++u)
                            if (j0 + u * PASS_BS < nw) w[j0 + u * PASS_BS] = xv[u];
                    }
                    outs[0] = S->Uc[0];
                } else {
                    AT *w = reinterpret_cast<AT *>(smem);
                    const double *xcs[B];
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        xcs[b] = S->xc[b];
                        outs[b] = inc ? S->W[b] : S->Uc[b];
                    }
                    for (int j0 = threadIdx.x; j0 < nw; j0 += SU * PASS_BS) {
                        double xv[SU], cv[B][SU];
#pragma unroll
                        for (int u = 0; u < SU; ++u) {
                            const int j = j0 + u * PASS_BS;
                            xv[u] = (inc && j < n) ? x[j] : 0.0;
#pragma unroll
                            for (int b = 0; b < B; ++b) cv[b][u] = j < n ? xcs[b][j] : 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < SU; ++u) {
                            const int j = j0 + u * PASS_BS;
                            if (j < nw) {
#pragma unroll
                                for (int b = 0; b < B; ++b)
                                    w[b * nw + j] = (AT)(inc ? cv[b][u] - xv[u] : cv[b][u]);
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (!active) continue;
        if (anchor) {
            // direct pass at the iterate, accumulated in FP64 whatever the storage type
            double *const o1[1] = {outs[0]};
            pass_rows_lpr<DT, double, 1, NT, PassShape<DT>::R, PassShape<DT>::UNR>(
                t.lpr, Q, n, ld, t.row0, t.nrows, reinterpret_cast<const double *>(smem), nw, o1, t.uoff);
        } else {
            double *const (&co)[B] = outs;
            pass_rows_lpr<DT, AT, B, NT, PassShape<DT>::R, PassShape<DT>::UNR>(
                t.lpr, Q, n, ld, t.row0, t.nrows, reinterpret_cast<const AT *>(smem), nw, co, t.uoff);
        }
    }
}

// plain single-matrix product z = Q_i v (power iteration for the default step size)
template <int DT>
__global__ void __launch_bounds__(PASS_BS) k_matvec1(const void *__restrict__ Q, int n, int ld,
                                                     int row_base, int lpr, int rows_per_block,
                                                     const double *__restrict__ v, int nw,
                                                     double *__restrict__ z)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double *w = reinterpret_cast<double *>(smem);
    for (int j = threadIdx.x; j < nw; j += PASS_BS) w[j] = j < n ? v[j] : 0.0;
    __syncthreads();
    const int r0 = blockIdx.x * rows_per_block;
    const int nr = min(rows_per_block, n - r0);
    if (nr <= 0) return;
    double *const outs[1] = {z - row_base};
    pass_rows_lpr<DT, double, 1>(lpr, Q, n, (size_t)ld, row_base + r0, nr, w, nw, outs, 0);
}

// z = H v (FP64); skipped once the inner loop is done unless force != 0
__global__ void __launch_bounds__(PASS_BS) k_hmv(const double *__restrict__ H, int n, int ldh,
                                                 int lpr, int rows_per_block,
                                                 const double *__restrict__ v, int nw,
                                                 double *__restrict__ z,
                                                 const double *__restrict__ ctl, int force)
{
    if (!force && ctl[3] != 0.0) return;
    extern __shared__ __align__(16) unsigned char smem[];
    double *w = reinterpret_cast<double *>(smem);
    for (int j = threadIdx.x; j < nw; j += PASS_BS) w[j] = j < n ? v[j] : 0.0;
    __syncthreads();
    const int r0 = blockIdx.x * rows_per_block;
    const int nr = min(rows_per_block, n - r0);
    if (nr <= 0) return;
    double *const outs[1] = {z};
    pass_rows_lpr<DT_F64, double, 1>(lpr, H, n, (size_t)ldh, r0, nr, w, nw, outs, 0);
}


int pass_rows_per_step(int dtype)
{
    return dtype == DT_F64 ? PassShape<DT_F64>::R : PassShape<DT_BF16>::R;
}

size_t pass_lds_bytes(int B, int dtype, int max_nw)
{
    const size_t accsz = dtype == DT_F64 ? sizeof(double) : sizeof(float);
    size_t lds = (size_t)max_nw * sizeof(double);
    const size_t trial = (size_t)B * max_nw * accsz;
    return trial > lds ? trial : lds;
}

template <int DT, int B>
static void launch_pass_dt(hipStream_t s, Slot *slots, const Tile *tiles, int ntiles,
                           const int *starts, size_t lds, int grid, int nt, int anchor_only)
{
    if (nt) k_pass<DT, B, true><<<grid, PASS_BS, lds, s>>>(slots, tiles, ntiles, starts, anchor_only);
    else k_pass<DT, B, false><<<grid, PASS_BS, lds, s>>>(slots, tiles, ntiles, starts, anchor_only);
}

template <int B>
static void launch_pass_b(hipStream_t s, Slot *slots, const Tile *tiles, int ntiles,
                          const int *starts, int dtype, int max_nw, int grid, int nt, int anchor_only = 0)
{
    // an anchor-only launch stages the FP64 iterate alone
    const size_t lds = anchor_only ? (size_t)max_nw * sizeof(double) : pass_lds_bytes(B, dtype, max_nw);
    if (grid > ntiles) grid = ntiles;
    if (grid < 1) grid = 1;
    switch (dtype) {
    case DT_F64: launch_pass_dt<DT_F64, B>(s, slots, tiles, ntiles, starts, lds, grid, nt, anchor_only); break;
    case DT_F32: launch_pass_dt<DT_F32, B>(s, slots, tiles, ntiles, starts, lds, grid, nt, anchor_only); break;
    case DT_BF16: launch_pass_dt<DT_BF16, B>(s, slots, tiles, ntiles, starts, lds, grid, nt, anchor_only); break;
    default: launch_pass_dt<DT_F16, B>(s, slots, tiles, ntiles, starts, lds, grid, nt, anchor_only); break;
    }
}

template <int DT, int B>
static int occ_dt(size_t lds)
{
    int a = 0, b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_pass<DT, B, false>, PASS_BS, lds) != hipSuccess) a = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_pass<DT, B, true>, PASS_BS, lds) != hipSuccess) b = 1;
    return a < b ? a : b;
}

template <int B>
static int occ_b(int dtype, size_t lds)
{
    switch (dtype) {
    case DT_F64: return occ_dt<DT_F64, B>(lds);
    case DT_F32: return occ_dt<DT_F32, B>(lds);
    case DT_BF16: return occ_dt<DT_BF16, B>(lds);
    default: return occ_dt<DT_F16, B>(lds);
    }
}

int pass_blocks_per_cu(int B, int dtype, int max_nw)
{
    const size_t lds = pass_lds_bytes(B, dtype, max_nw);
    int o = 1;
    switch (B) {
    case 1: o = occ_b<1>(dtype, lds); break;
    case 2: o = occ_b<2>(dtype, lds); break;
    case 3: o = occ_b<3>(dtype, lds); break;
    default: o = occ_b<4>(dtype, lds); break;
    }
    return o < 1 ? 1 : o;
}

// ---------------------------------------------------------------------------------------
// Packed symmetric pass.  Q_i = Q_i' (the problem class), so the tile Q_IJ of the upper
// triangle also holds Q_JI = Q_IJ'.  Streaming only the tiles I <= J gives every product
// (Q_i w)_r from the row dots of tile row I (J >= I) plus the column dots of tile column I
// (K < I): about half the bytes of the row-major pass.

// (I, J) of the k-th tile of a matrix, tiles ordered row of tiles by row of tiles, J >= I
__device__ __forceinline__ void sym_tile_ij(int k, int NT, int &I, int &J)
{
    int i = 0, base = 0;
    while (base + (NT - i) <= k) {
        base += NT - i;
        ++i;
    }
    I = i;
    J = i + (k - base);
}

__device__ __forceinline__ int sym_tile_index(int s, int I, int J, int NT, int ntt)
{
    return s * ntt + I * NT - I * (I - 1) / 2 + (J - I);
}

__global__ void __launch_bounds__(256) k_sym_pack(const double *__restrict__ Q, int64_t ld, SymPass sp,
                                                  double *__restrict__ P)
{
    const int t = blockIdx.x;
    const int s = t / sp.ntt;
    int I, J;
    sym_tile_ij(t - s * sp.ntt, sp.NT, I, J);
    double *dst = P + (size_t)t * SYM_TILE_STRIDE;
    const double *src = Q + (size_t)s * sp.n * ld;
    // a diagonal tile keeps its upper triangle with half the diagonal: its row dots then give
    // sum_{c >= r} and its column dots sum_{c < r} of (Q_II w)_r, each diagonal entry half in
    // each (halving is exact)
    for (int e = threadIdx.x; e < SYM_T * SYM_T; e += 256) {
        const int r = e / SYM_T, c = e % SYM_T;
        const int gr = I * SYM_T + r, gc = J * SYM_T + c;
        double v = (gr < sp.n && gc < sp.n) ? src[(size_t)gr * ld + gc] : 0.0;
        if (I == J) v = c > r ? v : (c == r ? 0.5 * v : 0.0);
        dst[e] = v;
    }
}

hipError_t launch_sym_pack(hipStream_t s, const double *Q, int64_t ld, const SymPass &sp, double *P)
{
    const int ntiles = sp.nq * sp.ntt;
    if (ntiles > 0) k_sym_pack<<<ntiles, 256, 0, s>>>(Q, ld, sp, P);
    return hipGetLastError();
}

// One tile by one 64-lane wave.  One 16-byte non-temporal buffer load per lane covers two
// doubles, so a load instruction covers half a tile row in each half of the wave: instruction k
// reads row pair p = k / 2 (lanes 0..31 row 2p, lanes 32..63 row 2p + 1) at column half k % 2,
// and lane l holds columns 2 (l mod 32) + {0, 1, 64, 65} of its rows.  The loads run WIN
// instructions ahead of the arithmetic in a rolling window: a group's registers are refilled
// with the instructions WIN further on as soon as the group is consumed, so about WIN KB of the
// tile stay in flight per wave.  The loop over the tile is unrolled at compile time so every
// window slot stays in one register (a rolled loop would copy the slots at its back edge and
// wait there for all loads in flight).
// Row dots: four products per lane, then over the row's 32 lanes by a transposing step that
// pairs two row pairs (one permlane16 swap) and four DPP rotations inside 16-lane rows (VALU
// only); the sums are parked in LDS.  Column dots stay in the lane's registers over the rows of
// its half, multiplied by w_I read from LDS (one broadcast read per half and row, no VALU), and
// the two halves are added once at the end.
// A diagonal tile is stored as its upper triangle with half the diagonal (k_sym_pack), so it
// runs the same code; lanes whose 16 bytes lie wholly below the diagonal fetch nothing.

// Cross-lane steps on doubles, VALU only (no LDS): exchange quarter-waves with the gfx950
// permlane16 swap, and rotate within 16-lane rows with DPP.
__device__ __forceinline__ void swap16(double &a, double &b)
{
    // lanes 16..31 (48..63) of a <-> lanes 0..15 (32..47) of b
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false, false);
    a = __hiloint2double((int)hi[0], (int)lo[0]);
    b = __hiloint2double((int)hi[1], (int)lo[1]);
}

// v of lane (i + K) mod 16 within the lane's 16-lane row
template <int K>
__device__ __forceinline__ double row_ror(double v)
{
    // every row and bank is enabled and a rotation reads no lane outside the row, so every lane
    // is written: no old value is needed (an update form would zero the destination first)
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x120 + K, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x120 + K, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

constexpr int SYM_WIN = 16;   // load instructions in flight per wave (half a row pair each)
constexpr int SYM_GRP = 4;    // instructions (rows) per transposing reduction
constexpr int SYM_WAVES = 3;  // register budget: waves per SIMD

// A buffer resource over the first `bytes` bytes of a tile: loads beyond it return zero without
// touching memory, so every load can be issued unconditionally (which keeps the in-order count
// of outstanding loads exact) and masked entries are fetched from nowhere.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const void *base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, bytes, 0x00020000);
}

constexpr int BUF_NT = 2;              // cache policy of the tile loads: non-temporal
constexpr int OFF_NONE = 0x40000000;   // a byte offset past every tile (load returns zero)

// Calls f(integral_constant<int, G>) for G = G0, G0 + 1, ... while G < GN and G * SYM_GRP < rows:
// a row loop unrolled at compile time, so that every window slot is a fixed register.
template <int G0, int GN>
struct GroupLoop {
    template <typename F>
    __device__ __forceinline__ static void run(F &&f, int rows)
    {
        if constexpr (G0 < GN) {
            if (G0 * SYM_GRP < rows) {
                f(std::integral_constant<int, G0>{});
                GroupLoop<G0 + 1, GN>::run(f, rows);
            }
        }
    }
};

// p0: each lane's share of tile rows 4g (lanes 0..31) and 4g + 1 (lanes 32..63); p1 the same for
// rows 4g + 2 and 4g + 3.  Returns in every lane of 16-lane row q the full sum of tile row
// 4g + {0, 2, 1, 3}[q], in a fixed order (one half-swap, then four rotations inside 16-lane rows)
__device__ __forceinline__ double reduce2d(double p0, double p1)
{
    swap16(p0, p1);
    double t = p0 + p1;
    t += row_ror<8>(t);
    t += row_ror<4>(t);
    t += row_ror<2>(t);
    t += row_ror<1>(t);
    return t;
}

template <int NB>
__device__ __forceinline__ void sym_tile(const double *__restrict__ q, int n, int I, int J,
                                         const double *const (&w)[NB], double *__restrict__ rp,
                                         double *__restrict__ cp, double (*__restrict__ wi)[SYM_T],
                                         double (*__restrict__ rbuf)[SYM_T])
{
    using T = Store<DT_F64>;
    constexpr int NSLOT = SYM_WIN / SYM_GRP;     // groups in flight
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    const int c = 2 * (lane & 31);                // columns c, c + 1 and c + 64, c + 65
    const int gc = J * SYM_T + c;
    const int rmax = min(SYM_T, n - I * SYM_T);
    // the resource spans the tile's valid rows; columns past n take a lane offset outside it
    // (rows past rmax, reached by the window's read-ahead and by the last group of four rows,
    // hold zeros in the packed tile)
    const __amdgpu_buffer_rsrc_t rs = tile_rsrc(q, rmax * SYM_T * 8);
    // instruction k: row pair p = k / 2 (lanes 0..31 row 2p, lanes 32..63 row 2p + 1), column
    // half h = k % 2.  The scalar offset is the pair's first row (uniform); the half's row and the
    // columns go into the lane offset.  On the diagonal tile a lane whose two columns both lie
    // below the diagonal (c_h + 1 < 2p + half, i.e. p >= pd_h) reads nothing.
    int vbase[2], pd[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int ch = c + 64 * h;
        vbase[h] = (J * SYM_T + ch < n ? ch * 8 : OFF_NONE) + half * SYM_T * 8;
        pd[h] = I == J ? (ch + 3 - half) >> 1 : SYM_T;
    }
    auto load = [&](int k) -> u32x4 {
        const int p = k >> 1, h = k & 1;
        const int vo = p >= pd[h] ? OFF_NONE : vbase[h];
        return __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, 2 * p * SYM_T * 8, BUF_NT));
    };
    // w_J at the lane's four columns and w_I at the tile's rows (zero past n); indices past n are
    // clamped, so that the loads are issued unconditionally and go out together
    double xj[NB][4], xi[NB][2];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int e = 0; e < 4; ++e) xj[b][e] = w[b][min(gc + (e & 1) + 64 * (e >> 1), n - 1)];
#pragma unroll
        for (int u = 0; u < 2; ++u) xi[b][u] = w[b][min(I * SYM_T + lane + 64 * u, n - 1)];
    }
    u32x4 v[SYM_WIN];
#pragma unroll
    for (int i = 0; i < SYM_WIN; ++i) v[i] = load(i);
    // (a wave's LDS accesses complete in order: the group loop reads these writes)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (gc + (e & 1) + 64 * (e >> 1) >= n) xj[b][e] = 0.0;
#pragma unroll
        for (int u = 0; u < 2; ++u) wi[b][lane + 64 * u] = lane + 64 * u < rmax ? xi[b][u] : 0.0;
    }
    double ca[NB][4];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) ca[b][e] = 0.0;
    GroupLoop<0, SYM_T / SYM_GRP>::run(
        [&](auto gconst) {
            constexpr int G = decltype(gconst)::value;
            constexpr int s0 = (G % NSLOT) * SYM_GRP;   // the group's window slots
            constexpr int k0 = G * SYM_GRP;             // its first load instruction (rows 4G..)
            __builtin_amdgcn_sched_barrier(0);
            double rp2[2][NB];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const u32x4 lo = v[s0 + 2 * j], hi = v[s0 + 2 * j + 1];   // column halves 0 and 1
                const double q0 = T::get(lo, 0), q1 = T::get(lo, 1), q2 = T::get(hi, 0), q3 = T::get(hi, 1);
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    rp2[j][b] = fma(q3, xj[b][3], fma(q2, xj[b][2], fma(q1, xj[b][1], q0 * xj[b][0])));
                    const double xv = wi[b][k0 + 2 * j + half];   // row 2 (k0 / 2 + j) + half
                    ca[b][0] = fma(q0, xv, ca[b][0]);
                    ca[b][1] = fma(q1, xv, ca[b][1]);
                    ca[b][2] = fma(q2, xv, ca[b][2]);
                    ca[b][3] = fma(q3, xv, ca[b][3]);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            // the group's instructions are consumed: refill its slots with those WIN further on
            // (a tile is SYM_T instructions: 64 row pairs, two column halves each)
            if constexpr (k0 + SYM_WIN < SYM_T) {
#pragma unroll
                for (int i = 0; i < SYM_GRP; ++i) v[s0 + i] = load(k0 + SYM_WIN + i);
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const double t = reduce2d(rp2[0][b], rp2[1][b]);
                // 16-lane row g holds tile row k0 + {0, 2, 1, 3}[g]
                if ((lane & 15) == 0) rbuf[b][k0 + ((lane >> 4) & 1) * 2 + (lane >> 5)] = t;
            }
        },
        rmax);
    __builtin_amdgcn_sched_barrier(0);
    // row results (coalesced; rows past rmax are never read), then the column results: the two
    // halves of the wave (even and odd rows) add in a fixed order (lower half first)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        for (int r = lane; r < rmax; r += 64) rp[b * SYM_T + r] = rbuf[b][r];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double o = __shfl_xor(ca[b][e], 32, 64);
            const int col = c + (e & 1) + 64 * (e >> 1);
            if (half == 0 && J * SYM_T + col < n) cp[b * SYM_T + col] = ca[b][e] + o;
        }
    }
}

template <int B>
__global__ void __launch_bounds__(64, SYM_WAVES) k_spass(Slot *__restrict__ slots, SymPass sp)
{
    __shared__ double wi[B][SYM_T];
    __shared__ double rbuf[B][SYM_T];
    Slot *S = slots;
    if (S->status != ST_RUNNING) return;
    const int t = blockIdx.x;
    const int s = t / sp.ntt;
    int I, J;
    sym_tile_ij(t - s * sp.ntt, sp.NT, I, J);
    const double *q = sp.P + (size_t)t * SYM_TILE_STRIDE;
    double *rp = sp.ws + (size_t)t * 2 * sp.B * SYM_T;
    double *cp = rp + (size_t)sp.B * SYM_T;
    if (S->mode == MODE_ANCHOR) {
        const double *const w1[1] = {S->x};
        sym_tile<1>(q, sp.n, I, J, w1, rp, cp, wi, rbuf);
    } else {
        const double *wb[B];
#pragma unroll
        for (int b = 0; b < B; ++b) wb[b] = S->xc[b];
        sym_tile<B>(q, sp.n, I, J, wb, rp, cp, wi, rbuf);
    }
}

// (Q_s w)_r for the rows of tile row I: the row results of tiles (I, J >= I), then the column
// results of tiles (K <= I, I) (the diagonal tile's column results carry its entries below
// the diagonal), in that order
template <int B>
__global__ void __launch_bounds__(SYM_T) k_sred(Slot *__restrict__ slots, SymPass sp)
{
    Slot *S = slots;
    if (S->status != ST_RUNNING) return;
    const int s = blockIdx.x / sp.NT, I = blockIdx.x % sp.NT;
    const int rr = threadIdx.x, gr = I * SYM_T + rr;
    if (gr >= sp.n) return;
    const bool anchor = S->mode == MODE_ANCHOR;
    const int nb = anchor ? 1 : B;
    const size_t stride = (size_t)2 * sp.B * SYM_T;
    const size_t ob = (size_t)sp.ubase[s] + gr;
    // terms k = 0 .. NT - I - 1: row result of (I, I + k); k = NT - I .. NT: column result of
    // (k - (NT - I), I); eight terms of every candidate are loaded at a time, so that the loads
    // are in flight together; each candidate's sum runs over k in order
    const int nrow = sp.NT - I, nterm = sp.NT + 1;
    double v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = 0.0;
    for (int k0 = 0; k0 < nterm; k0 += 8) {
        double t[B][8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + u;
            const size_t base = k < nrow ? (size_t)sym_tile_index(s, I, I + k, sp.NT, sp.ntt) * stride + rr
                                         : (size_t)sym_tile_index(s, k - nrow, I, sp.NT, sp.ntt) * stride +
                                               (size_t)sp.B * SYM_T + rr;
#pragma unroll
            for (int b = 0; b < B; ++b) t[b][u] = (k < nterm && b < nb) ? sp.ws[base + (size_t)b * SYM_T] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + u < nterm) v[b] += t[b][u];
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
        if (b < nb) {
            double *out = anchor ? S->Uc[0] : S->Uc[b];
            out[ob] = v[b];
        }
    }
}

template <int B>
static void launch_sym_b(hipStream_t s, Slot *slots, const SymPass &sp)
{
    const int ntiles = sp.nq * sp.ntt;
    if (ntiles <= 0) return;
    k_spass<B><<<ntiles, 64, 0, s>>>(slots, sp);
    k_sred<B><<<sp.nq * sp.NT, SYM_T, 0, s>>>(slots, sp);
}

// ---------------------------------------------------------------------------------------
// Packed symmetric pass for 16-bit storage (BF16 / FP16), trial passes of the incremental mode:
// W_b = Q_i d_b, d_b = x_b - x, with FP32 products and sums.  Tiles of SYM16_T x SYM16_T
// elements (128 KB, as the FP64 tiles): one 16-byte load per lane covers 8 elements, so a row
// of the tile is 32 lanes and one load instruction of the wave covers two rows (lanes 0..31 row
// 2k, lanes 32..63 row 2k + 1).  The wave streams the tile's rows in order with SYM16_WIN
// instructions in flight (the rolling window of the FP64 tiles).  Row dots: 8 products per lane,
// then over the row's 32 lanes by a transposing step that pairs two instructions (one permlane16
// swap) and four DPP rotations inside 16-lane rows.  Column dots: each lane keeps its 8 columns
// over the rows of its half of the wave (d_I from LDS), the halves are added at the end.  Results
// are FP32 per tile; k_sred16 adds them per output row in FP64 in a fixed order.

constexpr int SYM16_WIN = 16;  // load instructions in flight per wave (2 rows each)
constexpr int SYM16_GRP = 2;   // instructions per transposing reduction (4 rows)

__global__ void __launch_bounds__(256) k_sym_pack16(const uint16_t *__restrict__ Q, int64_t ld, int dt,
                                                    SymPass sp, uint16_t *__restrict__ P,
                                                    unsigned *__restrict__ inexact)
{
    const int t = blockIdx.x;
    const int s = t / sp.ntt;
    int I, J;
    sym_tile_ij(t - s * sp.ntt, sp.NT, I, J);
    uint16_t *dst = P + (size_t)t * SYM16_TILE;
    const uint16_t *src = Q + (size_t)s * sp.n * ld;
    // a diagonal tile keeps its upper triangle with half the diagonal (exact unless the half
    // would be subnormal in the storage type, which is flagged)
    for (int e = threadIdx.x; e < SYM16_TILE; e += 256) {
        const int r = e / SYM16_T, c = e % SYM16_T;
        const int gr = I * SYM16_T + r, gc = J * SYM16_T + c;
        uint16_t v = (gr < sp.n && gc < sp.n) ? src[(size_t)gr * ld + gc] : (uint16_t)0;
        if (I == J) {
            if (c < r) {
                v = 0;
            } else if (c == r) {
                float f = dt == DT_BF16 ? __uint_as_float((uint32_t)v << 16)
                                        : (float)__builtin_bit_cast(_Float16, v);
                const float h = 0.5f * f;
                uint16_t hv;
                if (dt == DT_BF16) {
                    hv = (uint16_t)(__float_as_uint(h) >> 16);
                    if (__uint_as_float((uint32_t)hv << 16) != h) atomicOr(inexact, 1u);
                } else {
                    const _Float16 hh = (_Float16)h;
                    hv = __builtin_bit_cast(uint16_t, hh);
                    if ((float)hh != h) atomicOr(inexact, 1u);
                }
                v = hv;
            }
        }
        dst[e] = v;
    }
}

hipError_t launch_sym_pack16(hipStream_t s, const void *Q, int64_t ld, int dt, const SymPass &sp, void *P,
                             unsigned *inexact)
{
    const int ntiles = sp.nq * sp.ntt;
    if (ntiles > 0)
        k_sym_pack16<<<ntiles, 256, 0, s>>>(static_cast<const uint16_t *>(Q), ld, dt, sp,
                                            static_cast<uint16_t *>(P), inexact);
    return hipGetLastError();
}

__device__ __forceinline__ void swap16f(float &a, float &b)
{
    // lanes 16..31 (48..63) of a <-> lanes 0..15 (32..47) of b
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}

template <int K>
__device__ __forceinline__ float row_rorf(float v)
{
    // (the update form lets the compiler fold the rotation into the following add)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + K, 0xf, 0xf, false));
}

// p0: each lane's share of rows 2k (lanes 0..31) and 2k+1 (lanes 32..63); p1 the same for
// instruction k+1.  Returns in every lane of 16-lane row q the full sum of tile row
// 2k + {0, 2, 1, 3}[q] (lanes 0..15: row 2k, 16..31: 2k+2, 32..47: 2k+1, 48..63: 2k+3)
__device__ __forceinline__ float reduce2f(float p0, float p1)
{
    swap16f(p0, p1);
    float t = p0 + p1;
    t += row_rorf<8>(t);
    t += row_rorf<4>(t);
    t += row_rorf<2>(t);
    t += row_rorf<1>(t);
    return t;
}

// Calls f(integral_constant<int, G>) for G = G0, G0 + 1, ... while G < GN and
// G * 2 * SYM16_GRP < rows (4 rows per group)
template <int G0, int GN>
struct Group16Loop {
    template <typename F>
    __device__ __forceinline__ static void run(F &&f, int rows)
    {
        if constexpr (G0 < GN) {
            if (G0 * 2 * SYM16_GRP < rows) {
                f(std::integral_constant<int, G0>{});
                Group16Loop<G0 + 1, GN>::run(f, rows);
            }
        }
    }
};

template <int DT, int NB>
__device__ __forceinline__ void sym16_tile(const uint16_t *__restrict__ q, int n, int I, int J,
                                           const double *const (&xc)[NB], const double *__restrict__ x,
                                           float *__restrict__ res, int Bw, float (*__restrict__ wi)[SYM16_T],
                                           float (*__restrict__ rbuf)[SYM16_T])
{
    using T = Store<DT>;
    // four candidates take more registers per group: a shorter window keeps 3 waves per SIMD
    constexpr int WIN = NB >= 4 ? 12 : SYM16_WIN;
    constexpr int NSLOT = WIN / SYM16_GRP;          // groups in flight
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    const int c8 = (lane & 31) * 8;
    const int gc = J * SYM16_T + c8;
    const int rmax = min(SYM16_T, n - I * SYM16_T);
    const __amdgpu_buffer_rsrc_t rs = tile_rsrc(q, rmax * SYM16_T * 2);
    const int voff = gc < n ? c8 * 2 : OFF_NONE;
    const int dmask = I == J ? OFF_NONE : 0;
    // row r of the tile in this lane's half; on the diagonal tile a lane whose eight columns
    // all lie below the diagonal (c8 + 7 < r) reads nothing (the packed tile holds zeros there).
    // The scalar offset is the wave's first row 2k (uniform); the half's row goes into the lane
    // offset, so that the load is one instruction for the whole wave (a lane-dependent scalar
    // offset would be issued once per distinct value).
    const int hoff = half * SYM16_T * 2;
    auto load = [&](int k) -> u32x4 {
        const int r = 2 * k + half;
        const int vo = (voff | (dmask & ((c8 + 7 - r) >> 31))) + hoff;
        return __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, 2 * k * SYM16_T * 2, BUF_NT));
    };
    // d_J of the lane's eight columns and d_I of the tile's rows (FP32 of the FP64 differences,
    // zero past n): the loads go out before the window and are converted behind it, so the first
    // group waits for them and the first rows only (with three or more candidates they are
    // converted before the window, which keeps the registers within the occupancy budget).
    // Indices past n are clamped, so that every load is issued unconditionally; their values
    // are then replaced by zero.
    double xi[SYM16_T / 64], ci[NB][SYM16_T / 64];
    float dj[NB][8];
    double xj[NB <= 2 ? 8 : 1], cj[NB <= 2 ? NB : 1][NB <= 2 ? 8 : 1];
    auto convert_dj = [&]() {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int e = 0; e < 8; ++e) dj[b][e] = gc + e < n ? (float)(cj[b][e] - xj[e]) : 0.0f;
    };
    if constexpr (NB <= 2) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int j = min(gc + e, n - 1);
            xj[e] = x[j];
#pragma unroll
            for (int b = 0; b < NB; ++b) cj[b][e] = xc[b][j];
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int j = min(gc + e, n - 1);
            const double xv = x[j];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float d = (float)(xc[b][j] - xv);
                dj[b][e] = gc + e < n ? d : 0.0f;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < SYM16_T / 64; ++u) {
        const int gr = min(I * SYM16_T + lane + 64 * u, n - 1);
        xi[u] = x[gr];
#pragma unroll
        for (int b = 0; b < NB; ++b) ci[b][u] = xc[b][gr];
    }
    // (a wave's LDS accesses complete in order: the group loop reads these writes)
    auto store_di = [&]() {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int u = 0; u < SYM16_T / 64; ++u)
                wi[b][lane + 64 * u] = lane + 64 * u < rmax ? (float)(ci[b][u] - xi[u]) : 0.0f;
    };
    if constexpr (NB > 2) store_di();
    u32x4 v[WIN];
#pragma unroll
    for (int i = 0; i < WIN; ++i) v[i] = load(i);
    if constexpr (NB <= 2) {
        convert_dj();
        store_di();
    }
    (void)convert_dj;
    float ca[NB][8];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int e = 0; e < 8; ++e) ca[b][e] = 0.0f;
    Group16Loop<0, SYM16_T / (2 * SYM16_GRP)>::run(
        [&](auto gconst) {
            constexpr int G = decltype(gconst)::value;
            constexpr int s0 = (G % NSLOT) * SYM16_GRP;   // the group's window slots
            constexpr int k0 = G * SYM16_GRP;             // its first load instruction
            __builtin_amdgcn_sched_barrier(0);
            float rp[SYM16_GRP][NB];
#pragma unroll
            for (int i = 0; i < SYM16_GRP; ++i) {
                float qv[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) qv[e] = T::get(v[s0 + i], e);
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    float a = qv[0] * dj[b][0];
#pragma unroll
                    for (int e = 1; e < 8; ++e) a = fmaf(qv[e], dj[b][e], a);
                    rp[i][b] = a;
                    const float dv = wi[b][2 * (k0 + i) + half];
#pragma unroll
                    for (int e = 0; e < 8; ++e) ca[b][e] = fmaf(qv[e], dv, ca[b][e]);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            // the group's rows are consumed: refill its slots with the instructions WIN ahead
            if constexpr (2 * (k0 + WIN) < SYM16_T) {
#pragma unroll
                for (int i = 0; i < SYM16_GRP; ++i) v[s0 + i] = load(k0 + WIN + i);
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float t = reduce2f(rp[0][b], rp[1][b]);
                // 16-lane row g holds tile row 2 k0 + {0, 2, 1, 3}[g]
                if ((lane & 15) == 0) rbuf[b][2 * k0 + ((lane >> 4) & 1) * 2 + (lane >> 5)] = t;
            }
        },
        rmax);
    __builtin_amdgcn_sched_barrier(0);
    // row results (rows past rmax are never read), then the column results: the two halves of
    // the wave add in a fixed order (lower half first)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int u = 0; u < SYM16_T / 64; ++u) res[b * SYM16_T + lane + 64 * u] = rbuf[b][lane + 64 * u];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float o = __shfl_xor(ca[b][e], 32, 64);
            if (half == 0) res[(size_t)(Bw + b) * SYM16_T + c8 + e] = ca[b][e] + o;
        }
    }
}

template <int DT, int B>
__global__ void __launch_bounds__(64, SYM_WAVES) k_spass16(Slot *__restrict__ slots,
                                                         const SymPass *__restrict__ descs,
                                                         const int2 *__restrict__ work)
{
    __shared__ float wi[B][SYM16_T];
    __shared__ float rbuf[B][SYM16_T];
    int si = 0, t = blockIdx.x;
    if (work) {
        const int2 w = work[blockIdx.x];
        si = w.x;
        t = w.y;
    }
    Slot *S = slots + si;
    if (S->status != ST_RUNNING || S->mode != MODE_TRIAL) return;
    const SymPass &sp = descs[si];
    const int s = t / sp.ntt;
    int I, J;
    sym_tile_ij(t - s * sp.ntt, sp.NT, I, J);
    const uint16_t *q = sp.P16 + (size_t)t * SYM16_TILE;
    float *res = sp.ws16 + (size_t)t * 2 * sp.B * SYM16_T;
    const double *xc[B];
#pragma unroll
    for (int b = 0; b < B; ++b) xc[b] = S->xc[b];
    sym16_tile<DT, B>(q, sp.n, I, J, xc, S->x, res, sp.B, wi, rbuf);
}

// W_b rows of tile row I of stored matrix s: the row results of tiles (I, J >= I), then the column
// results of tiles (K <= I, I), each converted to FP64 and added in that order
template <int B>
__global__ void __launch_bounds__(SYM16_T) k_sred16(Slot *__restrict__ slots, const SymPass *__restrict__ descs,
                                                    const int2 *__restrict__ work_r)
{
    int si = 0, k = blockIdx.x;
    if (work_r) {
        const int2 w = work_r[blockIdx.x];
        si = w.x;
        k = w.y;
    }
    Slot *S = slots + si;
    if (S->status != ST_RUNNING || S->mode != MODE_TRIAL) return;
    const SymPass &sp = descs[si];
    const int s = k / sp.NT, I = k % sp.NT;
    const int rr = threadIdx.x, gr = I * SYM16_T + rr;
    if (gr >= sp.n) return;
    const size_t stride = (size_t)2 * sp.B * SYM16_T;
    const size_t ob = (size_t)sp.ubase[s] + gr;
    const int nrow = sp.NT - I, nterm = sp.NT + 1;
    // eight terms of every candidate at a time (loads in flight together), each candidate's sum
    // over k in order
    double v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = 0.0;
    for (int k0 = 0; k0 < nterm; k0 += 8) {
        float t[B][8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + u;
            const size_t base = k < nrow ? (size_t)sym_tile_index(s, I, I + k, sp.NT, sp.ntt) * stride + rr
                                         : (size_t)sym_tile_index(s, k - nrow, I, sp.NT, sp.ntt) * stride +
                                               (size_t)sp.B * SYM16_T + rr;
#pragma unroll
            for (int b = 0; b < B; ++b) t[b][u] = k < nterm ? sp.ws16[base + (size_t)b * SYM16_T] : 0.0f;
        }
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + u < nterm) v[b] += (double)t[b][u];
    }
#pragma unroll
    for (int b = 0; b < B; ++b) S->W[b][ob] = v[b];
}

template <int DT, int B>
static void launch_sym16_dt(hipStream_t s, Slot *slots, const Sym16Launch &l)
{
    if (l.nwork > 0) k_spass16<DT, B><<<l.nwork, 64, 0, s>>>(slots, l.descs, l.work);
    if (l.nwork_r > 0) k_sred16<B><<<l.nwork_r, SYM16_T, 0, s>>>(slots, l.descs, l.work_r);
}

template <int B>
static void launch_sym16_b(hipStream_t s, Slot *slots, const Sym16Launch &l)
{
    if (l.dt == DT_BF16) launch_sym16_dt<DT_BF16, B>(s, slots, l);
    else launch_sym16_dt<DT_F16, B>(s, slots, l);
}

template <int B>
static void launch_pass16_b(hipStream_t s, Slot *slots, const Tile *tiles, int ntiles, const int *starts,
                            int dtype, int max_nw, int pass_grid, int nt, const Sym16Launch &l)
{
    if (!l.tiles) {
        // a single solve: every tile belongs to the packed slot, streamed for its anchors only
        launch_pass_b<B>(s, slots, tiles, ntiles, starts, dtype, max_nw, pass_grid, nt, 1);
    } else {
        // a batch: the row-major slots' tiles, then the packed slots' tiles for their anchors
        if (ntiles > 0) launch_pass_b<B>(s, slots, tiles, ntiles, starts, dtype, max_nw, pass_grid, nt, 0);
        if (l.ntiles > 0) launch_pass_b<B>(s, slots, l.tiles, l.ntiles, l.starts, dtype, max_nw, l.grid, nt, 1);
    }
    launch_sym16_b<B>(s, slots, l);
}

hipError_t launch_pass_only(hipStream_t s, Slot *slots, const Tile *tiles, int ntiles,
                            const int *starts, int B, int dtype, int max_nw, int pass_grid, int nt,
                            const SymPass *sym, const Sym16Launch *s16)
{
    if (s16) {
        // 16-bit packed slots: anchors (exact FP64 accumulation at the iterate) stream the
        // row-major stack, the trial passes the packed tiles
        switch (B) {
        case 1: launch_pass16_b<1>(s, slots, tiles, ntiles, starts, dtype, max_nw, pass_grid, nt, *s16); break;
        case 2: launch_pass16_b<2>(s, slots, tiles, ntiles, starts, dtype, max_nw, pass_grid, nt, *s16); break;
        case 3: launch_pass16_b<3>(s, slots, tiles, ntiles, starts, dtype, max_nw, pass_grid, nt, *s16); break;
        default: launch_pass16_b<4>(s, slots, tiles, ntiles, starts, dtype, max_nw, pass_grid, nt, *s16); break;
        }
        return hipGetLastError();
    }
    if (sym) {
        switch (B) {
        case 1: launch_sym_b<1>(s, slots, *sym); break;
        case 2: launch_sym_b<2>(s, slots, *sym); break;
        case 3: launch_sym_b<3>(s, slots, *sym); break;
        default: launch_sym_b<4>(s, slots, *sym); break;
        }
        return hipGetLastError();
    }
    switch (B) {
    case 1: launch_pass_b<1>(s, slots, tiles, ntiles, starts, dtype, max_nw, pass_grid, nt); break;
    case 2: launch_pass_b<2>(s, slots, tiles, ntiles, starts, dtype, max_nw, pass_grid, nt); break;
    case 3: launch_pass_b<3>(s, slots, tiles, ntiles, starts, dtype, max_nw, pass_grid, nt); break;
    default: launch_pass_b<4>(s, slots, tiles, ntiles, starts, dtype, max_nw, pass_grid, nt); break;
    }
    return hipGetLastError();
}

hipError_t launch_matvec1(hipStream_t s, const void *Q, int dtype, int n, int ld, int row_base,
                          const double *v, int nw, double *z)
{
    const int vec = dtype == DT_F64 ? 2 : (dtype == DT_F32 ? 4 : 8);
    const int vpr = (n + vec - 1) / vec;
    int lpr = 16;
    if (vpr >= 4 * 64) lpr = 64;
    else if (vpr >= 4 * 32) lpr = 32;
    const int rows_per_block = 32;
    const int nblk = (n + rows_per_block - 1) / rows_per_block;
    const size_t lds = (size_t)nw * sizeof(double);
    switch (dtype) {
    case DT_F64: k_matvec1<DT_F64><<<nblk, PASS_BS, lds, s>>>(Q, n, ld, row_base, lpr, rows_per_block, v, nw, z); break;
    case DT_F32: k_matvec1<DT_F32><<<nblk, PASS_BS, lds, s>>>(Q, n, ld, row_base, lpr, rows_per_block, v, nw, z); break;
    case DT_BF16: k_matvec1<DT_BF16><<<nblk, PASS_BS, lds, s>>>(Q, n, ld, row_base, lpr, rows_per_block, v, nw, z); break;
    default: k_matvec1<DT_F16><<<nblk, PASS_BS, lds, s>>>(Q, n, ld, row_base, lpr, rows_per_block, v, nw, z); break;
    }
    return hipGetLastError();
}

static void hmv_shape(int n, int *lpr, int *rpb)
{
    const int vpr = (n + 1) / 2;
    int l = 16;
    if (vpr >= 4 * 64) l = 64;
    else if (vpr >= 4 * 32) l = 32;
    *lpr = l;
    *rpb = 32;
}

hipError_t launch_hmv(hipStream_t s, const double *H, int n, int ldh, const double *v, int nw,
                      double *z, const double *ctl, int force)
{
    int lpr, rpb;
    hmv_shape(n, &lpr, &rpb);
    const int nblk_r = (n + rpb - 1) / rpb;
    k_hmv<<<nblk_r, PASS_BS, (size_t)nw * sizeof(double), s>>>(H, n, ldh, lpr, rpb, v, nw, z, ctl, force);
    return hipGetLastError();
}

template <int DT, int B>
static hipError_t set_attr_one(int max_lds)
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_pass<DT, B, false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_pass<DT, B, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    return e;
}

hipError_t prepare_kernels(int max_lds)
{
    hipError_t e = hipSuccess;
#define QCQP_ATTR(DT)                                    \
    if (e == hipSuccess) e = set_attr_one<DT, 1>(max_lds);      \
    if (e == hipSuccess) e = set_attr_one<DT, 2>(max_lds);      \
    if (e == hipSuccess) e = set_attr_one<DT, 3>(max_lds);      \
    if (e == hipSuccess) e = set_attr_one<DT, 4>(max_lds);
    QCQP_ATTR(DT_F64)
    QCQP_ATTR(DT_F32)
    QCQP_ATTR(DT_BF16)
    QCQP_ATTR(DT_F16)
#undef QCQP_ATTR
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_hmv),
                                hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_matvec1<DT_F64>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_matvec1<DT_F32>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_matvec1<DT_BF16>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_matvec1<DT_F16>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    return e;
}

}  // namespace qcqp
