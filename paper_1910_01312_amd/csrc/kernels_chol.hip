// Blocked fp64 Cholesky of a symmetric positive definite Newton matrix (the
// q x q M = I + sigma (X_J^T X_J - s s^T / p) of the linear path, the p x p
// I + sigma Pi Q_JJ Pi of the kernel path, K_rr + s I of the Nystroem map)
// above the LDS-resident kernel's limit, and the two triangular solves
// giving d = -M^{-1} g.  Right-looking with 64 x 64 blocks: for each block
// column kb, factor the diagonal block and form the inverse of its factor,
// compute the panel below it as A_panel L_kk^{-T} (a small GEMM), and update
// the trailing lower tiles (on the matrix cores, grouped so that the
// trailing matrix is rewritten once per eight block columns).  The factor is kept in the lower triangle of M
// and mirrored into the upper triangle (M[j][i] = L[i][j]), so that both
// triangular solves read it with consecutive lanes on consecutive addresses;
// the inverses of the diagonal factors turn the block solves into mat-vecs.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

constexpr int NB = 64;
constexpr int CHOL_BLOCKED_MAX = 2048;
constexpr int SOLVE_THREADS = 512;                  // 8 waves: 64 rows x 8 column groups
constexpr int SOLVE_PARTS = SOLVE_THREADS / NB;
constexpr int TILE_PER_THREAD = NB * NB / SSN_BLOCK;
constexpr int SOLVE_CHUNK = 16;                     // column loads in flight per thread

int chol_blocked_max() { return CHOL_BLOCKED_MAX; }
// per 64 x 64 diagonal block: its inverse factor X = L_kk^{-1} row-major and X^T
int64_t chol_inv_size(int64_t q) { return (q + NB - 1) / NB * 2 * NB * NB; }

// Factor diagonal block kb and form X = L_kk^{-1}, both right-looking in
// registers: thread t keeps row i = t % 64, columns 8 (t / 64) .. +7 of the
// block (a), and column j = t % 64, rows 8 (t / 64) .. +7 of B (initially
// I), so that each thread finds B[k][j] in its own column; B becomes X by
// forward substitution of L X = I carried along with the factorisation.  A
// non-positive pivot is replaced by 1 and reported in sc->chol_fail; rows
// past q are padded with the identity.  Eight waves, four columns per step,
// two barriers per step.  Step k0 = 4K:
//   1. the column group holding columns k0..k0+3 publishes them (raw values);
//   2. every thread factors the 4 x 4 diagonal block D = A[k0..+3][k0..+3]
//      itself (pivot reciprocal square roots from the hardware estimate and
//      two Newton steps) and computes its own row's entries of L in the four
//      columns, l_ic = (a_ic - sum_{m<c} l_im l_cm) / l_cc; wave 0 publishes
//      them for the rows past the block (zero for the rows up to k0 + 3), and
//      the owner group finishes rows k0..k0+3 of X = L^{-1} by forward
//      substitution with the 4 x 4 factor, published too;
//   3. a_ij -= sum_c l_ic l_jc for all the thread's columns j, and
//      B[j][i] -= sum_c l_jc X[k0+c][i] for all its rows j: the zero rows of
//      the published L leave the finished columns and rows as they are, so the
//      update runs without a branch per column (with one, 12 to 20% slower).
// The published buffers alternate between steps, so the next step's writes
// never meet this step's reads.
constexpr int DIAG_WAVES = 8;
constexpr int DIAG_THREADS = DIAG_WAVES * SSN_WAVE;
constexpr int DIAG_CPT = NB / DIAG_WAVES;     // columns of a (rows of B) per thread
__global__ __launch_bounds__(DIAG_THREADS) void k_chol_diag(double* __restrict__ M, int q, int kb,
                                                          double* __restrict__ inv, Scalars* sc) {
    __shared__ double raw[2][4][NB];
    __shared__ double Lc[2][NB][4];      // row-major: the four entries of a row together
    __shared__ double Bf[2][4][NB];
    const int tid = threadIdx.x;
    if (kb == 0 && tid == 0) sc->chol_fail = 0;
    const int o = kb * NB;
    const int m = min(NB, q - o);
    const int i = tid & (NB - 1), cg = tid >> 6;
    double a[DIAG_CPT], b[DIAG_CPT];      // a: A[i][8 cg + jj];  b: B[8 cg + jj][i]
#pragma unroll
    for (int jj = 0; jj < DIAG_CPT; ++jj) {
        const int j = cg * DIAG_CPT + jj;
        a[jj] = (i < m && j < m) ? M[(int64_t)(o + i) * q + o + j] : (i == j ? 1.0 : 0.0);
        b[jj] = i == j ? 1.0 : 0.0;
    }
    const int cgu = __builtin_amdgcn_readfirstlane(cg);
    bool bad = false;
#pragma unroll 1
    for (int kg = 0; kg < DIAG_WAVES; ++kg)
#pragma unroll
    for (int c0 = 0; c0 < DIAG_CPT; c0 += 4) {
        const int k0 = kg * DIAG_CPT + c0;
        const int par = (c0 >> 2) & 1;
        // 1. publish the four raw columns
        if (cgu == kg) {
#pragma unroll
            for (int c = 0; c < 4; ++c) raw[par][c][i] = a[c0 + c];
        }
        __syncthreads();
        // 2. the 4 x 4 factor (every thread), this row's L entries
        double d[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c <= r; ++c) d[r][c] = raw[par][c][k0 + r];
        double l4[4][4], rl[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double piv = d[c][c];
#pragma unroll
            for (int mm = 0; mm < c; ++mm) piv = fma(-l4[c][mm], l4[c][mm], piv);
            if (!(piv > 0.0)) {
                bad = true;
                piv = 1.0;
            }
            double r0 = __builtin_amdgcn_rsq(piv);
            r0 = r0 * fma(-0.5 * piv * r0, r0, 1.5);
            r0 = r0 * fma(-0.5 * piv * r0, r0, 1.5);
            rl[c] = r0;
            l4[c][c] = piv * r0;
#pragma unroll
            for (int r = c + 1; r < 4; ++r) {
                double v = d[r][c];
#pragma unroll
                for (int mm = 0; mm < c; ++mm) v = fma(-l4[r][mm], l4[c][mm], v);
                l4[r][c] = v * r0;
            }
        }
        double li[4];
        {
            double ar[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) ar[c] = raw[par][c][i];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double v = ar[c];
#pragma unroll
                for (int mm = 0; mm < c; ++mm) v = fma(-li[mm], l4[c][mm], v);
                // rows above k0 + c have no entry in column k0 + c
                li[c] = i > k0 + c ? v * rl[c] : (i == k0 + c ? l4[c][c] : 0.0);
            }
        }
        if (cgu == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) Lc[par][i][c] = i > k0 + 3 ? li[c] : 0.0;
        }
        if (cgu == kg) {
            // rows k0..k0+3 of X: forward substitution with the 4 x 4 factor in column i
            double x[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double v = b[c0 + c];
#pragma unroll
                for (int mm = 0; mm < c; ++mm) v = fma(-l4[c][mm], x[mm], v);
                x[c] = v * rl[c];
                b[c0 + c] = x[c];
                Bf[par][c][i] = x[c];
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) a[c0 + c] = li[c];
        }
        __syncthreads();
        // 3. rank-4 updates of the later columns and of the later rows of B
        if (cgu * DIAG_CPT + DIAG_CPT - 1 > k0 + 3) {
            double bx[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) bx[c] = Bf[par][c][i];
#pragma unroll
            for (int jj = 0; jj < DIAG_CPT; ++jj) {
                const int j = cgu * DIAG_CPT + jj;
                {
                    double lj[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) lj[c] = Lc[par][j][c];
                    double av = a[jj], bv = b[jj];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        av = fma(-li[c], lj[c], av);       // a_ij -= l_ic l_jc
                        bv = fma(-lj[c], bx[c], bv);       // B[j][i] -= l_jc X[k0+c][i]
                    }
                    a[jj] = av;
                    b[jj] = bv;
                }
            }
        }
    }
    if (bad && tid == 0) sc->chol_fail = 1;
    double* Xo = inv + (int64_t)kb * 2 * NB * NB;
    double* XTo = Xo + NB * NB;
#pragma unroll
    for (int jj = 0; jj < DIAG_CPT; ++jj) {
        const int j = cg * DIAG_CPT + jj;
        if (j <= i && i < m) {
            M[(int64_t)(o + i) * q + o + j] = a[jj];
            M[(int64_t)(o + j) * q + o + i] = a[jj];
        }
        const double x = i <= j ? b[jj] : 0.0;
        Xo[j * NB + i] = x;
        XTo[i * NB + j] = x;
    }
}

typedef double f64x4_t __attribute__((ext_vector_type(4)));

// Panel below block kb: L_ib,kb = A_ib,kb X^T, X = L_kb,kb^{-1}, for the
// 64-row block ib = kb + 1 + blockIdx.x, on the matrix cores
// (v_mfma_f64_16x16x4f64, each wave a 32 x 32 quarter as 2 x 2 tiles, the
// lane layout of the trailing update below: operand B[k][j] = X[j][k] read
// from the rows of X), written to the lower part and its upper mirror.
__global__ __launch_bounds__(SSN_BLOCK) void k_chol_panel(double* __restrict__ M, int q, int kb,
                                                          const double* __restrict__ inv) {
    __shared__ double Ap[NB][NB + 1];
    __shared__ double Xs[NB][NB + 1];
    const int o = kb * NB;
    const int m = min(NB, q - o);
    const int ro = (kb + 1 + blockIdx.x) * NB;
    const int rm = min(NB, q - ro);
    const double* Xo = inv + (int64_t)kb * 2 * NB * NB;
    {
        // all global loads of the tile first, then the LDS stores
        double va[TILE_PER_THREAD], vx[TILE_PER_THREAD];
#pragma unroll
        for (int h = 0; h < TILE_PER_THREAD; ++h) {
            const int e = threadIdx.x + h * SSN_BLOCK, a = e / NB, b = e % NB;
            va[h] = (a < rm && b < m) ? M[(int64_t)(ro + a) * q + o + b] : 0.0;
            vx[h] = Xo[e];
        }
#pragma unroll
        for (int h = 0; h < TILE_PER_THREAD; ++h) {
            const int e = threadIdx.x + h * SSN_BLOCK, a = e / NB, b = e % NB;
            Ap[a][b] = va[h];
            Xs[a][b] = vx[h];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int r16 = lane & 15, k4 = lane >> 4;
    f64x4_t acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = f64x4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int kk = 0; kk < NB; kk += 4) {
        const double a0 = Ap[wr + r16][kk + k4], a1 = Ap[wr + 16 + r16][kk + k4];
        const double b0 = Xs[wc + r16][kk + k4], b1 = Xs[wc + 16 + r16][kk + k4];   // X[j][k], zero for k > j
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = wr + 16 * u + 4 * e + k4, j = wc + 16 * v + r16;
                if (r < rm && j < m) {
                    M[(int64_t)(ro + r) * q + o + j] = acc[u][v][e];
                    M[(int64_t)(o + j) * q + ro + r] = acc[u][v][e];
                }
            }
}

// Trailing updates on the matrix cores (v_mfma_f64_16x16x4f64):
//   A_ib,jb -= sum over k-blocks kb in [k0, k1) of L_ib,kb L_jb,kb^T
// for the lower tiles jb in [j0, j1), ib in [jb, nblk) (grid x: ib - j0,
// y: jb - j0; blocks above the diagonal return).  The k-blocks are staged in
// LDS one at a time and accumulated in registers, so a tile is read and
// written once per launch whatever the number of k-blocks.  Each wave owns a
// 32 x 32 quarter of the 64 x 64 tile (2 x 2 MFMA tiles) and runs each
// 64-long contraction in 16 steps of 4; lane l supplies row l % 16, column
// l / 16 of the 16 x 4 operand from Li (rows of block ib) and likewise of the
// 4 x 16 operand from Lj (rows of block jb, i.e. L_jb^T), and holds rows
// 4 v + l / 16 (v = 0..3), column l % 16 of the 16 x 16 result.  The next
// k-block's tiles are loaded while the current one's products run, and the
// destination tile's entries at the start, so that no load is waited for at
// the end.
__global__ __launch_bounds__(SSN_BLOCK) void k_chol_update_mfma(double* __restrict__ M, int q, int k0,
                                                                int k1, int j0) {
    __shared__ double Li[NB][NB + 1];
    __shared__ double Lj[NB][NB + 1];
    const int ib = j0 + (int)blockIdx.x, jb = j0 + (int)blockIdx.y;
    if (ib < jb) return;
    const int io = ib * NB, jo = jb * NB;
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int r16 = lane & 15, k4 = lane >> 4;
    f64x4_t acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = f64x4_t{0.0, 0.0, 0.0, 0.0};
    // this thread's entries of the destination tile, loaded now so that the
    // final update does not wait for them (the tile is no operand of this
    // launch and no other workgroup writes it)
    double dst[2][2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = io + wr + 16 * u + 4 * e + k4, j = jo + wc + 16 * v + r16;
                dst[u][v][e] = (i < q && j < q && j <= i) ? M[(int64_t)i * q + j] : 0.0;
            }
    // the tiles of block column kb into registers; the next block column's
    // loads are issued before this one's products, so that they are in
    // flight while the matrix cores work
    double vi[TILE_PER_THREAD], vj[TILE_PER_THREAD];
    auto load_tiles = [&](int kb) {
        const int o = kb * NB;
        const int m = min(NB, q - o);
#pragma unroll
        for (int h = 0; h < TILE_PER_THREAD; ++h) {
            const int e = threadIdx.x + h * SSN_BLOCK, i = e / NB, k = e % NB;
            vi[h] = (io + i < q && k < m) ? M[(int64_t)(io + i) * q + o + k] : 0.0;
            vj[h] = (jo + i < q && k < m) ? M[(int64_t)(jo + i) * q + o + k] : 0.0;
        }
    };
    load_tiles(k0);
    for (int kb = k0; kb < k1; ++kb) {
        if (kb > k0) __syncthreads();            // the previous k-block's reads are done
#pragma unroll
        for (int h = 0; h < TILE_PER_THREAD; ++h) {
            const int e = threadIdx.x + h * SSN_BLOCK, i = e / NB, k = e % NB;
            Li[i][k] = vi[h];
            Lj[i][k] = vj[h];
        }
        __syncthreads();
        if (kb + 1 < k1) load_tiles(kb + 1);
#pragma unroll 4
        for (int kk = 0; kk < NB; kk += 4) {
            const double a0 = Li[wr + r16][kk + k4], a1 = Li[wr + 16 + r16][kk + k4];
            const double b0 = Lj[wc + r16][kk + k4], b1 = Lj[wc + 16 + r16][kk + k4];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = io + wr + 16 * u + 4 * e + k4, j = jo + wc + 16 * v + r16;
                if (i < q && j < q && j <= i) M[(int64_t)i * q + j] = dst[u][v][e] - acc[u][v][e];
            }
}

// The same update for the whole trailing matrix right of a group of block
// columns, in 128 x 128 tiles (twice the products per byte read of the 64 x 64
// kernel above): tile (ib, jb), ib >= jb, covers rows r0 + 128 ib .. +127 and
// columns r0 + 128 jb .. +127 of M, r0 = 64 j0.  Only the lower tiles are
// launched: workgroup b takes tile t = (b % 8) per + b / 8 of the row-major
// list of lower tiles, per = ceil(count / 8), so that the workgroups that share
// an XCD (dispatched round-robin) work on a contiguous run of tiles and share
// their rows of the panel in that XCD's L2.  The contraction runs in chunks of
// 32 columns staged in LDS (two tiles of 128 x 32, padded to an odd stride);
// the next chunk's loads are issued before this chunk's products, and the
// destination tile's entries at the start.  Eight
// waves, each owning a 64 x 32 part (4 x 2 MFMA tiles of 16 x 16, 8
// accumulators, so that two waves fit each SIMD), with the lane layout of the
// kernel above.
constexpr int UT = 128;                  // tile edge
constexpr int UKC = 32;                  // contraction chunk
constexpr int UTHREADS = 512;
constexpr int UPT = UT * UKC / UTHREADS; // loads per thread per tile per chunk
__global__ __launch_bounds__(UTHREADS) void k_chol_update_mfma128(double* __restrict__ M, int q, int kbeg,
                                                                   int kend, int r0, int nt, int per) {
    __shared__ double Li[UT][UKC + 1];
    __shared__ double Lj[UT][UKC + 1];
    const int count = nt * (nt + 1) / 2;
    const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (t >= count) return;
    // row-major lower-triangle index t -> (ib, jb), jb <= ib
    int ib = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ib + 1) * (ib + 2) / 2 <= t) ++ib;
    while (ib * (ib + 1) / 2 > t) --ib;
    const int jb = t - ib * (ib + 1) / 2;
    const int io = r0 + ib * UT, jo = r0 + jb * UT;
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    const int wr = (w >> 2) * 64, wc = (w & 3) * 32;
    const int r16 = lane & 15, k4 = lane >> 4;
    f64x4_t acc[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = f64x4_t{0.0, 0.0, 0.0, 0.0};
    // this thread's entries of the destination tile, loaded at the start (the
    // tile is no operand of this launch and no other workgroup writes it)
    double dst[4][2][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = io + wr + 16 * u + 4 * e + k4, j = jo + wc + 16 * v + r16;
                dst[u][v][e] = (i < q && j < q && j <= i) ? M[(int64_t)i * q + j] : 0.0;
            }
    double vi[UPT], vj[UPT];
    auto load_chunk = [&](int c0) {
#pragma unroll
        for (int h = 0; h < UPT; ++h) {
            const int e = threadIdx.x + h * UTHREADS, i = e / UKC, k = e % UKC;
            const bool kin = c0 + k < kend;
            vi[h] = (io + i < q && kin) ? M[(int64_t)(io + i) * q + c0 + k] : 0.0;
            vj[h] = (jo + i < q && kin) ? M[(int64_t)(jo + i) * q + c0 + k] : 0.0;
        }
    };
    load_chunk(kbeg);
    for (int c0 = kbeg; c0 < kend; c0 += UKC) {
        if (c0 > kbeg) __syncthreads();          // the previous chunk's reads are done
#pragma unroll
        for (int h = 0; h < UPT; ++h) {
            const int e = threadIdx.x + h * UTHREADS, i = e / UKC, k = e % UKC;
            Li[i][k] = vi[h];
            Lj[i][k] = vj[h];
        }
        __syncthreads();
        if (c0 + UKC < kend) load_chunk(c0 + UKC);
#pragma unroll 2
        for (int kk = 0; kk < UKC; kk += 4) {
            double a[4], b[2];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = Li[wr + 16 * u + r16][kk + k4];
#pragma unroll
            for (int v = 0; v < 2; ++v) b[v] = Lj[wc + 16 * v + r16][kk + k4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v)
                    acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[v], acc[u][v], 0, 0, 0);
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = io + wr + 16 * u + 4 * e + k4, j = jo + wc + 16 * v + r16;
                if (i < q && j < q && j <= i) M[(int64_t)i * q + j] = dst[u][v][e] - acc[u][v][e];
            }
}

// Sum of the column-group partials of every row (LDS), returned to the
// threads of group 0.
__device__ __forceinline__ double rows_reduce(double (*red)[NB], double s, int r, int part) {
    red[part][r] = s;
    __syncthreads();
    double t = 0.0;
    if (part == 0) {
#pragma unroll
        for (int pp = 0; pp < SOLVE_PARTS; ++pp) t += red[pp][r];
    }
    return t;
}

// d = -M^{-1} g with the factor in M (lower + mirror) and the diagonal-block
// inverses in inv, in one workgroup of SOLVE_THREADS threads: lane r of wave
// part handles row r of the current 64-row block and every SOLVE_PARTS-th
// column.
// Forward L w = -g, block by block:  y = z_B - L[B, <B] w[<B], w_B = X_B y,
// with L[o + r][c] read from the mirror M[c][o + r].
// Backward L^T d = w from the last block: y = w_B - L[>B, B]^T d[>B], with
// L[c][o + r] read from the lower part M[c][o + r]; then d_B = X_B^T y.
// y_r = sum over c in [c0, c1) of M[c][o + r] z[c] for this thread's columns
// c = c0 + part + SOLVE_PARTS h; the loads of a chunk are all issued before
// any FMA.
__device__ __forceinline__ double column_dot(const double* __restrict__ colp, const double* z,
                                             int c0, int c1, int part, int64_t q, bool active) {
    double s = 0.0;
    if (!active) return s;
    for (int base = c0 + part; base < c1; base += SOLVE_PARTS * SOLVE_CHUNK) {
        double v[SOLVE_CHUNK];
#pragma unroll
        for (int h = 0; h < SOLVE_CHUNK; ++h) {
            const int c = base + SOLVE_PARTS * h;
            v[h] = c < c1 ? colp[(int64_t)c * q] : 0.0;
        }
        double s2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int h = 0; h < SOLVE_CHUNK; ++h) {
            const int c = base + SOLVE_PARTS * h;
            s2[h & 3] = fma(v[h], c < c1 ? z[c] : 0.0, s2[h & 3]);
        }
        s += (s2[0] + s2[1]) + (s2[2] + s2[3]);
    }
    return s;
}

// d = -M^{-1} g with the factor in M (lower + mirror) and the diagonal-block
// inverses in inv, in one workgroup of SOLVE_THREADS threads: lane r of wave
// part handles row r of the current 64-row block and every SOLVE_PARTS-th
// column.
// Forward L w = -g, block by block:  y = z_B - L[B, <B] w[<B], w_B = X_B y,
// with L[o + r][c] read from the mirror M[c][o + r].
// Backward L^T d = w from the last block: y = w_B - L[>B, B]^T d[>B], with
// L[c][o + r] read from the lower part M[c][o + r]; then d_B = X_B^T y.
__global__ __launch_bounds__(SOLVE_THREADS) void k_chol_solve2(const double* __restrict__ M,
                                                               const double* __restrict__ inv,
                                                               const double* __restrict__ g,
                                                               double* __restrict__ d, int q) {
    extern __shared__ double z[];                    // q doubles
    __shared__ double red[SOLVE_PARTS][NB];
    __shared__ double yb[NB];
    const int tid = threadIdx.x, r = tid & (NB - 1), part = tid >> 6;
    g += (int64_t)blockIdx.x * q;                    // right-hand side blockIdx.x (one per block)
    d += (int64_t)blockIdx.x * q;
    for (int i = tid; i < q; i += blockDim.x) z[i] = -g[i];
    const int nblk = (q + NB - 1) / NB;
    for (int B = 0; B < nblk; ++B) {
        const int o = B * NB, m = min(NB, q - o);
        // w_r = sum_{mm <= r} X[r][mm] y_mm = sum_mm X^T[mm][r] y_mm: this thread's
        // four X^T entries, loaded ahead
        const double* XT = inv + (int64_t)B * 2 * NB * NB + NB * NB;
        double xv[NB / SOLVE_PARTS];
#pragma unroll
        for (int k = 0; k < NB / SOLVE_PARTS; ++k) xv[k] = XT[(part * (NB / SOLVE_PARTS) + k) * NB + r];
        __syncthreads();
        double t = rows_reduce(red, column_dot(M + o + r, z, 0, o, part, q, r < m), r, part);
        if (part == 0) yb[r] = r < m ? z[o + r] - t : 0.0;
        __syncthreads();
        double u = 0.0;
#pragma unroll
        for (int k = 0; k < NB / SOLVE_PARTS; ++k) u = fma(xv[k], yb[part * (NB / SOLVE_PARTS) + k], u);
        t = rows_reduce(red, u, r, part);
        if (part == 0 && r < m) z[o + r] = t;
    }
    for (int B = nblk - 1; B >= 0; --B) {
        const int o = B * NB, m = min(NB, q - o), e0 = o + m;
        // d_r = sum_{mm >= r} X[mm][r] y_mm
        const double* X = inv + (int64_t)B * 2 * NB * NB;
        double xv[NB / SOLVE_PARTS];
#pragma unroll
        for (int k = 0; k < NB / SOLVE_PARTS; ++k) xv[k] = X[(part * (NB / SOLVE_PARTS) + k) * NB + r];
        __syncthreads();
        double t = rows_reduce(red, column_dot(M + o + r, z, e0, q, part, q, r < m), r, part);
        if (part == 0) yb[r] = r < m ? z[o + r] - t : 0.0;
        __syncthreads();
        double u = 0.0;
#pragma unroll
        for (int k = 0; k < NB / SOLVE_PARTS; ++k) u = fma(xv[k], yb[part * (NB / SOLVE_PARTS) + k], u);
        t = rows_reduce(red, u, r, part);
        if (part == 0 && r < m) z[o + r] = t;
    }
    __syncthreads();
    for (int i = tid; i < q; i += blockDim.x) d[i] = z[i];
}

// d = -M^{-1} g from the same factor for any size, spread over the chip, one
// launch per diagonal block and direction: every workgroup solves the
// block's 64 x 64 system itself from the inverse of its diagonal factor (16
// products per thread, summed through LDS; workgroup 0 stores the result),
// then updates its part of the not-yet-solved vector with the block's 64
// columns of L (forward, read from the mirror in the upper triangle) or 64 rows
// of L (backward, read from the lower triangle), one thread per entry and the
// 64 loads of a thread in flight together, coalesced across threads:
//   forward  L w = -g:  w_B = X_B z_B;    z_i -= sum_k L[i][o + k] w_{o+k}  (i past B)
//   backward L^T d = w: d_B = X_B^T w_B;  w_j -= sum_r L[o + r][j] d_{o+r} (j before B)
// z lives in d during the forward pass; w is a separate q-vector, so that a
// block's entries are never written while other workgroups read them.
// Each pass reads the triangle of L once: p^2 doubles per solve in total.
__device__ __forceinline__ void trsv_block_solve(const double* __restrict__ Xm, const double* __restrict__ src,
                                                 int o, int m, double* zb, double (*part)[NB], double* out) {
    // out[r] = sum_k Xm[k * NB + r] src[o + k], r < m (zero past m)
    const int tid = threadIdx.x, r = tid & (NB - 1), h = tid / NB;
    if (tid < NB) zb[tid] = tid < m ? src[o + tid] : 0.0;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int kk = 0; kk < NB / 4; ++kk) {
        const int k = (NB / 4) * h + kk;
        t = fma(Xm[k * NB + r], zb[k], t);
    }
    part[h][r] = t;
    __syncthreads();
    if (tid < NB) out[tid] = tid < m ? (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]) : 0.0;
    __syncthreads();
}

// sum over k < m of col[k q] v[k]: for a full block all 64 loads in flight
// at once, else 16 per round
__device__ __forceinline__ double trsv_dot(const double* __restrict__ col, int q, int m, const double* v) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    if (m == NB) {
        double x[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) x[u] = col[(int64_t)u * q];
#pragma unroll
        for (int u = 0; u < NB; ++u) a[u & 3] = fma(x[u], v[u], a[u & 3]);
        return (a[0] + a[1]) + (a[2] + a[3]);
    }
    int k = 0;
    for (; k + 15 < m; k += 16) {
        double x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) x[u] = col[(int64_t)(k + u) * q];
#pragma unroll
        for (int u = 0; u < 16; ++u) a[u & 3] = fma(x[u], v[k + u], a[u & 3]);
    }
    for (; k < m; ++k) a[0] = fma(col[(int64_t)k * q], v[k], a[0]);
    return (a[0] + a[1]) + (a[2] + a[3]);
}

__global__ __launch_bounds__(SSN_BLOCK) void k_trsv_fwd(const double* __restrict__ M,
                                                        const double* __restrict__ inv, int q, int kb,
                                                        double* __restrict__ z, double* __restrict__ w) {
    __shared__ double zb[NB], wb[NB];
    __shared__ double part[4][NB];
    const int o = kb * NB, m = min(NB, q - o);
    // X^T of the block, row-major: element (k, r) is X[r][k]
    trsv_block_solve(inv + (int64_t)kb * 2 * NB * NB + NB * NB, z, o, m, zb, part, wb);
    if (blockIdx.x == 0 && threadIdx.x < m) w[o + threadIdx.x] = wb[threadIdx.x];
    const int64_t i = (int64_t)o + m + (int64_t)blockIdx.x * SSN_BLOCK + threadIdx.x;
    if (i >= q) return;
    z[i] -= trsv_dot(M + (int64_t)o * q + i, q, m, wb);   // M[o + k][i] = L[i][o + k]
}

__global__ __launch_bounds__(SSN_BLOCK) void k_trsv_bwd(const double* __restrict__ M,
                                                        const double* __restrict__ inv, int q, int kb,
                                                        double* __restrict__ w, double* __restrict__ d) {
    __shared__ double zb[NB], db[NB];
    __shared__ double part[4][NB];
    const int o = kb * NB, m = min(NB, q - o);
    // X of the block, row-major: element (k, r) is X[k][r], so the sum is X^T w_B
    trsv_block_solve(inv + (int64_t)kb * 2 * NB * NB, w, o, m, zb, part, db);
    if (blockIdx.x == 0 && threadIdx.x < m) d[o + threadIdx.x] = db[threadIdx.x];
    const int64_t j = (int64_t)blockIdx.x * SSN_BLOCK + threadIdx.x;
    if (j >= o) return;
    w[j] -= trsv_dot(M + (int64_t)o * q + j, q, m, db);   // M[o + r][j] = L[o + r][j]
}

__global__ void k_neg_copy(const double* __restrict__ g, double* __restrict__ d, int q) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < q) d[i] = -g[i];
}

void launch_chol_solve_blocked(const double* M, const double* inv, const double* g, double* d, int64_t q,
                               double* w, hipStream_t s) {
    const int nblk = (int)((q + NB - 1) / NB);
    SSN_LAUNCH(k_neg_copy, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, g, d, (int)q);
    for (int kb = 0; kb < nblk; ++kb) {
        const int64_t o = (int64_t)kb * NB, m = std::min<int64_t>(NB, q - o);
        const int64_t rows = q - o - m;
        const unsigned grid = (unsigned)std::max<int64_t>(1, (rows + SSN_BLOCK - 1) / SSN_BLOCK);
        SSN_LAUNCH(k_trsv_fwd, dim3(grid), dim3(SSN_BLOCK), 0, s, M, inv, (int)q, kb, d, w);
    }
    for (int kb = nblk - 1; kb >= 0; --kb) {
        const int64_t o = (int64_t)kb * NB;
        const unsigned grid = (unsigned)std::max<int64_t>(1, (o + SSN_BLOCK - 1) / SSN_BLOCK);
        SSN_LAUNCH(k_trsv_bwd, dim3(grid), dim3(SSN_BLOCK), 0, s, M, inv, (int)q, kb, w, d);
    }
}

// Two-level blocking: the 64-wide block columns are taken in groups of
// kCholGroup.  Inside a group each block column is factored (diagonal block,
// panel) and its rank-64 update applied only to the group's later block
// columns; the trailing matrix right of the group then takes one update of
// rank 64 kCholGroup, which reads and writes each of its tiles once per group
// instead of once per block column.
#ifndef SSN_CHOL_GROUP
#define SSN_CHOL_GROUP 8
#endif
constexpr int kCholGroup = SSN_CHOL_GROUP;
// The 128 x 128 update takes a trailing matrix of at least this many tiles of
// 128 (2048 rows): below it, one of its workgroups walks a contraction of 512
// in 16 chunks one after another (about 90 us whatever the size), while the
// 64 x 64 kernel spreads the same work over four times as many workgroups
// (30 to 52 us at 512 to 1600 rows); from 2048 rows on the 128 x 128 kernel
// is level with it or up to 10% faster (both near 40 TFLOP/s fp64 at 5000
// to 12000 rows).
constexpr int kUpdate128MinTiles = 16;
void launch_chol_factor_blocked(double* M, int64_t q, double* inv, Scalars* sc, hipStream_t s) {
    const int nblk = (int)((q + NB - 1) / NB);
    for (int K = 0; K < nblk; K += kCholGroup) {
        const int Kend = std::min(nblk, K + kCholGroup);
        for (int kb = K; kb < Kend; ++kb) {
            SSN_LAUNCH(k_chol_diag, dim3(1), dim3(DIAG_THREADS), 0, s, M, (int)q, kb, inv, sc);
            const int nt = nblk - kb - 1;
            if (nt > 0)
                SSN_LAUNCH(k_chol_panel, dim3(nt), dim3(SSN_BLOCK), 0, s, M, (int)q, kb, inv);
            if (kb + 1 < Kend)            // the group's later block columns, all rows below
                SSN_LAUNCH(k_chol_update_mfma, dim3(nblk - kb - 1, Kend - kb - 1), dim3(SSN_BLOCK), 0, s,
                           M, (int)q, kb, kb + 1, kb + 1);
        }
        if (Kend < nblk) {                // everything right of the group
            const int r0 = Kend * NB;
            const int nt = (int)((q - r0 + UT - 1) / UT);
            if (nt >= kUpdate128MinTiles) {
                const int per = (nt * (nt + 1) / 2 + 7) / 8;
                SSN_LAUNCH(k_chol_update_mfma128, dim3((unsigned)(8 * per)), dim3(UTHREADS), 0, s, M, (int)q,
                           K * NB, (int)std::min<int64_t>((int64_t)Kend * NB, q), r0, nt, per);
            } else {
                SSN_LAUNCH(k_chol_update_mfma, dim3(nblk - Kend, nblk - Kend), dim3(SSN_BLOCK), 0, s, M,
                           (int)q, K, Kend, Kend);
            }
        }
    }
}

void launch_chol_solve_factored(const double* M, const double* inv, const double* g, double* d,
                                int64_t q, hipStream_t s) {
    SSN_LAUNCH(k_chol_solve2, dim3(1), dim3(SOLVE_THREADS), (size_t)q * sizeof(double), s, M,
                       inv, g, d, (int)q);
}
void launch_chol_solve_factored_multi(const double* M, const double* inv, const double* G, double* D,
                                      int64_t q, int64_t k, hipStream_t s) {
    if (k <= 0) return;
    SSN_LAUNCH(k_chol_solve2, dim3((unsigned)k), dim3(SOLVE_THREADS), (size_t)q * sizeof(double), s, M,
               inv, G, D, (int)q);
}

}  // namespace ssn
