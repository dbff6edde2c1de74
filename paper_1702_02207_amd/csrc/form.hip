// FP64 formation of A = M^-1 K for dense systems of eq. (1).
//
// M = L L^T by a blocked right-looking Cholesky factorisation with 64-wide
// panels, then A = L^-T (L^-1 K) by blocked forward and back substitution.
// Every O(s^3) part is a 64x64-tiled FP64 matrix-core (MFMA 16x16x4) product.
// Per panel k, two launches:
//   * panel: every workgroup factors the diagonal block L_kk and inverts it
//     (in registers and LDS; the redundancy costs no time, the workgroups run
//     side by side), then one row tile of L_21 = W_21 L_kk^-T and one column
//     tile of the forward solve Y_k = L_kk^-1 R_k;
//   * update: W_22 -= L_21 L_21^T (lower tiles) and R_below -= L_21 Y_k;
// and after the factorisation, from the last panel up, two launches each:
//   * A_k = L_kk^-T R_k, then R_above -= L_k,above^T A_k (backward, in A).
// Triangular solves with an inverted diagonal block instead of substitution
// keep every product on the matrix cores; for SPD M the inverse of a
// triangular block is as accurate as substitution to within a small factor.
//
// Layouts: M, K and A are s x s row-major (M and K symmetric); L is kept
// column-major in the buffer Lc (L_ij at Lc[j*s + i], i below the diagonal
// block of column j; only i >= j is ever read); the inverted diagonal
// blocks are 64x64 row-major, one per panel.
// Systems are batched: every launch covers all of them.

#include "osc_internal.h"

namespace osc {
namespace {

constexpr int kNb = 64;        // panel width and product tile edge
constexpr int kLd = kNb + 1;   // LDS row pitch in doubles

typedef double v4d __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ tile helpers
// Stage a 64 (p) x 64 (q) operand tile into LDS as dst[p][q]: element (q, p)
// of the source at src[q*s_q + p*s_p], zero for q >= nq or p >= np.
// Consecutive threads take q when it has unit stride, else p.
__device__ __forceinline__ void stage_tile(double (*dst)[kLd], const double *src, int64_t s_q, int64_t s_p, int nq,
                                           int np, int tid) {
    if (s_q == 1) {
        for (int idx = tid; idx < kNb * kNb; idx += 256) {
            const int q = idx % kNb, p = idx / kNb;
            dst[p][q] = (q < nq && p < np) ? src[q + p * s_p] : 0.0;
        }
    } else {
        for (int idx = tid; idx < kNb * kNb; idx += 256) {
            const int p = idx % kNb, q = idx / kNb;
            dst[p][q] = (q < nq && p < np) ? src[q * s_q + p * s_p] : 0.0;
        }
    }
}

// acc += A B over p < k for the wave's 32x32 quarter (rows wi.., columns
// wj..) of a 64x64 tile; sa[p][i] = A(i, p), sb[p][j] = B(p, j).
__device__ __forceinline__ void mfma_tile(const double (*sa)[kLd], const double (*sb)[kLd], int k, int wi, int wj,
                                          int lane, v4d (&acc)[2][2]) {
    const int fr = lane % 16, fk = lane / 16;
    const int ksteps = (k + 3) / 4;
    for (int kk = 0; kk < ksteps; ++kk) {
        const int p = 4 * kk + fk;
        const double fa0 = sa[p][wi + fr], fa1 = sa[p][wi + 16 + fr];
        const double fb0 = sb[p][wj + fr], fb1 = sb[p][wj + 16 + fr];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa0, fb0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa0, fb1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa1, fb0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa1, fb1, acc[1][1], 0, 0, 0);
    }
}

// Tile-local (row, column) of accumulator element r of tile (a, b).  FP64
// 16x16x4: element r of lane l is row l/16 + 4r, column l%16 of its 16x16
// block (unlike the FP32-output shapes, rows interleave).
__device__ __forceinline__ int acc_row(int wi, int a, int lane, int r) { return wi + 16 * a + lane / 16 + 4 * r; }
__device__ __forceinline__ int acc_col(int wj, int b, int lane) { return wj + 16 * b + lane % 16; }

__device__ __forceinline__ void zero_acc(v4d (&acc)[2][2]) {
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
}

// C(i, j) = acc for i < m, j < n; C(i, j) at C[i*c_i + j*c_j]
__device__ __forceinline__ void store_acc(double *C, int64_t c_i, int64_t c_j, int m, int n, int wi, int wj,
                                          int lane, const v4d (&acc)[2][2]) {
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int r = 0; r < 4; ++r) {
                const int i = acc_row(wi, a, lane, r), j = acc_col(wj, b, lane);
                if (i < m && j < n) C[i * c_i + j * c_j] = acc[a][b][r];
            }
}

// ------------------------------------------------------------------- panel
struct Panel {
    int s, k0, nbk, rest;   // panel columns k0 .. k0+nbk-1, rest = rows below
    int tiles_below, tiles_n, per_sys;
    double *Lc;             // factor in progress, column-major
    double *R;              // forward right-hand sides (row-major, in A)
    double *Inv;            // this panel's inverted diagonal block (row-major 64x64)
    size_t lstride, istride;
    int *status;
};

// Every workgroup: factor the nbk x nbk diagonal block (padded to 64 with the
// identity, its own factor and inverse) and invert it; thread t holds column
// t%64, rows t/64 + 4q of the block in registers.  Then workgroup w computes
// row tile w of L_21 and column tile w of Y_k.  Workgroup 0 stores
// inv(L_kk); L_kk itself is never needed again (every later use of the
// diagonal block goes through its inverse), so W_kk stays in Lc, and no
// workgroup writes what another one reads.
__global__ void __launch_bounds__(256) panel_kernel(Panel P) {
    __shared__ double sx[kNb][kLd];   // sx[p][i] = inv(L_kk)(i, p)
    __shared__ double sw[kNb][kLd];   // L_kk, then operand staging
    __shared__ double bcast[2][kNb];
    __shared__ double rdiag[kNb];
    const int tid = threadIdx.x, lane = tid % 64;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);   // wave-uniform: branches on it do not diverge
    const int c = lane, r0 = wave;
    const int64_t sys = blockIdx.x / P.per_sys;
    const int w = (int)(blockIdx.x % P.per_sys);
    const int s = P.s, k0 = P.k0, nbk = P.nbk;
    double *Lc = P.Lc + sys * P.lstride;
    double *R = P.R + sys * P.lstride;

    double v[kNb / 4];
#pragma unroll
    for (int q = 0; q < kNb / 4; ++q) {
        const int r = r0 + 4 * q;
        v[q] = (r < nbk && c < nbk && c <= r) ? Lc[(size_t)(k0 + c) * s + k0 + r] : (r == c ? 1.0 : 0.0);
    }
    // Right-looking factorisation, one barrier per column: the owners of
    // column j publish its entries on and below the diagonal (zeros above),
    // unscaled; every thread scales them on the fly for its trailing update.
    // Lanes of finished columns (c <= j) take an update with a zero factor,
    // which leaves them exactly unchanged, so the loop body is the same
    // straight-line code for every lane; each lane scales its own column by
    // the factors it kept from its pivot step once the loop is done.  Entries
    // above the diagonal take meaningless updates and are discarded; no
    // update reaches an entry on or below the diagonal from one above it.  The
    // broadcast buffer alternates, so step j+1 can publish while step j still
    // reads.
    bool failed = false;
    double my_l = 1.0, my_inv = 1.0;
    for (int j = 0; j < nbk; ++j) {
        double *col = bcast[j & 1];
        if (c == j) {
#pragma unroll
            for (int q = 0; q < kNb / 4; ++q) col[r0 + 4 * q] = r0 + 4 * q >= j ? v[q] : 0.0;
        }
        __syncthreads();
        const double d = col[j];
        const bool ok = d > 0.0 && __builtin_isfinite(d);
        failed |= !ok;
        const double ljj = ok ? sqrt(d) : __builtin_nan("");
        const double inv = 1.0 / ljj;
        my_l = c == j ? ljj : my_l;
        my_inv = c == j ? inv : my_inv;
        const double lcj = c > j ? col[c] * inv : 0.0;
#pragma unroll
        for (int q = 0; q < kNb / 4; ++q) v[q] -= (col[r0 + 4 * q] * inv) * lcj;
    }
#pragma unroll
    for (int q = 0; q < kNb / 4; ++q) {
        const int r = r0 + 4 * q;
        v[q] = r == c ? my_l : v[q] * my_inv;
    }
    if (failed && w == 0 && tid == 0) atomicOr(P.status, 1);
#pragma unroll
    for (int q = 0; q < kNb / 4; ++q) {
        const int r = r0 + 4 * q;
        sw[r][c] = r >= c ? v[q] : 0.0;
    }
    __syncthreads();
    if (tid < kNb) rdiag[tid] = 1.0 / sw[tid][tid];
    __syncthreads();
    // X = inv(L_kk) row by row: row k is final once rows < k are applied;
    // its owners (wave k%4) publish it and every thread updates its rows > k.
#pragma unroll
    for (int q = 0; q < kNb / 4; ++q) v[q] = (r0 + 4 * q == c) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < kNb; ++k) {
        double *row = bcast[k & 1];
        if (r0 == (k & 3)) {
            v[k / 4] *= rdiag[k];
            row[c] = v[k / 4];
        }
        __syncthreads();
        const double xk = row[c];
#pragma unroll
        for (int q = k / 4; q < kNb / 4; ++q) {
            const int r = r0 + 4 * q;
            if (r > k) v[q] -= sw[r][k] * xk;
        }
    }
#pragma unroll
    for (int q = 0; q < kNb / 4; ++q) {
        const int r = r0 + 4 * q;
        const double x = (r < nbk && c < nbk) ? v[q] : 0.0;
        sx[c][r] = x;
        if (w == 0) P.Inv[sys * P.istride + r * kNb + c] = x;
    }
    __syncthreads();

    const int wi = (wave / 2) * 32, wj = (wave % 2) * 32;
    v4d acc[2][2];
    if (w < P.tiles_below) {
        // L_21 tile = W_21 tile inv(L_kk)^T; B(p, j) = inv(L_kk)(j, p) = sx[p][j]
        double *w21 = Lc + (size_t)k0 * s + k0 + nbk + kNb * w;
        const int nrow = min(kNb, P.rest - kNb * w);
        stage_tile(sw, w21, 1, s, nrow, nbk, tid);
        __syncthreads();
        zero_acc(acc);
        mfma_tile(sw, sx, nbk, wi, wj, lane, acc);
        store_acc(w21, 1, s, nrow, nbk, wi, wj, lane, acc);
        __syncthreads();
    }
    if (w < P.tiles_n) {
        // Y_k column tile = inv(L_kk) R_k column tile, in place
        double *rk = R + (size_t)k0 * s + kNb * w;
        const int ncol = min(kNb, s - kNb * w);
        stage_tile(sw, rk, 1, s, ncol, nbk, tid);
        __syncthreads();
        zero_acc(acc);
        mfma_tile(sx, sw, nbk, wi, wj, lane, acc);
        store_acc(rk, s, 1, nbk, ncol, wi, wj, lane, acc);
    }
}

// ---------------------------------------------------------------- products
// C(i, j) = A B  or  C(i, j) -= A B  over an m x n x k product (k <= 64) of
// strided FP64 operands: element (i, p) of A at A[i*a_i + p*a_p], (p, j) of B
// at B[p*b_p + j*b_j], (i, j) of C at C[i*c_i + j*c_j]; system z adds z times
// the *_sys strides.  One 256-thread workgroup per 64x64 tile of C (lower
// tiles only when `lower`), each wave a 32x32 quarter as 2x2 MFMA 16x16x4
// blocks; the k dimension runs in chunks of 64 staged through LDS.  A tile
// reads all of its operands before it writes, so C may alias A (when
// n <= 64) or B (when m <= 64).
struct Product {
    int m, n, k;
    int tiles_n;
    int64_t tiles;   // tiles per system
    int overwrite;   // 1: C = A B; 0: C -= A B
    int lower;
    const double *A;
    int64_t a_i, a_p;
    size_t a_sys;
    const double *B;
    int64_t b_p, b_j;
    size_t b_sys;
    double *C;
    int64_t c_i, c_j;
    size_t c_sys;
};

// Up to two independent products in one launch (tiles of the first, then of
// the second, per system).
struct ProductPair {
    Product g[2];
    int64_t per_sys;
};

__global__ void __launch_bounds__(256) product_kernel(ProductPair pp) {
    __shared__ double sa[kNb][kLd];   // [p][i]
    __shared__ double sb[kNb][kLd];   // [p][j]
    const int64_t sys = blockIdx.x / pp.per_sys;
    int64_t t = blockIdx.x % pp.per_sys;
    const int which = t < pp.g[0].tiles ? 0 : 1;
    const Product &g = pp.g[which];
    if (which) t -= pp.g[0].tiles;
    int ti, tj;
    if (g.lower) {
        // t -> (ti >= tj) in row order of the lower triangle
        ti = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while ((int64_t)(ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while ((int64_t)ti * (ti + 1) / 2 > t) --ti;
        tj = (int)(t - (int64_t)ti * (ti + 1) / 2);
    } else {
        ti = (int)(t / g.tiles_n);
        tj = (int)(t % g.tiles_n);
    }
    const int i0 = ti * kNb, j0 = tj * kNb;
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int wi = (wave / 2) * 32, wj = (wave % 2) * 32;
    const double *A = g.A + sys * g.a_sys + i0 * g.a_i;
    const double *B = g.B + sys * g.b_sys + j0 * g.b_j;
    double *C = g.C + sys * g.c_sys + i0 * g.c_i + j0 * g.c_j;
    const int m = min(kNb, g.m - i0), n = min(kNb, g.n - j0);
    // the old C values load while the first operands stage
    double old[2][2][4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int r = 0; r < 4; ++r) {
                const int i = acc_row(wi, a, lane, r), j = acc_col(wj, b, lane);
                old[a][b][r] = (!g.overwrite && i < m && j < n) ? C[i * g.c_i + j * g.c_j] : 0.0;
            }
    v4d acc[2][2];
    zero_acc(acc);
    for (int p0 = 0; p0 < g.k; p0 += kNb) {
        const int kc = min(kNb, g.k - p0);
        if (p0 > 0) __syncthreads();   // every wave is done with the previous chunk
        stage_tile(sa, A + p0 * g.a_p, g.a_i, g.a_p, m, kc, tid);
        // B staged as [p][j]: its "q" index is j
        const double *Bp = B + p0 * g.b_p;
        if (g.b_j == 1) {
            for (int idx = tid; idx < kNb * kNb; idx += 256) {
                const int j = idx % kNb, p = idx / kNb;
                sb[p][j] = (j < n && p < kc) ? Bp[j + p * g.b_p] : 0.0;
            }
        } else {
            for (int idx = tid; idx < kNb * kNb; idx += 256) {
                const int p = idx % kNb, j = idx / kNb;
                sb[p][j] = (j < n && p < kc) ? Bp[j * g.b_j + p * g.b_p] : 0.0;
            }
        }
        __syncthreads();
        mfma_tile(sa, sb, kc, wi, wj, lane, acc);
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int r = 0; r < 4; ++r) acc[a][b][r] = g.overwrite ? acc[a][b][r] : old[a][b][r] - acc[a][b][r];
    store_acc(C, g.c_i, g.c_j, m, n, wi, wj, lane, acc);
}

bool prepare(Product &g) {
    if (g.m <= 0 || g.n <= 0 || g.k <= 0) {
        g.tiles = 0;
        return false;
    }
    const int tm = (g.m + kNb - 1) / kNb;
    g.tiles_n = (g.n + kNb - 1) / kNb;
    g.tiles = g.lower ? (int64_t)tm * (tm + 1) / 2 : (int64_t)tm * g.tiles_n;
    return true;
}

osc_status run_products(Product g0, Product g1, int64_t nsys, hipStream_t st) {
    ProductPair pp{};
    prepare(g0);
    prepare(g1);
    if (g0.tiles == 0) std::swap(g0, g1);
    pp.g[0] = g0;
    pp.g[1] = g1;
    pp.per_sys = g0.tiles + g1.tiles;
    if (pp.per_sys == 0 || nsys == 0) return OSC_OK;
    const int64_t blocks = pp.per_sys * nsys;
    if (blocks > 0x7fffffff) return fail(OSC_EINVAL, "too many systems for one formation launch");
    hipLaunchKernelGGL(product_kernel, dim3((unsigned)blocks), dim3(256), 0, st, pp);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

}  // namespace

osc_status gemm64(const Gemm64 &p, int64_t nsys, hipStream_t st) {
    Product g{};
    g.m = p.m, g.n = p.n, g.k = p.k;
    g.overwrite = p.overwrite;
    g.A = p.A, g.a_i = p.a_i, g.a_p = p.a_p, g.a_sys = p.a_sys;
    g.B = p.B, g.b_p = p.b_p, g.b_j = p.b_j, g.b_sys = p.b_sys;
    g.C = p.C, g.c_i = p.c_i, g.c_j = p.c_j, g.c_sys = p.c_sys;
    return run_products(g, Product{}, nsys, st);
}

size_t dense_form_scratch_elems(int s) {
    return (size_t)((s + kNb - 1) / kNb) * kNb * kNb;
}

osc_status dense_form_a(int s, int64_t nsys, const double *M, const double *K, double *Lc, double *Inv, double *A,
                        int *status, hipStream_t st) {
    if (nsys == 0 || s == 0) return OSC_OK;
    if (nsys > 0x7fffffff) return fail(OSC_EINVAL, "too many systems for one formation launch");
    const size_t ss = (size_t)s * s;
    const size_t is = dense_form_scratch_elems(s);
    OSC_HIP(hipMemcpyAsync(Lc, M, nsys * ss * sizeof(double), hipMemcpyDeviceToDevice, st));
    OSC_HIP(hipMemcpyAsync(A, K, nsys * ss * sizeof(double), hipMemcpyDeviceToDevice, st));
    const int nblk = (s + kNb - 1) / kNb;
    osc_status r;
    for (int kb = 0; kb < nblk; ++kb) {
        const int k0 = kb * kNb, nbk = std::min(kNb, s - k0), rest = s - k0 - nbk;
        Panel P{};
        P.s = s, P.k0 = k0, P.nbk = nbk, P.rest = rest;
        P.tiles_below = (rest + kNb - 1) / kNb;
        P.tiles_n = (s + kNb - 1) / kNb;
        P.per_sys = std::max(P.tiles_below, P.tiles_n);
        P.Lc = Lc, P.R = A, P.Inv = Inv + (size_t)kb * kNb * kNb;
        P.lstride = ss, P.istride = is;
        P.status = status;
        const int64_t blocks = (int64_t)P.per_sys * nsys;
        if (blocks > 0x7fffffff) return fail(OSC_EINVAL, "too many systems for one formation launch");
        hipLaunchKernelGGL(panel_kernel, dim3((unsigned)blocks), dim3(256), 0, st, P);
        OSC_HIP(hipGetLastError());
        double *w21 = Lc + (size_t)k0 * s + k0 + nbk;   // (i, p): rows below the block, panel columns
        // W_22 -= L_21 L_21^T (lower tiles) and R_below -= L_21 Y_k
        Product g0{}, g1{};
        g0.m = rest, g0.n = rest, g0.k = nbk, g0.lower = 1;
        g0.A = w21, g0.a_i = 1, g0.a_p = s, g0.a_sys = ss;
        g0.B = w21, g0.b_p = s, g0.b_j = 1, g0.b_sys = ss;
        g0.C = Lc + (size_t)(k0 + nbk) * s + k0 + nbk, g0.c_i = 1, g0.c_j = s, g0.c_sys = ss;
        g1.m = rest, g1.n = s, g1.k = nbk;
        g1.A = w21, g1.a_i = 1, g1.a_p = s, g1.a_sys = ss;
        g1.B = A + (size_t)k0 * s, g1.b_p = s, g1.b_j = 1, g1.b_sys = ss;
        g1.C = A + (size_t)(k0 + nbk) * s, g1.c_i = s, g1.c_j = 1, g1.c_sys = ss;
        if ((r = run_products(g0, g1, nsys, st))) return r;
    }
    for (int kb = nblk - 1; kb >= 0; --kb) {
        const int k0 = kb * kNb, nbk = std::min(kNb, s - k0);
        const double *inv = Inv + (size_t)kb * kNb * kNb;
        double *rk = A + (size_t)k0 * s;
        // A_k = inv(L_kk)^T R_k in place
        Product g{};
        g.m = nbk, g.n = s, g.k = nbk, g.overwrite = 1;
        g.A = inv, g.a_i = 1, g.a_p = kNb, g.a_sys = is;
        g.B = rk, g.b_p = s, g.b_j = 1, g.b_sys = ss;
        g.C = rk, g.c_i = s, g.c_j = 1, g.c_sys = ss;
        if ((r = run_products(g, Product{}, nsys, st))) return r;
        // R_above -= (L_k,above)^T A_k: element (i, p) = L(k0 + p, i) at Lc[i*s + k0 + p]
        g = Product{};
        g.m = k0, g.n = s, g.k = nbk;
        g.A = Lc + k0, g.a_i = s, g.a_p = 1, g.a_sys = ss;
        g.B = rk, g.b_p = s, g.b_j = 1, g.b_sys = ss;
        g.C = A, g.c_i = s, g.c_j = 1, g.c_sys = ss;
        if ((r = run_products(g, Product{}, nsys, st))) return r;
    }
    return OSC_OK;
}

}  // namespace osc
