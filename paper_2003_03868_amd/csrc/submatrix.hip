// Submatrix method (section "Submatrix Method"): the density matrix from
// one small dense problem per block column instead of sparse products over
// the whole matrix.
//
// For block column j let N_j be the block rows with a stored block in
// column j (ascending; j itself included).  T_j = H[N_j, N_j] is the dense
// principal submatrix over those block rows, P_j = (I - sign(T_j - mu I))/2
// its density matrix, and block column j of P is P_j's block column of j,
// on H's pattern; P is filtered with the block-norm rule at the end.
//
// Each sign(T_j - mu I) is taken by the dense Newton-Schulz iteration
//   X_0 = (T_j - mu I) / ||T_j - mu I||_inf
//   k = 0, 1, ...:  Y = X_k X_k;  r_k = ||Y - I||_F / n_j;  stop if r_k < tol
//                   X_{k+1} = 1.5 X_k - 0.5 X_k Y
// with every submatrix of a batch advanced together and each stopped on its
// own residual.  Submatrices live densely in HBM, padded to multiples of 32
// (the padding stays zero through both products); the products run on the
// FP64 matrix cores in one launch over the 64 x 64 tiles of all active
// submatrices, the last tile row and column 32 wide where the edge ends there.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "bsm_internal.h"

namespace bsm {

namespace {

constexpr int kTile = 64;      // output tile edge of the dense product
constexpr int kPad = 32;       // submatrix edges are padded to a multiple of this
constexpr int kTk = 16;        // k depth staged per LDS stage
constexpr int kLdA = 68;       // LDS row pitch (doubles) of the k-major A stage
constexpr int kLdB = 80;       // LDS row pitch (doubles) of the B stage

struct SubGemm {
    const int4 *tiles;         // (submatrix, tile row, tile column, buffer of X)
    int32_t ntiles;
    const int64_t *base;       // per submatrix: offset (doubles) in every buffer
    const int32_t *npad;       // per submatrix: padded edge (multiple of 32)
    const int32_t *ndim;       // per submatrix: true edge n_j
    double *buf0, *buf1, *ybuf;
    int32_t mode;              // 0: Y = X X (+ residual partials); 1: X' = 1.5 X - 0.5 X Y
    double *partial;           // mode 0: per tile, sum over its entries of (Y - I)^2
};

// One 64 x 64 tile of D = A B (mode 0: A = B = X, D = Y; mode 1: A = X,
// B = Y, D = 1.5 X - 0.5 A B into the other X buffer).  Four waves, each a
// 32 x 32 quarter as 8 x 8 blocks of 4 x 4 on V_MFMA_F64_4X4X4_4B_F64: lane
// (x, b, y) = lane / 16, lane / 4 % 4, lane % 4 feeds A(i = y, k = x) and
// B(k = x, j = y) of block b and receives D(i = x, j = y).  A is staged
// k-major so the eight A operands of a k step are conflict-free LDS reads.
// A tile that reaches past the padded edge is 32 rows or columns wide: the
// waves of its missing half skip their products and stores, and the
// staging loads of that half are clamped to addresses inside the square
// (data that only those idle waves would read).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_sub_gemm(SubGemm g) {
    // consecutive tiles (one submatrix) on one XCD: workgroups b, b+8, ...
    // share an XCD's L2
    const int per = (g.ntiles + kXcds - 1) / kXcds;
    const int tix = static_cast<int>(blockIdx.x % kXcds) * per + static_cast<int>(blockIdx.x / kXcds);
    if (tix >= g.ntiles) return;
    const int4 td = g.tiles[tix];
    const int sub = td.x;
    const int ld = g.npad[sub];
    const int64_t base = g.base[sub];
    const double *X = (td.w ? g.buf1 : g.buf0) + base;
    const double *Bm = g.mode == 0 ? X : g.ybuf + base;
    double *D = g.mode == 0 ? g.ybuf + base : (td.w ? g.buf0 : g.buf1) + base;
    const int r0 = td.y * kTile, c0 = td.z * kTile;
    const int vr = min(kTile, ld - r0), vc = min(kTile, ld - c0);   // 32 or 64

    __shared__ double As[2][kTk][kLdA];
    __shared__ double Bs[2][kTk][kLdB];
    __shared__ double red[4];

    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int x = lane >> 4, bb = (lane >> 2) & 3, y = lane & 3;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    // global -> LDS staging: A rows r0 + t/4, four k from (t%4)*4 (pitch 68:
    // each transposed store spreads over all banks); B k row t/16, columns
    // 2c, 2c+1 and 32+2c, 33+2c for c = t%16, so each 16-byte store of a row
    // is contiguous with its neighbours' and the global reads are two
    // 256-byte runs per row
    const int ar = t >> 2, ak = (t & 3) << 2;
    const int bk = t >> 4, bc = (t & 15) << 1;
    const double *ga = X + static_cast<int64_t>(r0 + (ar < vr ? ar : 0)) * ld + ak;
    const double *gb = Bm + static_cast<int64_t>(bk) * ld + c0 + bc;
    const int bhi = vc > 32 ? 32 : 0;                  // second column half, or a repeat
    const bool busy = wr < vr && wc < vc;              // wave-uniform

    // two register sets of staged operands in flight: the loads for k step
    // i + 3 are issued at step i and written to LDS at step i + 2
    struct Regs { double2 a0, a1, b0, b1; };
    auto load = [&](int k, Regs &r) {
        const double2 *a2 = reinterpret_cast<const double2 *>(ga + k);
        const double *bp = gb + static_cast<int64_t>(k) * ld;
        r.a0 = a2[0]; r.a1 = a2[1];
        r.b0 = *reinterpret_cast<const double2 *>(bp);
        r.b1 = *reinterpret_cast<const double2 *>(bp + bhi);
    };
    auto stage = [&](int buf, const Regs &r) {
        As[buf][ak + 0][ar] = r.a0.x; As[buf][ak + 1][ar] = r.a0.y;
        As[buf][ak + 2][ar] = r.a1.x; As[buf][ak + 3][ar] = r.a1.y;
        *reinterpret_cast<double2 *>(&Bs[buf][bk][bc]) = r.b0;
        *reinterpret_cast<double2 *>(&Bs[buf][bk][bc + 32]) = r.b1;
    };

    double acc[8][2];
#pragma unroll
    for (int R = 0; R < 8; ++R) { acc[R][0] = 0.0; acc[R][1] = 0.0; }
    auto compute = [&](int cur) {
        if (!busy) return;
#pragma unroll
        for (int kk = 0; kk < kTk; kk += 4) {
            double a[8], b[2];
#pragma unroll
            for (int R = 0; R < 8; ++R) a[R] = As[cur][kk + x][wr + 4 * R + y];
#pragma unroll
            for (int G = 0; G < 2; ++G) b[G] = Bs[cur][kk + x][wc + 16 * G + 4 * bb + y];
#pragma unroll
            for (int R = 0; R < 8; ++R)
#pragma unroll
                for (int G = 0; G < 2; ++G)
                    acc[R][G] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[R], b[G], acc[R][G], 0, 0, 0);
        }
    };

    // k steps of kTk up to the edge rounded to kTk (the padding beyond it is
    // zero, so the remaining steps would add nothing): nk >= 1.  Set s0
    // carries steps 0, 2, 4, ..., set s1 steps 1, 3, 5, ...; buffer i & 1
    // holds step i.
    const int nk = (g.ndim[sub] + kTk - 1) / kTk;
    Regs s0, s1;
    load(0, s0);
    stage(0, s0);
    if (nk > 1) load(kTk, s1);
    if (nk > 2) load(2 * kTk, s0);
    __syncthreads();
    for (int i = 0; i < nk; i += 2) {
        compute(0);                                   // step i
        if (i + 1 < nk) stage(1, s1);                 // step i + 1
        if (i + 3 < nk) load((i + 3) * kTk, s1);
        __syncthreads();
        if (i + 1 < nk) {
            compute(1);                               // step i + 1
            if (i + 2 < nk) stage(0, s0);             // step i + 2
            if (i + 4 < nk) load((i + 4) * kTk, s0);
            __syncthreads();
        }
    }

    const int n = g.ndim[sub];
    double res = 0.0;
#pragma unroll
    for (int R = 0; R < 8 && busy; ++R) {
        const int r = r0 + wr + 4 * R + x;
#pragma unroll
        for (int G = 0; G < 2; ++G) {
            const int c = c0 + wc + 16 * G + 4 * bb + y;
            const int64_t o = static_cast<int64_t>(r) * ld + c;
            if (g.mode == 0) {
                const double v = acc[R][G];
                D[o] = v;
                const double d = v - ((r == c && r < n) ? 1.0 : 0.0);
                res += d * d;
            } else {
                D[o] = 1.5 * X[o] - 0.5 * acc[R][G];
            }
        }
    }
    if (g.mode == 0) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) res += __shfl_xor(res, off);
        if (lane == 0) red[w] = res;
        __syncthreads();
        if (t == 0) g.partial[tix] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// r = ||Y - I||_F / n per active submatrix from its tiles' partial sums
// (tiles of one submatrix are consecutive; summed in tile order).
__global__ void k_sub_resid(const double *partial, const int32_t *act_sub, const int32_t *tile_lo,
                            const int32_t *tile_hi, const int32_t *ndim, double *r, int32_t nact) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nact) return;
    double s = 0.0;
    for (int u = tile_lo[a]; u < tile_hi[a]; ++u) s += partial[u];
    r[a] = sqrt(s) / static_cast<double>(ndim[act_sub[a]]);
}

// Dense T_j - mu I from the stored blocks: one 64-lane group per (submatrix,
// block row a); lane f looks block column f of the submatrix up in H's row
// N_j[a] and copies it when stored.  The buffer is zero beforehand.
__global__ void k_sub_gather(const int64_t *row_ptr, const int32_t *col_idx, const int64_t *blk_off,
                             const double *vals, const int32_t *rbs, const int32_t *ent_row,
                             const int32_t *ent_soff, const int32_t *ent_sub,
                             const int64_t *sub_ent0, const int64_t *base, const int32_t *npad,
                             double mu, double *X, int64_t nent) {
    const int64_t e = blockIdx.x;
    if (e >= nent) return;
    const int sub = ent_sub[e];
    const int i = ent_row[e];
    const int ra = ent_soff[e];
    const int bi = rbs[i];
    const int ld = npad[sub];
    double *T = X + base[sub];
    const int64_t p0 = row_ptr[i], p1 = row_ptr[i + 1];
    for (int64_t f = sub_ent0[sub] + threadIdx.x; f < sub_ent0[sub + 1]; f += blockDim.x) {
        const int k = ent_row[f];
        int64_t lo = p0, hi = p1;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (col_idx[mid] < k) lo = mid + 1; else hi = mid;
        }
        if (lo >= p1 || col_idx[lo] != k) continue;
        const int bk = rbs[k];
        const int cb = ent_soff[f];
        const double *src = vals + blk_off[lo];
        for (int u = 0; u < bi; ++u)
            for (int v = 0; v < bk; ++v)
                T[static_cast<int64_t>(ra + u) * ld + cb + v] =
                    src[u * bk + v] - ((k == i && u == v) ? mu : 0.0);
    }
}

// ||T_j - mu I||_inf per submatrix: one workgroup each, a wave per row.
__global__ __launch_bounds__(256) void k_sub_infnorm(const double *X, const int64_t *base,
                                                     const int32_t *npad, const int32_t *ndim,
                                                     double *scale) {
    const int sub = blockIdx.x;
    const double *T = X + base[sub];
    const int ld = npad[sub], n = ndim[sub];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double mx = 0.0;
    for (int r = w; r < n; r += 4) {
        double s = 0.0;
        for (int c = lane; c < n; c += 64) s += fabs(T[static_cast<int64_t>(r) * ld + c]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        mx = fmax(mx, s);
    }
    __shared__ double red[4];
    if (lane == 0) red[w] = mx;
    __syncthreads();
    if (threadIdx.x == 0) scale[sub] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// X_0 = T / s over each submatrix's padded square (submatrices strided
// over grid.y).
__global__ void k_sub_scale(double *X, const int64_t *base, const int32_t *npad,
                            const double *scale, int32_t nsub) {
    for (int sub = blockIdx.y; sub < nsub; sub += gridDim.y) {
        const int64_t len = static_cast<int64_t>(npad[sub]) * npad[sub];
        const double f = 1.0 / scale[sub];
        double *T = X + base[sub];
        for (int64_t u = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; u < len;
             u += static_cast<int64_t>(gridDim.x) * blockDim.x)
            T[u] *= f;
    }
}

// Block (N_j[a], j) of P = (delta - X_j[a-th rows, j's columns]) / 2 into P's
// values (H's pattern); one 64-lane group per (submatrix, block row a).
__global__ void k_sub_extract(const int64_t *row_ptr, const int32_t *col_idx, const int64_t *blk_off,
                              const int32_t *rbs, const int32_t *ent_row, const int32_t *ent_soff,
                              const int32_t *ent_sub, const int32_t *sub_col,
                              const int32_t *sub_csoff, const int64_t *base, const int32_t *npad,
                              const int32_t *parity, const double *buf0, const double *buf1,
                              double *pvals, int64_t nent) {
    const int64_t e = blockIdx.x;
    if (e >= nent) return;
    const int sub = ent_sub[e];
    const int i = ent_row[e], j = sub_col[sub];
    const int ra = ent_soff[e], cj = sub_csoff[sub];
    const int bi = rbs[i], bj = rbs[j];
    const int ld = npad[sub];
    const double *Xs = (parity[sub] ? buf1 : buf0) + base[sub];
    int64_t lo = row_ptr[i], hi = row_ptr[i + 1];
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (col_idx[mid] < j) lo = mid + 1; else hi = mid;
    }
    if (lo >= row_ptr[i + 1] || col_idx[lo] != j) return;   // cannot happen: i is in N_j
    double *dst = pvals + blk_off[lo];
    for (int u = threadIdx.x; u < bi * bj; u += blockDim.x) {
        const int p = u / bj, q = u % bj;
        const double xv = Xs[static_cast<int64_t>(ra + p) * ld + cj + q];
        dst[u] = 0.5 * (((i == j && p == q) ? 1.0 : 0.0) - xv);
    }
}

template <class T>
int upload(T **d, const std::vector<T> &h, hipStream_t s) {
    BSM_TRY(dalloc(d, std::max<size_t>(h.size(), 1), s));
    if (!h.empty())
        BSM_HIP(hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return BSM_OK;
}

size_t batch_bytes_cap() {
    const char *e = std::getenv("BSM_SUB_BATCH_BYTES");
    if (e) {
        const long long v = std::atoll(e);
        if (v > 0) return static_cast<size_t>(v);
    }
    return size_t(48) << 30;
}

}  // namespace

int submatrix_density(Mat &H, double mu, const bsm_sign_opts &o, Mat **p_out, bsm_sub_stats *st,
                      hipStream_t s) {
    *p_out = nullptr;
    if (H.nbrows != H.nbcols || H.h_rbs != H.h_cbs) {
        set_error("submatrix: H must be square with square diagonal blocks");
        return BSM_EINVAL;
    }
    if (!std::isfinite(mu) || !(o.eps_filter >= 0.0) || !std::isfinite(o.eps_filter) ||
        !(o.tol > 0.0) || o.max_iter < 0 || o.max_iter > 120 ||
        (o.norm != BSM_NORM_FROB && o.norm != BSM_NORM_MAXABS)) {
        set_error("submatrix: need a finite mu, eps_filter >= 0, tol > 0, 0 <= max_iter <= 120, "
                  "a known norm");
        return BSM_EINVAL;
    }
    // pattern on the host: the column sets N_j (rows ascending)
    const int nb = H.nbrows;
    std::vector<int64_t> rp(nb + 1);
    std::vector<int32_t> ci(H.nnzb);
    BSM_HIP(hipMemcpyAsync(rp.data(), H.row_ptr, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost, s));
    if (H.nnzb)
        BSM_HIP(hipMemcpyAsync(ci.data(), H.col_idx, sizeof(int32_t) * H.nnzb, hipMemcpyDeviceToHost, s));
    BSM_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> cp(nb + 1, 0);
    for (int64_t t = 0; t < H.nnzb; ++t) cp[ci[t] + 1]++;
    for (int j = 0; j < nb; ++j) cp[j + 1] += cp[j];
    std::vector<int32_t> crow(H.nnzb);
    {
        std::vector<int64_t> fill(cp.begin(), cp.end() - 1);
        for (int i = 0; i < nb; ++i)
            for (int64_t t = rp[i]; t < rp[i + 1]; ++t) crow[fill[ci[t]]++] = i;
    }
    std::vector<int32_t> dim(nb), pad(nb), csoff(nb);
    for (int j = 0; j < nb; ++j) {
        int64_t n = 0;
        int pos = -1;
        for (int64_t u = cp[j]; u < cp[j + 1]; ++u) {
            if (crow[u] == j) { pos = static_cast<int>(u - cp[j]); csoff[j] = static_cast<int32_t>(n); }
            n += H.h_rbs[crow[u]];
        }
        if (pos < 0) {
            set_error("submatrix: block column %d has no stored diagonal block", j);
            return BSM_EINVAL;
        }
        if (n > (1 << 15)) {
            set_error("submatrix: block column %d spans %lld rows (at most 32768)", j,
                      static_cast<long long>(n));
            return BSM_EINVAL;
        }
        dim[j] = static_cast<int32_t>(n);
        pad[j] = static_cast<int32_t>((n + kPad - 1) / kPad * kPad);
    }

    hipEvent_t t0, t1;
    BSM_HIP(hipEventCreate(&t0));
    BSM_HIP(hipEventCreate(&t1));
    BSM_HIP(hipEventRecord(t0, s));
    Mat *P = nullptr;
    int rc = copy_mat(H, &P, s);

    st->n_sub = nb;
    double sum_dim = 0.0;
    for (int j = 0; j < nb; ++j) {
        st->max_dim = std::max(st->max_dim, dim[j]);
        sum_dim += dim[j];
    }
    st->mean_dim = nb ? sum_dim / nb : 0.0;

    const size_t cap = batch_bytes_cap();
    std::vector<std::pair<hipEvent_t, hipEvent_t>> gev;
    int64_t n_noconv = 0;            // submatrices left above tol (every batch still runs)
    int j0 = 0;
    while (rc == BSM_OK && j0 < nb) {
        // the batch: consecutive block columns while three padded squares fit
        size_t bytes = 0;
        int j1 = j0;
        while (j1 < nb) {
            const size_t b = size_t(3) * sizeof(double) * size_t(pad[j1]) * size_t(pad[j1]);
            if (j1 > j0 && bytes + b > cap) break;
            bytes += b;
            ++j1;
        }
        const int ns = j1 - j0;
        st->n_batches++;
        std::vector<int64_t> base(ns), ent0(ns + 1, 0);
        std::vector<int32_t> npad(ns), ndim(ns), scol(ns), scs(ns), ent_row, ent_soff, ent_sub;
        int64_t tot = 0;
        for (int q = 0; q < ns; ++q) {
            const int j = j0 + q;
            base[q] = tot;
            tot += int64_t(pad[j]) * pad[j];
            npad[q] = pad[j];
            ndim[q] = dim[j];
            scol[q] = j;
            scs[q] = csoff[j];
            int32_t off = 0;
            for (int64_t u = cp[j]; u < cp[j + 1]; ++u) {
                ent_row.push_back(crow[u]);
                ent_soff.push_back(off);
                ent_sub.push_back(q);
                off += H.h_rbs[crow[u]];
            }
            ent0[q + 1] = static_cast<int64_t>(ent_row.size());
        }
        const int64_t nent = static_cast<int64_t>(ent_row.size());
        int64_t *d_base = nullptr, *d_ent0 = nullptr;
        int32_t *d_npad = nullptr, *d_ndim = nullptr, *d_scol = nullptr, *d_scs = nullptr,
                *d_erow = nullptr, *d_esoff = nullptr, *d_esub = nullptr, *d_par = nullptr;
        double *buf0 = nullptr, *buf1 = nullptr, *ybuf = nullptr, *d_scale = nullptr,
               *d_r = nullptr, *d_part = nullptr;
        int4 *d_tiles = nullptr;
        int32_t *d_act = nullptr, *d_tlo = nullptr, *d_thi = nullptr;
        auto release = [&]() {
            dfree(d_base, s); dfree(d_ent0, s); dfree(d_npad, s); dfree(d_ndim, s);
            dfree(d_scol, s); dfree(d_scs, s); dfree(d_erow, s); dfree(d_esoff, s);
            dfree(d_esub, s); dfree(d_par, s); dfree(buf0, s); dfree(buf1, s); dfree(ybuf, s);
            dfree(d_scale, s); dfree(d_r, s); dfree(d_part, s); dfree(d_tiles, s);
            dfree(d_act, s); dfree(d_tlo, s); dfree(d_thi, s);
        };
        rc = upload(&d_base, base, s);
        if (rc == BSM_OK) rc = upload(&d_ent0, ent0, s);
        if (rc == BSM_OK) rc = upload(&d_npad, npad, s);
        if (rc == BSM_OK) rc = upload(&d_ndim, ndim, s);
        if (rc == BSM_OK) rc = upload(&d_scol, scol, s);
        if (rc == BSM_OK) rc = upload(&d_scs, scs, s);
        if (rc == BSM_OK) rc = upload(&d_erow, ent_row, s);
        if (rc == BSM_OK) rc = upload(&d_esoff, ent_soff, s);
        if (rc == BSM_OK) rc = upload(&d_esub, ent_sub, s);
        if (rc == BSM_OK) rc = dalloc(&buf0, static_cast<size_t>(tot), s);
        if (rc == BSM_OK) rc = dalloc(&buf1, static_cast<size_t>(tot), s);
        if (rc == BSM_OK) rc = dalloc(&ybuf, static_cast<size_t>(tot), s);
        if (rc == BSM_OK) rc = dalloc(&d_scale, static_cast<size_t>(ns), s);
        if (rc == BSM_OK) rc = dalloc(&d_r, static_cast<size_t>(ns), s);
        if (rc != BSM_OK) { release(); break; }

        // X_0 = (T - mu I) / ||T - mu I||_inf, zero padding
        if (hipMemsetAsync(buf0, 0, sizeof(double) * tot, s) != hipSuccess ||
            hipMemsetAsync(buf1, 0, sizeof(double) * tot, s) != hipSuccess) {
            set_error("submatrix: memset failed");
            rc = BSM_EDEVICE;
            release();
            break;
        }
        if (nent > 0)
            hipLaunchKernelGGL(k_sub_gather, dim3(static_cast<unsigned>(nent)), dim3(64), 0, s,
                               H.row_ptr, H.col_idx, H.blk_off, H.values, H.rbs, d_erow, d_esoff,
                               d_esub, d_ent0, d_base, d_npad, mu, buf0, nent);
        hipLaunchKernelGGL(k_sub_infnorm, dim3(ns), dim3(256), 0, s, buf0, d_base, d_npad, d_ndim,
                           d_scale);
        std::vector<double> scale(ns);
        if (hipMemcpyAsync(scale.data(), d_scale, sizeof(double) * ns, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            set_error("submatrix: %s", hipGetErrorString(hipGetLastError()));
            rc = BSM_EDEVICE;
            release();
            break;
        }
        for (int q = 0; q < ns && rc == BSM_OK; ++q) {
            if (!std::isfinite(scale[q])) {
                set_error("submatrix: H holds NaN or Inf (block column %d)", j0 + q);
                rc = BSM_ENONFINITE;
            } else if (scale[q] == 0.0) {
                set_error("submatrix: T - mu I is zero for block column %d", j0 + q);
                rc = BSM_EINVAL;
            }
        }
        if (rc != BSM_OK) { release(); break; }
        {
            int mxp = 0;
            for (int q = 0; q < ns; ++q) mxp = std::max(mxp, npad[q]);
            const unsigned gx = grid_for(int64_t(mxp) * mxp, 256 * 4);
            hipLaunchKernelGGL(k_sub_scale, dim3(gx, std::min(ns, 65535)), dim3(256), 0, s, buf0,
                               d_base, d_npad, d_scale, ns);
        }

        // Newton-Schulz on every submatrix of the batch
        std::vector<int32_t> parity(ns, 0), active;
        for (int q = 0; q < ns; ++q) active.push_back(q);
        std::vector<int> iters(ns, 0);
        std::vector<double> rfin(ns, 0.0);
        size_t tiles_cap = 0;
        for (int32_t k = 0; rc == BSM_OK && !active.empty(); ++k) {
            std::vector<int4> tiles;
            std::vector<int32_t> tlo, thi;
            for (int q : active) {
                const int nt = (npad[q] + kTile - 1) / kTile;
                tlo.push_back(static_cast<int32_t>(tiles.size()));
                for (int a = 0; a < nt; ++a)
                    for (int b = 0; b < nt; ++b) tiles.push_back(make_int4(q, a, b, parity[q]));
                thi.push_back(static_cast<int32_t>(tiles.size()));
            }
            if (tiles.size() > static_cast<size_t>(INT32_MAX / 2)) {
                set_error("submatrix: too many tiles in one batch");
                rc = BSM_EINVAL;
                break;
            }
            if (tiles.size() > tiles_cap) {
                dfree(d_tiles, s); dfree(d_part, s);
                d_tiles = nullptr; d_part = nullptr;
                tiles_cap = tiles.size();
                rc = dalloc(&d_tiles, tiles_cap, s);
                if (rc == BSM_OK) rc = dalloc(&d_part, tiles_cap, s);
                if (rc != BSM_OK) break;
            }
            dfree(d_act, s); dfree(d_tlo, s); dfree(d_thi, s);
            d_act = d_tlo = d_thi = nullptr;
            rc = upload(&d_act, active, s);
            if (rc == BSM_OK) rc = upload(&d_tlo, tlo, s);
            if (rc == BSM_OK) rc = upload(&d_thi, thi, s);
            if (rc != BSM_OK) break;
            if (hipMemcpyAsync(d_tiles, tiles.data(), sizeof(int4) * tiles.size(),
                               hipMemcpyHostToDevice, s) != hipSuccess) {
                set_error("submatrix: tile upload failed");
                rc = BSM_EDEVICE;
                break;
            }
            SubGemm g{d_tiles, static_cast<int32_t>(tiles.size()), d_base, d_npad, d_ndim,
                      buf0, buf1, ybuf, 0, d_part};
            const unsigned grid = static_cast<unsigned>((tiles.size() + kXcds - 1) / kXcds * kXcds);
            hipEvent_t e0, e1;
            (void)hipEventCreate(&e0);
            (void)hipEventCreate(&e1);
            (void)hipEventRecord(e0, s);
            hipLaunchKernelGGL(k_sub_gemm, dim3(grid), dim3(256), 0, s, g);       // Y = X X
            (void)hipEventRecord(e1, s);
            gev.emplace_back(e0, e1);
            for (int q : active) st->flops += 2.0 * double(ndim[q]) * ndim[q] * ndim[q];
            const int nact = static_cast<int>(active.size());
            hipLaunchKernelGGL(k_sub_resid, dim3(grid_for(nact, 128)), dim3(128), 0, s, d_part,
                               d_act, d_tlo, d_thi, d_ndim, d_r, nact);
            std::vector<double> r(nact);
            if (hipMemcpyAsync(r.data(), d_r, sizeof(double) * nact, hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                set_error("submatrix: %s", hipGetErrorString(hipGetLastError()));
                rc = BSM_EDEVICE;
                break;
            }
            std::vector<int32_t> next;
            for (int a = 0; a < nact; ++a) {
                const int q = active[a];
                rfin[q] = r[a];
                iters[q] = k;
                if (!std::isfinite(r[a])) {
                    set_error("submatrix: residual not finite (block column %d)", j0 + q);
                    rc = BSM_ENONFINITE;
                } else if (!(r[a] < o.tol)) {
                    next.push_back(q);
                }
            }
            if (rc != BSM_OK) break;
            if (next.empty()) { active.clear(); break; }
            if (k >= o.max_iter) {
                n_noconv += static_cast<int64_t>(next.size());   // keep their last iterates
                break;
            }
            // X' = 1.5 X - 0.5 X Y for those not yet converged (their tiles
            // only; the list is rebuilt in the order of `next`)
            if (next.size() != active.size()) {
                tiles.clear();
                for (int q : next) {
                    const int nt = (npad[q] + kTile - 1) / kTile;
                    for (int a = 0; a < nt; ++a)
                        for (int b = 0; b < nt; ++b) tiles.push_back(make_int4(q, a, b, parity[q]));
                }
                if (hipMemcpyAsync(d_tiles, tiles.data(), sizeof(int4) * tiles.size(),
                                   hipMemcpyHostToDevice, s) != hipSuccess) {
                    set_error("submatrix: tile upload failed");
                    rc = BSM_EDEVICE;
                    break;
                }
            }
            g.ntiles = static_cast<int32_t>(tiles.size());
            g.mode = 1;
            const unsigned grid2 = static_cast<unsigned>((tiles.size() + kXcds - 1) / kXcds * kXcds);
            hipEvent_t f0, f1;
            (void)hipEventCreate(&f0);
            (void)hipEventCreate(&f1);
            (void)hipEventRecord(f0, s);
            hipLaunchKernelGGL(k_sub_gemm, dim3(grid2), dim3(256), 0, s, g);
            (void)hipEventRecord(f1, s);
            gev.emplace_back(f0, f1);
            for (int q : next) {
                st->flops += 2.0 * double(ndim[q]) * ndim[q] * ndim[q];
                parity[q] ^= 1;
            }
            active.swap(next);
        }
        if (rc == BSM_OK) {
            for (int q = 0; q < ns; ++q) {
                st->max_iterations = std::max(st->max_iterations, iters[q]);
                st->r_max = std::max(st->r_max, rfin[q]);
            }
            int r2 = upload(&d_par, parity, s);
            if (r2 == BSM_OK && nent > 0)
                hipLaunchKernelGGL(k_sub_extract, dim3(static_cast<unsigned>(nent)), dim3(64), 0, s,
                                   P->row_ptr, P->col_idx, P->blk_off, P->rbs, d_erow, d_esoff,
                                   d_esub, d_scol, d_scs, d_base, d_npad, d_par, buf0, buf1,
                                   P->values, nent);
            if (r2 != BSM_OK) rc = r2;
        }
        release();
        if (rc != BSM_OK) break;
        j0 = j1;
    }
    if (rc == BSM_OK) {
        const int r2 = filter_inplace(*P, o.eps_filter, o.norm, s);
        if (r2 != BSM_OK) rc = r2;
    }
    if (rc == BSM_OK && n_noconv > 0) {
        set_error("submatrix: %lld submatrices above tol after max_iter",
                  static_cast<long long>(n_noconv));
        rc = BSM_ENOCONV;
    }
    (void)hipEventRecord(t1, s);
    (void)hipEventSynchronize(t1);
    float ms = 0.f;
    for (auto &p : gev) {
        if (hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess) st->gemm_ms += ms;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    if (hipEventElapsedTime(&ms, t0, t1) == hipSuccess) st->device_ms = ms;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (rc == BSM_OK || rc == BSM_ENOCONV) {
        st->nnzb = P->nnzb;
        *p_out = P;
    } else {
        free_mat(P, s);
    }
    return rc;
}

}  // namespace bsm
