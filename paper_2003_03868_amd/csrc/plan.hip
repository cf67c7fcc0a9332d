// Numeric-only repetition of a multiply from its retained symbolic state.
#include <algorithm>

#include "plan.h"

namespace bsm {

int run_op(const MulOp &op, hipStream_t s) {
    switch (op.kind) {
        case kOpVariant: return smm_launch(op.a, op.id, s);
        case kOpClass: return launch_class(op.a, op.id, s);
        case kOpRt: return launch_rt(op.a, op.prm, s);
        case kOpLowp: return smm_launch_lowp(op.a, s);
        case kOpQuad: return launch_quad(op.a, s);
        case kOpMQuad: return launch_mquad(op.a, s);
        default: set_error("internal: unknown launch kind %d", op.kind); return BSM_EINVAL;
    }
}

void free_plan(MulPlan *p) {
    if (!p) return;
    for (void *q : p->owned) dfree(q, p->s);
    delete p;
}

__global__ void k_zero_flag(int *f) { *f = 0; }

int zero_flag(int *f, hipStream_t s) {
    k_zero_flag<<<1, 1, 0, s>>>(f);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// The filter's decision for every unfiltered block, compared with the one
// the plan recorded (kidx[t+1] - kidx[t] is 1 for a kept block).
__global__ void k_keep_check(const double *sq, const double *mx, const int64_t *kidx, int64_t n,
                             double eps, int norm, int *flags) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const bool keep = (norm == BSM_NORM_MAXABS) ? !(mx[t] < eps) : !(sq[t] < eps * eps);
    const bool kept = kidx[t + 1] != kidx[t];
    if (keep != kept) atomicOr(flags, kFlagPattern);
}

// Values of the kept blocks into the filtered layout: one wave per block.
__global__ void __launch_bounds__(64)
k_gather_kept(const int64_t *kidx, const int64_t *koff, const int64_t *blk_off,
              const double *vals, int64_t n, double *out) {
    const int64_t t = blockIdx.x;
    if (t >= n || kidx[t + 1] == kidx[t]) return;
    const int64_t src = blk_off[t], len = blk_off[t + 1] - src, dst = koff[t];
    for (int64_t e = threadIdx.x; e < len; e += 64) out[dst + e] = vals[src + e];
}

int replay_multiply(MulPlan &p, const Mat &A, const Mat &B, const Mat *Cin, double *out,
                    int *flags, hipStream_t s) {
    if (A.nnzb != p.a_nnzb || B.nnzb != p.b_nnzb || A.nvalues != p.a_nval ||
        B.nvalues != p.b_nval || (p.use_c && (!Cin || Cin->nnzb != p.cin_nnzb))) {
        set_error("replay: operand patterns differ from the plan");
        return BSM_EINVAL;
    }
    if (p.nnzb_u == 0) return BSM_OK;
    if (p.prec != BSM_FP64) {
        BSM_TRY(pack_lowp(A.values, A.nvalues, p.apk, p.prec, s));
        if (!p.same_ab) BSM_TRY(pack_lowp(B.values, B.nvalues, p.bpk, p.prec, s));
    }
    double *cv = p.compacted ? p.c_vals_u : out;
    for (const MulOp &op : p.ops) {
        MulOp r = op;
        SmmArgs &a = r.a;
        a.a_col_idx = A.col_idx; a.a_blk_off = A.blk_off; a.a_vals = A.values; a.k_size = A.cbs;
        a.b_blk_off = B.blk_off; a.b_vals = B.values;
        a.c_rbs = A.rbs; a.c_cbs = B.cbs;
        a.cin_blk_off = p.use_c ? Cin->blk_off : nullptr;
        a.cin_vals = p.use_c ? Cin->values : nullptr;
        a.c_vals = cv;
        a.flags = flags;
        a.a_pk = p.apk;
        a.b_pk = p.same_ab ? p.apk : p.bpk;
        BSM_TRY(run_op(r, s));
    }
    if (p.eps > 0.0) {
        k_keep_check<<<grid_for(p.nnzb_u, 256), 256, 0, s>>>(p.sq, p.mx, p.kidx, p.nnzb_u, p.eps,
                                                             p.norm, flags);
        if (p.compacted)
            k_gather_kept<<<static_cast<unsigned>(p.nnzb_u), 64, 0, s>>>(
                p.kidx, p.koff, p.c_blk_off_u, p.c_vals_u, p.nnzb_u, out);
    }
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

int refilter(const MulPlan &p, const double *vals_u, Mat &m, hipStream_t s) {
    int64_t *rp = nullptr, *bo = nullptr;
    int32_t *ci = nullptr;
    double *v = nullptr;
    int st = dalloc(&rp, m.nbrows + 1, s);
    if (st == BSM_OK) st = dalloc(&ci, p.nnzb_u, s);
    if (st == BSM_OK) st = dalloc(&bo, p.nnzb_u + 1, s);
    if (st == BSM_OK) st = dalloc(&v, p.nval_u, s);
    hipError_t e = hipSuccess;
    if (st == BSM_OK) {
        e = hipMemcpyAsync(rp, p.c_row_ptr_u, sizeof(int64_t) * (m.nbrows + 1), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && p.nnzb_u)
            e = hipMemcpyAsync(ci, p.c_col_u, sizeof(int32_t) * p.nnzb_u, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(bo, p.c_blk_off_u, sizeof(int64_t) * (p.nnzb_u + 1), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && p.nval_u)
            e = hipMemcpyAsync(v, vals_u, sizeof(double) * p.nval_u, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) { set_error("refilter: %s", hipGetErrorString(e)); st = BSM_EDEVICE; }
    }
    if (st != BSM_OK) {
        dfree(rp, s); dfree(ci, s); dfree(bo, s); dfree(v, s);
        return st;
    }
    free_mat_arrays(m, s);
    m.row_ptr = rp; m.col_idx = ci; m.blk_off = bo; m.values = v;
    m.nnzb = p.nnzb_u;
    m.nvalues = p.nval_u;
    int64_t after = 0;
    return compact_by_norm(m, p.sq, p.mx, p.eps, p.norm, s, &after);
}

__global__ void k_pattern_diff(const int64_t *rp_a, const int32_t *ci_a, const int64_t *rp_b,
                               const int32_t *ci_b, int32_t nbrows, int64_t nnzb, int *diff) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    bool d = false;
    if (t <= nbrows && rp_a[t] != rp_b[t]) d = true;
    if (t < nnzb && ci_a[t] != ci_b[t]) d = true;
    if (d) atomicOr(diff, 1);
}

int pattern_differs(const int64_t *rp_a, const int32_t *ci_a, const int64_t *rp_b,
                    const int32_t *ci_b, int32_t nbrows, int64_t nnzb, int *diff, hipStream_t s) {
    BSM_TRY(zero_flag(diff, s));
    const int64_t n = std::max<int64_t>(nnzb, static_cast<int64_t>(nbrows) + 1);
    k_pattern_diff<<<grid_for(n, 256), 256, 0, s>>>(rp_a, ci_a, rp_b, ci_b, nbrows, nnzb, diff);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

}  // namespace bsm
