// Online solve of Section 4.1: f^ = F K~^* u (direct) and FP64 iterative
// refinement f <- f + F K~^*_prec (u - K~ f) for the low-precision applies.
#include "bf.h"

#include <cmath>

struct hss_ulv_s;

namespace fio {
void ulv_solve_impl(hss_ulv_s *f, const double2 *Y, long ldy, double2 *C, long ldc, int nrhs, void *ws, hipStream_t s);
size_t ulv_ws_bytes_pub(const hss_ulv_s *f, int nrhs);

// R = U - R (in place), N x nrhs blocks
__global__ void k_resid(const double2 *__restrict__ U, long ldu, double2 *__restrict__ R, long ldr, long n, int nrhs) {
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= (size_t)n * nrhs) return;
    long i = id % n;
    int j = id / n;
    double2 u = U[i + (size_t)j * ldu], r = R[i + (size_t)j * ldr];
    R[i + (size_t)j * ldr] = zc(u.x - r.x, u.y - r.y);
}

// F += D
__global__ void k_axpy(double2 *__restrict__ F, long ldf, const double2 *__restrict__ D, long ldd, long n, int nrhs) {
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= (size_t)n * nrhs) return;
    long i = id % n;
    int j = id / n;
    double2 a = F[i + (size_t)j * ldf], b = D[i + (size_t)j * ldd];
    F[i + (size_t)j * ldf] = zc(a.x + b.x, a.y + b.y);
}

// out[j] = sum_i |X(i, j)|^2, one workgroup per column (fixed reduction order)
__global__ void k_colnorm2(const double2 *__restrict__ X, long ldx, long n, double *out) {
    __shared__ double sh[4];
    const int j = blockIdx.x;
    double p = 0.0;
    for (long i = threadIdx.x; i < n; i += blockDim.x) {
        double2 v = X[i + (size_t)j * ldx];
        p += v.x * v.x + v.y * v.y;
    }
    for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = p;
    __syncthreads();
    if (threadIdx.x == 0) out[j] = sh[0] + sh[1] + sh[2] + sh[3];
}

struct SolveWs {
    double2 *t, *R;
    void *bfws, *ulvws;
    double *nrm;
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t solve_ws_bytes(fio_bf_s *bf, hss_ulv_s *f, int nrhs, const fio_solve_opts *o) {
    size_t blk = align256((size_t)bf->N * nrhs * sizeof(double2));
    size_t bfw = bf_ws_bytes(bf, nrhs, (fio_prec)o->prec);
    size_t b64 = bf_ws_bytes(bf, nrhs, FIO_PREC_FP64);
    if (o->mode == FIO_SOLVE_IR && b64 > bfw) bfw = b64;
    return 2 * blk + align256(bfw) + align256(ulv_ws_bytes_pub(f, nrhs)) + align256(2 * nrhs * sizeof(double)) + 256;
}

static SolveWs carve(fio_bf_s *bf, hss_ulv_s *f, int nrhs, const fio_solve_opts *o, void *ws) {
    char *p = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    SolveWs w;
    size_t blk = align256((size_t)bf->N * nrhs * sizeof(double2));
    w.t = (double2 *)p;
    p += blk;
    w.R = (double2 *)p;
    p += blk;
    w.bfws = p;
    size_t bfw = bf_ws_bytes(bf, nrhs, (fio_prec)o->prec);
    size_t b64 = bf_ws_bytes(bf, nrhs, FIO_PREC_FP64);
    if (o->mode == FIO_SOLVE_IR && b64 > bfw) bfw = b64;
    p += align256(bfw);
    w.ulvws = p;
    p += align256(ulv_ws_bytes_pub(f, nrhs));
    w.nrm = (double *)p;
    return w;
}

static fio_status solve_impl(fio_bf_s *bf, hss_ulv_s *f, const double2 *U, long ldu, double2 *F, long ldf, int nrhs,
                             const fio_solve_opts *o, fio_solve_info *info, void *ws, hipStream_t s) {
    SolveWs w = carve(bf, f, nrhs, o, ws);
    const long N = bf->N;
    const fio_prec lp = (fio_prec)o->prec;
    const unsigned TB = 256;
    const size_t ne = (size_t)N * nrhs;
    // 2D: the HSS factorization F lives in the Morton order of the frequencies, so K~^*
    // writes that order and the solution is mapped back to the user's order
    const bool d2 = bf->dim == 2;
    // f0 = F K~^*_prec u
    bf_apply_impl(bf, true, U, ldu, w.t, N, nrhs, lp, w.bfws, s, d2);
    if (d2) {
        ulv_solve_impl(f, w.t, N, w.t, N, nrhs, w.ulvws, s);
        permute2d((int)bf->n1, false, w.t, N, F, ldf, nrhs, s);
    } else {
        ulv_solve_impl(f, w.t, N, F, ldf, nrhs, w.ulvws, s);
    }
    if (info) {
        info->ir_steps = 0;
        info->rel_res = -1.0;
    }
    if (o->mode != FIO_SOLVE_IR) return FIO_OK;
    std::vector<double> hn(2 * nrhs);
    if (o->rel_res_tol > 0.0) k_colnorm2<<<nrhs, 256, 0, s>>>(U, ldu, N, w.nrm + nrhs);
    for (int step = 0;; ++step) {
        const bool measure = o->rel_res_tol > 0.0;
        if (!measure && step == o->max_ir) break;
        // R = u - K~ f in FP64
        bf_apply_impl(bf, false, F, ldf, w.R, N, nrhs, FIO_PREC_FP64, w.bfws, s);
        k_resid<<<grid1d(ne, TB), TB, 0, s>>>(U, ldu, w.R, N, N, nrhs);
        if (measure) {
            k_colnorm2<<<nrhs, 256, 0, s>>>(w.R, N, N, w.nrm);
            FIO_HIP(hipMemcpyAsync(hn.data(), w.nrm, 2 * nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
            FIO_HIP(hipStreamSynchronize(s));
            double worst = 0.0;
            for (int j = 0; j < nrhs; ++j) {
                double den = hn[nrhs + j] > 0.0 ? hn[nrhs + j] : 1.0;
                double v = std::sqrt(hn[j] / den);
                worst = v > worst ? v : worst;
            }
            if (info) {
                info->ir_steps = step;
                info->rel_res = worst;
            }
            if (worst <= o->rel_res_tol) return FIO_OK;
            if (step == o->max_ir) return FIO_ERR_NOT_CONVERGED;
        }
        // f += F K~^*_prec r
        bf_apply_impl(bf, true, w.R, N, w.t, N, nrhs, lp, w.bfws, s, d2);
        ulv_solve_impl(f, w.t, N, w.t, N, nrhs, w.ulvws, s);
        if (d2) {
            permute2d((int)bf->n1, false, w.t, N, w.R, N, nrhs, s);
            k_axpy<<<grid1d(ne, TB), TB, 0, s>>>(F, ldf, w.R, N, N, nrhs);
        } else {
            k_axpy<<<grid1d(ne, TB), TB, 0, s>>>(F, ldf, w.t, N, N, nrhs);
        }
        if (info && !measure) info->ir_steps = step + 1;
    }
    FIO_HIP(hipGetLastError());
    return FIO_OK;
}

}  // namespace fio

using namespace fio;

struct hss_ulv_s;

extern "C" fio_status fio_solve_workspace_size(fio_bf_t bf, hss_ulv_t f, int nrhs, const fio_solve_opts *opts,
                                               size_t *bytes) {
    FIO_CHECK_ARG(bf && f && opts && bytes && nrhs >= 0);
    *bytes = solve_ws_bytes(bf, f, nrhs, opts);
    return FIO_OK;
}

extern "C" fio_status fio_approx_solve(fio_bf_t bf, hss_ulv_t f, const void *U, long ldu, void *F, long ldf, int nrhs,
                                       const fio_solve_opts *opts, fio_solve_info *info, void *ws, size_t ws_bytes,
                                       void *stream) {
    FIO_CHECK_ARG(bf && f && opts && nrhs >= 0);
    if (nrhs == 0) return FIO_OK;
    FIO_CHECK_ARG(U && F && U != F && ldu >= bf->N && ldf >= bf->N);
    FIO_CHECK_ARG(opts->mode == FIO_SOLVE_DIRECT || opts->mode == FIO_SOLVE_IR);
    FIO_CHECK_ARG(opts->prec >= FIO_PREC_FP64 && opts->prec <= FIO_PREC_SPLIT_FP16);
    FIO_CHECK_ARG(opts->max_ir >= 0);
    if (opts->prec == FIO_PREC_FP32 && !bf->f32.p) return FIO_ERR_ARG;
    if (opts->prec == FIO_PREC_SPLIT_FP16 && !bf->f16.p) return FIO_ERR_ARG;
    size_t need = solve_ws_bytes(bf, f, nrhs, opts);
    FIO_CHECK_ARG(ws && ws_bytes >= need);
    return guarded([&] {
        return solve_impl(bf, f, (const double2 *)U, ldu, (double2 *)F, ldf, nrhs, opts, info, ws, as_stream(stream));
    });
}
