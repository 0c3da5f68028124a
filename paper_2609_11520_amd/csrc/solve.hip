// Online solve of Section 4.1: f^ = F K~^* u (direct) and FP64 iterative
// refinement f <- f + F K~^*_prec (u - K~ f) for the low-precision applies.
#include "bf.h"

#include <cmath>
#include <vector>

struct hss_ulv_s;

namespace fio {
void ulv_solve_impl(hss_ulv_s *f, const double2 *Y, long ldy, double2 *C, long ldc, int nrhs, void *ws, hipStream_t s,
                    bool accumulate = false);
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
// Column reductions in two stages with a fixed order: each column is cut into kRedChunks
// row ranges (the cut depends on n only, so a column's result does not depend on the
// other columns of the batch), one workgroup reduces a range into a partial, and one wave
// per column sums the partials.
constexpr int kRedChunks = 32;

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// part[j kRedChunks + c] = sum over rows of chunk c of |X(i, j)|^2
__global__ void __launch_bounds__(256) k_colnorm2_part(const double2 *__restrict__ X, long ldx, long n,
                                                      double *__restrict__ part) {
    __shared__ double sh[4];
    const int c = blockIdx.x % kRedChunks, j = blockIdx.x / kRedChunks, t = threadIdx.x;
    const long len = (n + kRedChunks - 1) / kRedChunks;
    const long i0 = c * len, i1 = i0 + len < n ? i0 + len : n;
    const double2 *x = X + (size_t)j * ldx;
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    for (long i = i0 + t; i < i1; i += 1024) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long r = i + 256 * u;
            if (r < i1) {
                const double2 v = x[r];
                p[u] += v.x * v.x + v.y * v.y;
            }
        }
    }
    const double w = wave_sum((p[0] + p[1]) + (p[2] + p[3]));
    if ((t & 63) == 0) sh[t >> 6] = w;
    __syncthreads();
    if (t == 0) part[(size_t)j * kRedChunks + c] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// part[j kRedChunks + c] = sum over rows of chunk c of conj(A(i, j)) B(i, j)
__global__ void __launch_bounds__(256) k_coldot_part(const double2 *__restrict__ A, long lda,
                                                    const double2 *__restrict__ B, long ldb, long n,
                                                    double2 *__restrict__ part) {
    __shared__ double shr[4], shi[4];
    const int c = blockIdx.x % kRedChunks, j = blockIdx.x / kRedChunks, t = threadIdx.x;
    const long len = (n + kRedChunks - 1) / kRedChunks;
    const long i0 = c * len, i1 = i0 + len < n ? i0 + len : n;
    const double2 *a = A + (size_t)j * lda, *b = B + (size_t)j * ldb;
    double pr[4] = {0.0, 0.0, 0.0, 0.0}, pi[4] = {0.0, 0.0, 0.0, 0.0};
    for (long i = i0 + t; i < i1; i += 1024) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long r = i + 256 * u;
            if (r < i1) {
                const double2 av = a[r], bv = b[r];
                pr[u] += av.x * bv.x + av.y * bv.y;
                pi[u] += av.x * bv.y - av.y * bv.x;
            }
        }
    }
    const double wr = wave_sum((pr[0] + pr[1]) + (pr[2] + pr[3]));
    const double wi = wave_sum((pi[0] + pi[1]) + (pi[2] + pi[3]));
    if ((t & 63) == 0) {
        shr[t >> 6] = wr;
        shi[t >> 6] = wi;
    }
    __syncthreads();
    if (t == 0) part[(size_t)j * kRedChunks + c] = zc((shr[0] + shr[1]) + (shr[2] + shr[3]),
                                                      (shi[0] + shi[1]) + (shi[2] + shi[3]));
}

// out[j] = sum_c part[j kRedChunks + c], one wave per column
__global__ void __launch_bounds__(64) k_colsum(const double *__restrict__ part, double *__restrict__ out) {
    const int j = blockIdx.x, t = threadIdx.x;
    const double v = wave_sum(t < kRedChunks ? part[(size_t)j * kRedChunks + t] : 0.0);
    if (t == 0) out[j] = v;
}

__global__ void __launch_bounds__(64) k_colsum2(const double2 *__restrict__ part, double2 *__restrict__ out) {
    const int j = blockIdx.x, t = threadIdx.x;
    const double2 p = t < kRedChunks ? part[(size_t)j * kRedChunks + t] : zc(0.0, 0.0);
    const double vr = wave_sum(p.x), vi = wave_sum(p.y);
    if (t == 0) out[j] = zc(vr, vi);
}

// out[j] = ||X(:, j)||^2 for j < nrhs; part holds nrhs * kRedChunks doubles
static void colnorm2(const double2 *X, long ldx, long n, int nrhs, double *part, double *out, hipStream_t s) {
    k_colnorm2_part<<<(unsigned)nrhs * kRedChunks, 256, 0, s>>>(X, ldx, n, part);
    k_colsum<<<nrhs, 64, 0, s>>>(part, out);
}

// out[j] = A(:, j)^* B(:, j) for j < nrhs; part holds nrhs * kRedChunks complex values
static void coldot(const double2 *A, long lda, const double2 *B, long ldb, long n, int nrhs, double2 *part,
                   double2 *out, hipStream_t s) {
    k_coldot_part<<<(unsigned)nrhs * kRedChunks, 256, 0, s>>>(A, lda, B, ldb, n, part);
    k_colsum2<<<nrhs, 64, 0, s>>>(part, out);
}

__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return zc((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// CG step: alpha_j = rz_j / pAp_j; X += alpha P; R -= alpha AP (column j of each block)
__global__ void k_cg_step(double2 *__restrict__ X, long ldx, double2 *__restrict__ R, const double2 *__restrict__ P,
                          const double2 *__restrict__ AP, long ld, long n, int nrhs, const double2 *__restrict__ rz,
                          const double2 *__restrict__ pap) {
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= (size_t)n * nrhs) return;
    const long i = id % n;
    const int j = id / n;
    const double2 al = zdiv(rz[j], pap[j]);
    const size_t e = i + (size_t)j * ld;
    const double2 pv = P[e], av = AP[e];
    double2 &x = X[i + (size_t)j * ldx];
    x = zc(x.x + al.x * pv.x - al.y * pv.y, x.y + al.x * pv.y + al.y * pv.x);
    double2 &r = R[e];
    r = zc(r.x - (al.x * av.x - al.y * av.y), r.y - (al.x * av.y + al.y * av.x));
}

// direction update: beta_j = rz_new_j / rz_j; P = Z + beta P
__global__ void k_cg_dir(double2 *__restrict__ P, const double2 *__restrict__ Z, long ld, long n, int nrhs,
                         const double2 *__restrict__ rz_new, const double2 *__restrict__ rz) {
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= (size_t)n * nrhs) return;
    const long i = id % n;
    const int j = id / n;
    const double2 be = zdiv(rz_new[j], rz[j]);
    const size_t e = i + (size_t)j * ld;
    const double2 pv = P[e], zv = Z[e];
    P[e] = zc(zv.x + be.x * pv.x - be.y * pv.y, zv.y + be.x * pv.y + be.y * pv.x);
}

__global__ void k_zero(double2 *__restrict__ X, long ldx, long n, int nrhs) {
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= (size_t)n * nrhs) return;
    X[id % n + (size_t)(id / n) * ldx] = zc(0.0, 0.0);
}

__global__ void k_copy(double2 *__restrict__ Y, const double2 *__restrict__ X, long ld, long n, int nrhs) {
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= (size_t)n * nrhs) return;
    const size_t e = id % n + (size_t)(id / n) * ld;
    Y[e] = X[e];
}

struct SolveWs {
    double2 *t, *R;
    void *bfws, *ulvws;
    double *nrm;
    double *part;                      // partials of the column reductions
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t pcg_ws_bytes(fio_bf_s *bf, hss_ulv_s *f, int nrhs) {
    const size_t blk = align256((size_t)bf->N * nrhs * sizeof(double2));
    return 5 * blk + align256(bf_ws_bytes(bf, nrhs, FIO_PREC_FP64)) + align256(ulv_ws_bytes_pub(f, nrhs)) +
           align256(3 * nrhs * sizeof(double2)) + align256(2 * nrhs * sizeof(double)) +
           align256((size_t)nrhs * kRedChunks * sizeof(double2)) + 256;
}

static size_t solve_ws_bytes(fio_bf_s *bf, hss_ulv_s *f, int nrhs, const fio_solve_opts *o) {
    if (o->mode == FIO_SOLVE_PCG) return pcg_ws_bytes(bf, f, nrhs);
    size_t blk = align256((size_t)bf->N * nrhs * sizeof(double2));
    size_t bfw = bf_ws_bytes(bf, nrhs, (fio_prec)o->prec);
    size_t b64 = bf_ws_bytes(bf, nrhs, FIO_PREC_FP64);
    if (o->mode == FIO_SOLVE_IR && b64 > bfw) bfw = b64;
    return 2 * blk + align256(bfw) + align256(ulv_ws_bytes_pub(f, nrhs)) + align256(2 * nrhs * sizeof(double)) +
           align256((size_t)nrhs * kRedChunks * sizeof(double)) + 256;
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
    p += align256(2 * nrhs * sizeof(double));
    w.part = (double *)p;
    return w;
}

// Preconditioned CG on the normal equation K~^* K~ f = K~^* u (Section 4.1, eq.
// fio_approx_normal_eq) with G~^{-1} (the ULV solve) as the preconditioner, from f = 0,
// every right-hand side its own recurrence; all applies in FP64.  2D: the iteration runs
// in the Morton order of the frequencies (the order of G~) and the result is mapped back.
static fio_status pcg_impl(fio_bf_s *bf, hss_ulv_s *f, const double2 *U, long ldu, double2 *F, long ldf, int nrhs,
                           const fio_solve_opts *o, fio_solve_info *info, void *ws, hipStream_t s) {
    const long N = bf->N;
    const bool d2 = bf->dim == 2;
    const size_t blk = align256((size_t)N * nrhs * sizeof(double2));
    char *q = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    double2 *R = (double2 *)q, *Z = (double2 *)(q + blk), *P = (double2 *)(q + 2 * blk),
            *AP = (double2 *)(q + 3 * blk), *XT = (double2 *)(q + 4 * blk);
    q += 5 * blk;
    void *bfws = q;
    q += align256(bf_ws_bytes(bf, nrhs, FIO_PREC_FP64));
    void *ulvws = q;
    q += align256(ulv_ws_bytes_pub(f, nrhs));
    double2 *rz[2] = {(double2 *)q, (double2 *)q + nrhs};
    double2 *pap = (double2 *)q + 2 * nrhs;
    q += align256(3 * nrhs * sizeof(double2));
    double *nrm = (double *)q;             // [0, nrhs): ||r_j||^2, [nrhs, 2 nrhs): ||b_j||^2
    q += align256(2 * nrhs * sizeof(double));
    double2 *part = (double2 *)q;          // partials of the column reductions
    const unsigned TB = 256;
    const size_t ne = (size_t)N * nrhs;
    const unsigned g = grid1d(ne, TB);
    double2 *X = d2 ? XT : F;
    const long ldxx = d2 ? N : ldf;
    const bool measure = o->rel_res_tol > 0.0;
    std::vector<double> hn(measure ? 2 * nrhs : 0);   // host copy of the norms (only when measuring)
    if (info) {
        info->ir_steps = 0;
        info->rel_res = -1.0;
    }
    // r = b = K~^* u, x = 0, z = G~^{-1} r, p = z
    bf_apply_impl(bf, true, U, ldu, R, N, nrhs, FIO_PREC_FP64, bfws, s, d2);
    if (measure) colnorm2(R, N, N, nrhs, (double *)part, nrm + nrhs, s);
    k_zero<<<g, TB, 0, s>>>(X, ldxx, N, nrhs);
    ulv_solve_impl(f, R, N, Z, N, nrhs, ulvws, s);
    coldot(R, N, Z, N, N, nrhs, part, rz[0], s);
    k_copy<<<g, TB, 0, s>>>(P, Z, N, N, nrhs);
    int cur = 0;
    fio_status st = FIO_OK;
    for (int it = 1; it <= o->max_ir; ++it) {
        // A p = K~^* (K~ p), K~ p staged in Z
        bf_apply_impl(bf, false, P, N, Z, N, nrhs, FIO_PREC_FP64, bfws, s, d2);
        bf_apply_impl(bf, true, Z, N, AP, N, nrhs, FIO_PREC_FP64, bfws, s, d2);
        coldot(P, N, AP, N, N, nrhs, part, pap, s);
        k_cg_step<<<g, TB, 0, s>>>(X, ldxx, R, P, AP, N, N, nrhs, rz[cur], pap);
        if (info) info->ir_steps = it;
        if (measure) {
            colnorm2(R, N, N, nrhs, (double *)part, nrm, s);
            FIO_HIP(hipMemcpyAsync(hn.data(), nrm, 2 * nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
            FIO_HIP(hipStreamSynchronize(s));
            double worst = 0.0;
            for (int j = 0; j < nrhs; ++j) {
                const double den = hn[nrhs + j] > 0.0 ? hn[nrhs + j] : 1.0;
                const double v = std::sqrt(hn[j] / den);
                worst = v > worst ? v : worst;
            }
            if (info) info->rel_res = worst;
            if (worst <= o->rel_res_tol) break;
            if (it == o->max_ir) st = FIO_ERR_NOT_CONVERGED;
        }
        if (it == o->max_ir) break;
        ulv_solve_impl(f, R, N, Z, N, nrhs, ulvws, s);
        coldot(R, N, Z, N, N, nrhs, part, rz[1 - cur], s);
        k_cg_dir<<<g, TB, 0, s>>>(P, Z, N, N, nrhs, rz[1 - cur], rz[cur]);
        cur = 1 - cur;
    }
    if (d2) permute2d((int)bf->n1, false, XT, N, F, ldf, nrhs, s);
    FIO_HIP(hipGetLastError());
    return st;
}

static fio_status solve_impl(fio_bf_s *bf, hss_ulv_s *f, const double2 *U, long ldu, double2 *F, long ldf, int nrhs,
                             const fio_solve_opts *o, fio_solve_info *info, void *ws, hipStream_t s) {
    if (o->mode == FIO_SOLVE_PCG) return pcg_impl(bf, f, U, ldu, F, ldf, nrhs, o, info, ws, s);
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
    std::vector<double> hn(o->rel_res_tol > 0.0 ? 2 * nrhs : 0);   // host copy of the norms (only when measuring)
    if (o->rel_res_tol > 0.0) colnorm2(U, ldu, N, nrhs, w.part, w.nrm + nrhs, s);
    for (int step = 0;; ++step) {
        const bool measure = o->rel_res_tol > 0.0;
        if (!measure && step == o->max_ir) break;
        // R = u - K~ f in FP64
        if (!bf_residual_f64(bf, F, ldf, U, ldu, w.R, N, nrhs, w.bfws, s)) {
            bf_apply_impl(bf, false, F, ldf, w.R, N, nrhs, FIO_PREC_FP64, w.bfws, s);
            k_resid<<<grid1d(ne, TB), TB, 0, s>>>(U, ldu, w.R, N, N, nrhs);
        }
        if (measure) {
            colnorm2(w.R, N, N, nrhs, w.part, w.nrm, s);
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
        // f += F K~^*_prec r (1D: the ULV solve's last level adds to f)
        bf_apply_impl(bf, true, w.R, N, w.t, N, nrhs, lp, w.bfws, s, d2);
        if (d2) {
            ulv_solve_impl(f, w.t, N, w.t, N, nrhs, w.ulvws, s);
            permute2d((int)bf->n1, false, w.t, N, w.R, N, nrhs, s);
            k_axpy<<<grid1d(ne, TB), TB, 0, s>>>(F, ldf, w.R, N, N, nrhs);
        } else {
            ulv_solve_impl(f, w.t, N, F, ldf, nrhs, w.ulvws, s, true);
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
    FIO_CHECK_ARG(opts->mode == FIO_SOLVE_DIRECT || opts->mode == FIO_SOLVE_IR || opts->mode == FIO_SOLVE_PCG);
    FIO_CHECK_ARG(opts->mode != FIO_SOLVE_PCG || opts->prec == FIO_PREC_FP64);
    FIO_CHECK_ARG(opts->prec >= FIO_PREC_FP64 && opts->prec <= FIO_PREC_SPLIT_FP16);
    FIO_CHECK_ARG(opts->max_ir >= 0);
    if (opts->prec == FIO_PREC_FP32 && !bf->f32.p) return FIO_ERR_ARG;
    if (opts->prec == FIO_PREC_SPLIT_FP16 && !bf->split16) return FIO_ERR_ARG;
    size_t need = solve_ws_bytes(bf, f, nrhs, opts);
    FIO_CHECK_ARG(ws && ws_bytes >= need);
    return guarded([&] {
        return solve_impl(bf, f, (const double2 *)U, ldu, (double2 *)F, ldf, nrhs, opts, info, ws, as_stream(stream));
    });
}

// ---------------------------------------------------------------------------
// The solve without any allocation: its workspace is a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes the array's name (a host-side
// stand-in) to a kernel: the device address comes from hipGetSymbolAddress, taken once per
// device with that device current and kept per device.  Nothing in the workspace has to start
// at zero (every solve writes each buffer before reading it), and calls that overlap on one GPU
// share the array and race.
namespace {
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

fio_status static_scratch(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FIO_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            fprintf(stderr, "fiohss: hipGetSymbolAddress(scratch) failed on device %d: %s\n", dev,
                    hipGetErrorString(e));
            return FIO_ERR_HIP;
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return FIO_OK;
}
}  // namespace

extern "C" size_t fio_approx_solve_static_max_bytes(void) { return kStaticScratchBytes; }

extern "C" fio_status fio_approx_solve_static(fio_bf_t bf, hss_ulv_t f, const void *U, long ldu, void *F, long ldf,
                                              int nrhs, const fio_solve_opts *opts, fio_solve_info *info,
                                              void *stream) {
    FIO_CHECK_ARG(bf && f && opts && nrhs >= 0);
    if (nrhs == 0) return FIO_OK;
    FIO_CHECK_ARG(U && F && U != F && ldu >= bf->N && ldf >= bf->N);
    FIO_CHECK_ARG(opts->mode == FIO_SOLVE_DIRECT || opts->mode == FIO_SOLVE_IR || opts->mode == FIO_SOLVE_PCG);
    FIO_CHECK_ARG(opts->mode != FIO_SOLVE_PCG || opts->prec == FIO_PREC_FP64);
    FIO_CHECK_ARG(opts->prec >= FIO_PREC_FP64 && opts->prec <= FIO_PREC_SPLIT_FP16);
    FIO_CHECK_ARG(opts->max_ir >= 0);
    // a fixed step count: the residual-checked forms read norms back into host memory
    FIO_CHECK_ARG(opts->mode == FIO_SOLVE_DIRECT || opts->rel_res_tol <= 0.0);
    if (opts->prec == FIO_PREC_FP32 && !bf->f32.p) return FIO_ERR_ARG;
    if (opts->prec == FIO_PREC_SPLIT_FP16 && !bf->split16) return FIO_ERR_ARG;
    const size_t need = solve_ws_bytes(bf, f, nrhs, opts);
    if (need > kStaticScratchBytes) {
        fprintf(stderr, "fiohss: fio_approx_solve_static: %d columns at N = %ld need %zu bytes of workspace, "
                        "more than its %zu-byte scratch array\n", nrhs, bf->N, need, kStaticScratchBytes);
        return FIO_ERR_ARG;
    }
    void *ws = nullptr;
    const fio_status st = static_scratch(&ws);
    if (st != FIO_OK) return st;
    return guarded([&] {
        return solve_impl(bf, f, (const double2 *)U, ldu, (double2 *)F, ldf, nrhs, opts, info, ws, as_stream(stream));
    });
}
