// Butterfly factorization of a 1D discrete FIO on gfx950 (Section 2.2):
// on-device evaluation of the explicit factors and their batched apply.
//
// Factor layout (complex entries, all row-major blocks), identical to the
// import layout documented with fio_bf_import:
//   V[sigma][tau][j][s], C^[L'] .. C^[h+1] (each (N/2) x 2q x 2q), M[p][i][j],
//   B^[h+1] .. B^[L'] (each (N/2) x 2q x 2q), U[tau][sigma][s][i].
// Coefficient buffers: entry (pair p, coefficient i, column col) at
//   (p * q + i) * nrhs + col, so that consecutive lanes of a wave work on
//   consecutive right-hand sides of the same pair.
#include "bf.h"
#include "timing.h"

#include <cmath>
#include <cstring>

namespace fio {

// Points per leaf box: N / 2^L' = 8 for every N >= 64 when L' = L - 3.
constexpr int kLeafPts = 8;

// ---------------------------------------------------------------------------
// geometry
fio_status bf_plan(const fio_bf_desc *d, fio_bf_s *bf) {
    if (!d || d->dim != 1) return d ? FIO_ERR_UNSUPPORTED : FIO_ERR_ARG;
    if (d->n < 64 || (d->n & (d->n - 1))) return FIO_ERR_ARG;
    int L = 0;
    while ((1L << L) < d->n) ++L;
    if (L % 2) return FIO_ERR_UNSUPPORTED;
    if (d->q < 2 || d->q > 16 || d->level_offset < 1) return FIO_ERR_ARG;
    bf->desc = *d;
    bf->N = d->n;
    bf->L = L;
    bf->h = L / 2;
    bf->Lp = (L - d->level_offset > bf->h) ? L - d->level_offset : bf->h;
    bf->nl = bf->Lp - bf->h;
    bf->q = d->q;
    bf->b = (int)(d->n >> bf->Lp);
    bf->nsl = 1 << (L - bf->Lp);
    if (bf->b != kLeafPts) return FIO_ERR_UNSUPPORTED;
    const size_t q = bf->q, N = bf->N;
    size_t off = 0;
    bf->offV = off;
    off += (size_t)(1L << bf->Lp) * bf->nsl * q * bf->b;
    bf->offC.assign(bf->nl, 0);
    for (int lev = bf->nl - 1; lev >= 0; --lev) {
        bf->offC[lev] = off;
        off += (N / 2) * 4 * q * q;
    }
    bf->offM = off;
    off += N * q * q;
    bf->offB.assign(bf->nl, 0);
    for (int lev = 0; lev < bf->nl; ++lev) {
        bf->offB[lev] = off;
        off += (N / 2) * 4 * q * q;
    }
    bf->offU = off;
    off += (size_t)(1L << bf->Lp) * bf->nsl * bf->b * q;
    bf->total = off;
    return FIO_OK;
}

size_t bf_coef_elems(const fio_bf_s *bf, int nrhs) { return (size_t)bf->N * bf->q * (size_t)nrhs; }

// ---------------------------------------------------------------------------
// factor evaluation (Section 2.2).  Phase differences are formed as
// differences (centers are exact binary fractions / integers), so an entry's
// phase carries only the rounding of O(1)-sized terms; M's full phase keeps
// its large exact parts exact (integer products and two-product splits).
struct Geo {
    long N;
    int L, h, Lp, q, b, nsl;
    double c0, c1;
};

__device__ __forceinline__ double cheb_t(int i, int q) { return cospi((2.0 * i + 1.0) / (2.0 * q)); }

// Lagrange basis of node t on the reference first-kind grid, at u in [-1, 1].
__device__ double lagr(double u, int t, int q) {
    double tt = cheb_t(t, q), p = 1.0;
    for (int k = 0; k < q; ++k) {
        if (k == t) continue;
        double tk = cheb_t(k, q);
        p *= (u - tk) / (tt - tk);
    }
    return p;
}

__device__ __forceinline__ double frac_rint(double x) { return x - rint(x); }

__device__ __forceinline__ double2 e2pi(double ph) {
    double t = frac_rint(ph), s, c;
    sincospi(2.0 * t, &s, &c);
    return zc(c, s);
}

__device__ __forceinline__ double c_of(const Geo &g, double x) { return g.c0 + g.c1 * sinpi(2.0 * x); }

// V[sigma][tau][j][s]
__global__ void gen_V(Geo g, double2 *out) {
    size_t n = (size_t)(1L << g.Lp) * g.nsl * g.q * g.b;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= n) return;
    int s = id % g.b;
    size_t r = id / g.b;
    int j = r % g.q;
    r /= g.q;
    int tau = r % g.nsl;
    long sigma = r / g.nsl;
    double w = (double)g.b;                                   // frequency leaf width
    double eta = -0.5 * g.N + (sigma + 0.5) * w;
    double sgn = eta > 0 ? 1.0 : -1.0;
    double tj = cheb_t(j, g.q);
    double dxi = (s - 0.5 * w) - 0.5 * w * tj;                // xi_s - gamma_j
    double y = (tau + 0.5) / g.nsl;
    double ph = (y + sgn * c_of(g, y)) * dxi;
    double qv = lagr((s - 0.5 * w) / (0.5 * w), j, g.q);
    double2 e = e2pi(ph);
    out[id] = zc(e.x * qv, e.y * qv);
}

// C^[l+1]: group (alpha at spatial level L-l-1, sigma at frequency level l)
__global__ void gen_C(Geo g, int l, double2 *out) {
    const int q = g.q, q2 = 2 * q;
    size_t n = (size_t)(g.N / 2) * q2 * q2;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= n) return;
    int col = id % q2, row = (id / q2) % q2;
    long grp = id / ((size_t)q2 * q2);
    long G = 1L << l;
    long alpha = grp / G, sigma = grp % G;
    int cout = row / q, j = row % q, cin = col / q, t = col % q;
    long tau = 2 * alpha + cout;
    double y = (tau + 0.5) / (double)(1L << (g.L - l));
    double ws = (double)g.N / (double)(1L << l), wb = 0.5 * ws;
    double eta_s = -0.5 * g.N + (sigma + 0.5) * ws;
    double sgn = eta_s > 0 ? 1.0 : -1.0;
    double tj = cheb_t(j, q), tt = cheb_t(t, q);
    double dgam = (cin - 0.5) * wb + 0.5 * wb * tt - 0.5 * ws * tj;   // gamma_beta,t - gamma_sigma,j
    double ph = (y + sgn * c_of(g, y)) * dgam;
    double qv = lagr((cin - 0.5) + 0.5 * tt, j, q);
    double2 e = e2pi(ph);
    out[id] = zc(e.x * qv, e.y * qv);
}

// M[p][i][j] = k(z_tau,i, gamma_sigma,j), p = tau 2^h + sigma
__global__ void gen_M(Geo g, double2 *out) {
    const int q = g.q;
    size_t n = (size_t)g.N * q * q;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= n) return;
    int j = id % q, i = (id / q) % q;
    long p = id / ((size_t)q * q);
    long H = 1L << g.h;
    long tau = p / H, sigma = p % H;
    double wsp = 1.0 / (double)H;
    double y = (tau + 0.5) * wsp;
    double dz = 0.5 * wsp * cheb_t(i, q);
    double z = y + dz;
    double wf = (double)g.N / (double)H;
    long eta_i = -(g.N / 2) + (long)((sigma + 0.5) * wf);      // exact: wf is even
    double eta = (double)eta_i;
    double dg = 0.5 * wf * cheb_t(j, q);
    double gam = eta + dg;
    double sgn = eta > 0 ? 1.0 : -1.0;
    double aeta = fabs(eta);
    // x*xi part: y*eta exactly (y = (2 tau + 1) / 2^(h+1)), plus the small cross terms
    long long P = (long long)(2 * tau + 1) * (long long)eta_i;
    long long mod = 1LL << (g.h + 1);
    long long Pr = P % mod;
    double f_yeta = (double)Pr / (double)mod;
    double ph = f_yeta + y * dg + dz * gam;
    // c(z) |gamma| = (c0 + c1 sin 2 pi z)(|eta| + sgn dg), large products split exactly
    double p0 = g.c0 * aeta, e0 = fma(g.c0, aeta, -p0);
    double sz = g.c1 * sinpi(2.0 * z);
    double p1 = sz * aeta, e1 = fma(sz, aeta, -p1);
    ph += frac_rint(p0) + e0 + frac_rint(p1) + e1 + (g.c0 + sz) * sgn * dg;
    out[id] = e2pi(ph);
}

// B^[l+1]: group (alpha at spatial level l, sigma at frequency level L-l-1)
__global__ void gen_B(Geo g, int l, double2 *out) {
    const int q = g.q, q2 = 2 * q;
    size_t n = (size_t)(g.N / 2) * q2 * q2;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= n) return;
    int col = id % q2, row = (id / q2) % q2;
    long grp = id / ((size_t)q2 * q2);
    long G = 1L << (g.L - l - 1);
    long alpha = grp / G, sigma = grp % G;
    int cout = row / q, i = row % q, cin = col / q, t = col % q;
    double wa = 1.0 / (double)(1L << l), wt = 0.5 * wa;
    double ya = (alpha + 0.5) * wa;
    double ti = cheb_t(i, q), tt = cheb_t(t, q);
    double dyt = (cout - 0.5) * wt;                              // y_tau - y_alpha
    double dz = dyt + 0.5 * wt * ti - 0.5 * wa * tt;             // z_tau,i - z_alpha,t
    double sz = 2.0 * ya + dyt + 0.5 * wt * ti + 0.5 * wa * tt;  // z_tau,i + z_alpha,t
    long beta = 2 * sigma + cin;
    double wf = (double)g.N / (double)(1L << (g.L - l));
    double eta = -0.5 * g.N + (beta + 0.5) * wf;
    double ph = dz * eta + 2.0 * g.c1 * cospi(sz) * sinpi(dz) * fabs(eta);
    double pv = lagr((cout - 0.5) + 0.5 * ti, t, q);
    double2 e = e2pi(ph);
    out[id] = zc(e.x * pv, e.y * pv);
}

// U[tau][sigma][s][i]
__global__ void gen_U(Geo g, double2 *out) {
    const int q = g.q;
    size_t n = (size_t)(1L << g.Lp) * g.nsl * g.b * q;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= n) return;
    int i = id % q;
    size_t r = id / q;
    int s = r % g.b;
    r /= g.b;
    int sigma = r % g.nsl;
    long tau = r / g.nsl;
    double w = 1.0 / (double)(1L << g.Lp);
    double y = (tau + 0.5) * w;
    double dxy = (s - 0.5 * g.b) / (double)g.N;                  // x_s - y_tau
    double ti = cheb_t(i, q);
    double dx = dxy - 0.5 * w * ti;                              // x_s - z_tau,i
    double sx = 2.0 * y + dxy + 0.5 * w * ti;                    // x_s + z_tau,i
    double eta = -0.5 * g.N + (sigma + 0.5) * ((double)g.N / g.nsl);
    double ph = dx * eta + 2.0 * g.c1 * cospi(sx) * sinpi(dx) * fabs(eta);
    double pv = lagr((s - 0.5 * g.b) / (0.5 * g.b), i, q);
    double2 e = e2pi(ph);
    out[id] = zc(e.x * pv, e.y * pv);
}

__global__ void cvt_f64_f32(const double2 *in, float2 *out, size_t n) {
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id < n) {
        double2 v = in[id];
        out[id] = make_float2((float)v.x, (float)v.y);
    }
}

static Geo geo_of(const fio_bf_s *bf) {
    return Geo{bf->N, bf->L, bf->h, bf->Lp, bf->q, bf->b, bf->nsl, bf->desc.c0, bf->desc.c1};
}

static void bf_generate(fio_bf_s *bf, hipStream_t s) {
    Geo g = geo_of(bf);
    double2 *base = bf->f64.as<double2>();
    const unsigned T = 256;
    size_t nV = (size_t)(1L << bf->Lp) * bf->nsl * bf->q * bf->b;
    gen_V<<<grid1d(nV, T), T, 0, s>>>(g, base + bf->offV);
    size_t nT = (size_t)(bf->N / 2) * 4 * bf->q * bf->q;
    for (int lev = 0; lev < bf->nl; ++lev) {
        gen_C<<<grid1d(nT, T), T, 0, s>>>(g, bf->h + lev, base + bf->offC[lev]);
        gen_B<<<grid1d(nT, T), T, 0, s>>>(g, bf->h + lev, base + bf->offB[lev]);
    }
    size_t nM = (size_t)bf->N * bf->q * bf->q;
    gen_M<<<grid1d(nM, T), T, 0, s>>>(g, base + bf->offM);
    gen_U<<<grid1d(nV, T), T, 0, s>>>(g, base + bf->offU);
    FIO_HIP(hipGetLastError());
}

void bf_make_lowprec(fio_bf_s *bf, hipStream_t s);   // bf_lowprec.hip

static void bf_make_copies(fio_bf_s *bf, hipStream_t s) {
    if (bf->desc.prec_mask & (1u << FIO_PREC_FP32)) {
        bf->f32.alloc(bf->total * sizeof(float2));
        cvt_f64_f32<<<grid1d(bf->total, 256), 256, 0, s>>>(bf->f64.as<double2>(), bf->f32.as<float2>(),
                                                         bf->total);
        FIO_HIP(hipGetLastError());
    }
    if (bf->desc.prec_mask & (1u << FIO_PREC_SPLIT_FP16)) bf_make_lowprec(bf, s);
}

// ---------------------------------------------------------------------------
// apply kernels.  One thread per (unit, column); a unit is a leaf box, a
// transfer group or a middle-level pair.  Template Q = q keeps the 2q input
// and output coefficients of a unit in registers.
template <typename T> __device__ __forceinline__ cpx<T> ld_in(const double2 *p) {
    double2 v = *p;
    return cmake<cpx<T>>((T)v.x, (T)v.y);
}

// V (forward): coef[(tau 2^L' + sigma) q + j] = sum_s V[sigma][tau][j][s] x[sigma b + s]
template <typename T, int Q>
__global__ void k_leaf_in_fwd(Geo g, const cpx<T> *__restrict__ V, const double2 *__restrict__ X, long ldx,
                              cpx<T> *__restrict__ out, int nrhs) {
    using C = cpx<T>;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t nunit = (size_t)(1L << g.Lp) * g.nsl;
    if (id >= nunit * nrhs) return;
    int col = id % nrhs;
    size_t unit = id / nrhs;
    int tau = unit % g.nsl;
    long sigma = unit / g.nsl;
    C x[kLeafPts];
    const double2 *xp = X + (size_t)col * ldx + sigma * kLeafPts;
#pragma unroll
    for (int s = 0; s < kLeafPts; ++s) x[s] = ld_in<T>(xp + s);
    const C *blk = V + (sigma * g.nsl + tau) * (size_t)Q * kLeafPts;
    size_t p = (size_t)tau * (1L << g.Lp) + sigma;
    C *op = out + p * Q * nrhs + col;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        C acc = czero<C>();
#pragma unroll
        for (int s = 0; s < kLeafPts; ++s) cfma(acc, blk[j * kLeafPts + s], x[s]);
        op[(size_t)j * nrhs] = acc;
    }
}

// U^* (adjoint): coef[(tau nsl + sigma) q + i] = sum_s conj(U[tau][sigma][s][i]) u[tau b + s]
template <typename T, int Q>
__global__ void k_leaf_in_adj(Geo g, const cpx<T> *__restrict__ U, const double2 *__restrict__ X, long ldx,
                              cpx<T> *__restrict__ out, int nrhs) {
    using C = cpx<T>;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t nunit = (size_t)(1L << g.Lp) * g.nsl;
    if (id >= nunit * nrhs) return;
    int col = id % nrhs;
    size_t unit = id / nrhs;              // = tau * nsl + sigma = pair index at U-level L'
    long tau = unit / g.nsl;
    C x[kLeafPts];
    const double2 *xp = X + (size_t)col * ldx + tau * kLeafPts;
#pragma unroll
    for (int s = 0; s < kLeafPts; ++s) x[s] = ld_in<T>(xp + s);
    const C *blk = U + unit * (size_t)kLeafPts * Q;
    C *op = out + unit * Q * nrhs + col;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        C acc = czero<C>();
#pragma unroll
        for (int s = 0; s < kLeafPts; ++s) cfmac(acc, blk[s * Q + i], x[s]);
        op[(size_t)i * nrhs] = acc;
    }
}

// One transfer factor (B or C, forward or conjugate-transposed).
// Group grp = alpha G + sigma; forward inputs at pairs alpha 2G + 2 sigma + c,
// outputs at pairs (2 alpha + c) G + sigma.
template <typename T, int Q, bool ADJ, bool UNI>
__global__ void __launch_bounds__(256) k_transfer(const cpx<T> *__restrict__ A, long G,
                                                  const cpx<T> *__restrict__ in, cpx<T> *__restrict__ out,
                                                  long ngroups, int nrhs) {
    using C = cpx<T>;
    constexpr int Q2 = 2 * Q;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= (size_t)ngroups * nrhs) return;
    int col = id % nrhs;
    long grp = id / nrhs;
    if (UNI) grp = __builtin_amdgcn_readfirstlane(grp);
    long alpha = grp / G, sigma = grp % G;
    size_t pin0 = alpha * 2 * G + 2 * sigma;          // pairs pin0, pin0 + 1
    size_t pout0 = 2 * alpha * G + sigma;             // pairs pout0, pout0 + G
    size_t src0 = ADJ ? pout0 : pin0, src1 = ADJ ? pout0 + G : pin0 + 1;
    size_t dst0 = ADJ ? pin0 : pout0, dst1 = ADJ ? pin0 + 1 : pout0 + G;
    C x[Q2];
#pragma unroll
    for (int t = 0; t < Q; ++t) {
        x[t] = in[(src0 * Q + t) * nrhs + col];
        x[Q + t] = in[(src1 * Q + t) * nrhs + col];
    }
    const C *a = A + (size_t)grp * Q2 * Q2;
#pragma unroll
    for (int r = 0; r < Q2; ++r) {
        C acc = czero<C>();
#pragma unroll
        for (int c = 0; c < Q2; ++c) {
            if (ADJ)
                cfmac(acc, a[c * Q2 + r], x[c]);
            else
                cfma(acc, a[r * Q2 + c], x[c]);
        }
        size_t dst = (r < Q) ? dst0 : dst1;
        out[(dst * Q + (r % Q)) * nrhs + col] = acc;
    }
}

template <typename T, int Q, bool ADJ, bool UNI>
__global__ void __launch_bounds__(256) k_middle(const cpx<T> *__restrict__ M, const cpx<T> *__restrict__ in,
                                                cpx<T> *__restrict__ out, long npairs, int nrhs) {
    using C = cpx<T>;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= (size_t)npairs * nrhs) return;
    int col = id % nrhs;
    long p = id / nrhs;
    if (UNI) p = __builtin_amdgcn_readfirstlane(p);
    C x[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) x[j] = in[(p * Q + j) * nrhs + col];
    const C *m = M + (size_t)p * Q * Q;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        C acc = czero<C>();
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            if (ADJ)
                cfmac(acc, m[j * Q + i], x[j]);
            else
                cfma(acc, m[i * Q + j], x[j]);
        }
        out[(p * Q + i) * nrhs + col] = acc;
    }
}

// U (forward): y[tau b + s] = sum_sigma sum_i U[tau][sigma][s][i] coef[(tau nsl + sigma) q + i]
template <typename T, int Q>
__global__ void k_leaf_out_fwd(Geo g, const cpx<T> *__restrict__ U, const cpx<T> *__restrict__ in,
                               double2 *__restrict__ Y, long ldy, int nrhs) {
    using C = cpx<T>;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t nunit = (size_t)1 << g.Lp;
    if (id >= nunit * nrhs) return;
    int col = id % nrhs;
    long tau = id / nrhs;
    C acc[kLeafPts];
#pragma unroll
    for (int s = 0; s < kLeafPts; ++s) acc[s] = czero<C>();
    for (int sg = 0; sg < g.nsl; ++sg) {
        size_t p = (size_t)tau * g.nsl + sg;
        C d[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = in[(p * Q + i) * nrhs + col];
        const C *blk = U + p * (size_t)kLeafPts * Q;
#pragma unroll
        for (int s = 0; s < kLeafPts; ++s) {
#pragma unroll
            for (int i = 0; i < Q; ++i) cfma(acc[s], blk[s * Q + i], d[i]);
        }
    }
    double2 *yp = Y + (size_t)col * ldy + tau * kLeafPts;
#pragma unroll
    for (int s = 0; s < kLeafPts; ++s) yp[s] = zc((double)acc[s].x, (double)acc[s].y);
}

// V^* (adjoint): f[sigma b + s] = sum_tau sum_j conj(V[sigma][tau][j][s]) coef[(tau 2^L' + sigma) q + j]
template <typename T, int Q>
__global__ void k_leaf_out_adj(Geo g, const cpx<T> *__restrict__ V, const cpx<T> *__restrict__ in,
                               double2 *__restrict__ Y, long ldy, int nrhs) {
    using C = cpx<T>;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t nunit = (size_t)1 << g.Lp;
    if (id >= nunit * nrhs) return;
    int col = id % nrhs;
    long sigma = id / nrhs;
    C acc[kLeafPts];
#pragma unroll
    for (int s = 0; s < kLeafPts; ++s) acc[s] = czero<C>();
    for (int t = 0; t < g.nsl; ++t) {
        size_t p = (size_t)t * (1L << g.Lp) + sigma;
        C c[Q];
#pragma unroll
        for (int j = 0; j < Q; ++j) c[j] = in[(p * Q + j) * nrhs + col];
        const C *blk = V + ((size_t)sigma * g.nsl + t) * Q * kLeafPts;
#pragma unroll
        for (int j = 0; j < Q; ++j)
#pragma unroll
            for (int s = 0; s < kLeafPts; ++s) cfmac(acc[s], blk[j * kLeafPts + s], c[j]);
    }
    double2 *yp = Y + (size_t)col * ldy + sigma * kLeafPts;
#pragma unroll
    for (int s = 0; s < kLeafPts; ++s) yp[s] = zc((double)acc[s].x, (double)acc[s].y);
}

template <typename T, int Q>
static void apply_q(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                    const cpx<T> *F, cpx<T> *c0, cpx<T> *c1, hipStream_t s) {
    Geo g = geo_of(bf);
    const unsigned TB = 256;
    const bool uni = (nrhs % 64) == 0;
    const size_t nleaf = (size_t)(1L << bf->Lp) * bf->nsl;
    const long ng = bf->N / 2, np = bf->N;
    cpx<T> *cur = c0, *nxt = c1;
    const bool f64 = sizeof(T) == 8;
    auto transfer = [&](size_t off, long G, bool a) {
        size_t nt = (size_t)ng * nrhs;
        FIO_TIMED(f64 ? "bf_transfer_f64" : "bf_transfer_f32", s);
        if (a) {
            if (uni)
                k_transfer<T, Q, true, true><<<grid1d(nt, TB), TB, 0, s>>>(F + off, G, cur, nxt, ng, nrhs);
            else
                k_transfer<T, Q, true, false><<<grid1d(nt, TB), TB, 0, s>>>(F + off, G, cur, nxt, ng, nrhs);
        } else {
            if (uni)
                k_transfer<T, Q, false, true><<<grid1d(nt, TB), TB, 0, s>>>(F + off, G, cur, nxt, ng, nrhs);
            else
                k_transfer<T, Q, false, false><<<grid1d(nt, TB), TB, 0, s>>>(F + off, G, cur, nxt, ng, nrhs);
        }
        std::swap(cur, nxt);
    };
    auto middle = [&](bool a) {
        size_t nt = (size_t)np * nrhs;
        FIO_TIMED(f64 ? "bf_middle_f64" : "bf_middle_f32", s);
        if (a) {
            if (uni)
                k_middle<T, Q, true, true><<<grid1d(nt, TB), TB, 0, s>>>(F + bf->offM, cur, nxt, np, nrhs);
            else
                k_middle<T, Q, true, false><<<grid1d(nt, TB), TB, 0, s>>>(F + bf->offM, cur, nxt, np, nrhs);
        } else {
            if (uni)
                k_middle<T, Q, false, true><<<grid1d(nt, TB), TB, 0, s>>>(F + bf->offM, cur, nxt, np, nrhs);
            else
                k_middle<T, Q, false, false><<<grid1d(nt, TB), TB, 0, s>>>(F + bf->offM, cur, nxt, np, nrhs);
        }
        std::swap(cur, nxt);
    };
    if (!adj) {
        {
            FIO_TIMED(f64 ? "bf_leaf_in_f64" : "bf_leaf_in_f32", s);
            k_leaf_in_fwd<T, Q><<<grid1d(nleaf * nrhs, TB), TB, 0, s>>>(g, F + bf->offV, X, ldx, cur, nrhs);
        }
        for (int lev = bf->nl - 1; lev >= 0; --lev) transfer(bf->offC[lev], 1L << (bf->h + lev), false);
        middle(false);
        for (int lev = 0; lev < bf->nl; ++lev) transfer(bf->offB[lev], 1L << (bf->L - bf->h - lev - 1), false);
        FIO_TIMED(f64 ? "bf_leaf_out_f64" : "bf_leaf_out_f32", s);
        k_leaf_out_fwd<T, Q><<<grid1d(((size_t)1 << bf->Lp) * nrhs, TB), TB, 0, s>>>(g, F + bf->offU, cur, Y,
                                                                                       ldy, nrhs);
    } else {
        {
            FIO_TIMED(f64 ? "bf_leaf_in_f64" : "bf_leaf_in_f32", s);
            k_leaf_in_adj<T, Q><<<grid1d(nleaf * nrhs, TB), TB, 0, s>>>(g, F + bf->offU, X, ldx, cur, nrhs);
        }
        for (int lev = bf->nl - 1; lev >= 0; --lev) transfer(bf->offB[lev], 1L << (bf->L - bf->h - lev - 1), true);
        middle(true);
        for (int lev = 0; lev < bf->nl; ++lev) transfer(bf->offC[lev], 1L << (bf->h + lev), true);
        FIO_TIMED(f64 ? "bf_leaf_out_f64" : "bf_leaf_out_f32", s);
        k_leaf_out_adj<T, Q><<<grid1d(((size_t)1 << bf->Lp) * nrhs, TB), TB, 0, s>>>(g, F + bf->offV, cur, Y,
                                                                                       ldy, nrhs);
    }
    FIO_HIP(hipGetLastError());
}

template <typename T>
static void apply_t(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                    const cpx<T> *F, void *ws, hipStream_t s) {
    cpx<T> *c0 = reinterpret_cast<cpx<T> *>(ws);
    cpx<T> *c1 = c0 + bf_coef_elems(bf, nrhs);
    switch (bf->q) {
#define FIO_Q(QQ) \
    case QQ: apply_q<T, QQ>(bf, adj, X, ldx, Y, ldy, nrhs, F, c0, c1, s); break;
        FIO_Q(2) FIO_Q(3) FIO_Q(4) FIO_Q(5) FIO_Q(6) FIO_Q(7) FIO_Q(8) FIO_Q(9)
        FIO_Q(10) FIO_Q(11) FIO_Q(12) FIO_Q(13) FIO_Q(14) FIO_Q(15) FIO_Q(16)
#undef FIO_Q
        default: throw Err{FIO_ERR_UNSUPPORTED};
    }
}

void bf_apply_split16(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                      void *ws, hipStream_t s);   // bf_lowprec.hip
size_t bf_ws_bytes_split16(const fio_bf_s *bf, int nrhs);

size_t bf_ws_bytes(const fio_bf_s *bf, int nrhs, fio_prec prec) {
    size_t e = bf_coef_elems(bf, nrhs);
    switch (prec) {
        case FIO_PREC_FP64: return 2 * e * sizeof(double2);
        case FIO_PREC_FP32: return 2 * e * sizeof(float2);
        case FIO_PREC_SPLIT_FP16: return bf_ws_bytes_split16(bf, nrhs);
    }
    return 0;
}

void bf_apply_impl(fio_bf_s *bf, bool adjoint, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                   fio_prec prec, void *ws, hipStream_t s) {
    if (nrhs <= 0) return;
    switch (prec) {
        case FIO_PREC_FP64:
            apply_t<double>(bf, adjoint, X, ldx, Y, ldy, nrhs, bf->f64.as<double2>(), ws, s);
            break;
        case FIO_PREC_FP32:
            if (!bf->f32.p) throw Err{FIO_ERR_ARG};
            apply_t<float>(bf, adjoint, X, ldx, Y, ldy, nrhs, bf->f32.as<float2>(), ws, s);
            break;
        case FIO_PREC_SPLIT_FP16:
            if (!bf->f16.p) throw Err{FIO_ERR_ARG};
            bf_apply_split16(bf, adjoint, X, ldx, Y, ldy, nrhs, ws, s);
            break;
    }
}

}  // namespace fio

using namespace fio;

// ---------------------------------------------------------------------------
// C ABI
extern "C" size_t fio_bf_factor_count(const fio_bf_desc *desc) {
    fio_bf_s tmp;
    if (bf_plan(desc, &tmp) != FIO_OK) return 0;
    return tmp.total;
}

static fio_status bf_new(const fio_bf_desc *desc, fio_bf_t *out, fio_bf_s **bfp) {
    if (!desc || !out) return FIO_ERR_ARG;
    fio_bf_s *bf = new fio_bf_s();
    fio_status st = bf_plan(desc, bf);
    if (st != FIO_OK) {
        delete bf;
        return st;
    }
    *bfp = bf;
    return FIO_OK;
}

extern "C" fio_status fio_bf_build(const fio_bf_desc *desc, void *stream, fio_bf_t *out) {
    fio_bf_s *bf = nullptr;
    fio_status st = bf_new(desc, out, &bf);
    if (st != FIO_OK) return st;
    st = guarded([&] {
        hipStream_t s = as_stream(stream);
        bf->f64.alloc(bf->total * sizeof(double2));
        bf_generate(bf, s);
        bf_make_copies(bf, s);
        FIO_HIP(hipStreamSynchronize(s));
        return FIO_OK;
    });
    if (st != FIO_OK) {
        delete bf;
        return st;
    }
    *out = bf;
    return FIO_OK;
}

extern "C" fio_status fio_bf_import(const fio_bf_desc *desc, const void *host_factors, size_t count, void *stream,
                                    fio_bf_t *out) {
    if (!host_factors) return FIO_ERR_ARG;
    fio_bf_s *bf = nullptr;
    fio_status st = bf_new(desc, out, &bf);
    if (st != FIO_OK) return st;
    if (count != bf->total) {
        delete bf;
        return FIO_ERR_ARG;
    }
    st = guarded([&] {
        hipStream_t s = as_stream(stream);
        bf->f64.alloc(bf->total * sizeof(double2));
        FIO_HIP(hipMemcpyAsync(bf->f64.p, host_factors, bf->total * sizeof(double2), hipMemcpyHostToDevice, s));
        bf_make_copies(bf, s);
        FIO_HIP(hipStreamSynchronize(s));
        return FIO_OK;
    });
    if (st != FIO_OK) {
        delete bf;
        return st;
    }
    *out = bf;
    return FIO_OK;
}

extern "C" fio_status fio_bf_export(fio_bf_t bf, void *host_out, size_t count, void *stream) {
    FIO_CHECK_ARG(bf && host_out && count == bf->total);
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        FIO_HIP(hipMemcpyAsync(host_out, bf->f64.p, bf->total * sizeof(double2), hipMemcpyDeviceToHost, s));
        FIO_HIP(hipStreamSynchronize(s));
        return FIO_OK;
    });
}

extern "C" fio_status fio_bf_workspace_size(fio_bf_t bf, int nrhs, fio_prec prec, size_t *bytes) {
    FIO_CHECK_ARG(bf && bytes && nrhs >= 0 && prec >= FIO_PREC_FP64 && prec <= FIO_PREC_SPLIT_FP16);
    *bytes = bf_ws_bytes(bf, nrhs, prec);
    return FIO_OK;
}

static fio_status bf_apply_api(fio_bf_t bf, bool adj, const void *X, long ldx, void *Y, long ldy, int nrhs,
                               fio_prec prec, void *ws, size_t ws_bytes, void *stream) {
    FIO_CHECK_ARG(bf && nrhs >= 0);
    if (nrhs == 0) return FIO_OK;
    FIO_CHECK_ARG(X && Y && ldx >= bf->N && ldy >= bf->N);
    FIO_CHECK_ARG(prec >= FIO_PREC_FP64 && prec <= FIO_PREC_SPLIT_FP16);
    if (prec == FIO_PREC_FP32 && !bf->f32.p) return FIO_ERR_ARG;
    if (prec == FIO_PREC_SPLIT_FP16 && !bf->f16.p) return FIO_ERR_ARG;
    size_t need = bf_ws_bytes(bf, nrhs, prec);
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        if (ws) {
            if (ws_bytes < need) return FIO_ERR_ARG;
            bf_apply_impl(bf, adj, (const double2 *)X, ldx, (double2 *)Y, ldy, nrhs, prec, ws, s);
        } else {
            std::lock_guard<std::mutex> lk(bf->ws_mu);
            if (bf->ws.bytes < need) {
                FIO_HIP(hipStreamSynchronize(s));
                bf->ws.alloc(need);
            }
            bf_apply_impl(bf, adj, (const double2 *)X, ldx, (double2 *)Y, ldy, nrhs, prec, bf->ws.p, s);
        }
        return FIO_OK;
    });
}

extern "C" fio_status fio_bf_apply(fio_bf_t bf, const void *X, long ldx, void *Y, long ldy, int nrhs, fio_prec prec,
                                   void *ws, size_t ws_bytes, void *stream) {
    return bf_apply_api(bf, false, X, ldx, Y, ldy, nrhs, prec, ws, ws_bytes, stream);
}

extern "C" fio_status fio_bf_apply_adj(fio_bf_t bf, const void *X, long ldx, void *Y, long ldy, int nrhs,
                                       fio_prec prec, void *ws, size_t ws_bytes, void *stream) {
    return bf_apply_api(bf, true, X, ldx, Y, ldy, nrhs, prec, ws, ws_bytes, stream);
}

extern "C" void fio_bf_destroy(fio_bf_t bf) { delete bf; }

extern "C" const char *fio_status_str(fio_status s) {
    switch (s) {
        case FIO_OK: return "ok";
        case FIO_ERR_ARG: return "invalid argument";
        case FIO_ERR_OOM: return "out of device memory";
        case FIO_ERR_HIP: return "HIP runtime error";
        case FIO_ERR_NOT_HPD: return "matrix not Hermitian positive definite";
        case FIO_ERR_NOT_CONVERGED: return "refinement did not converge";
        case FIO_ERR_UNSUPPORTED: return "unsupported configuration";
        case FIO_ERR_CALLBACK: return "callback failed";
        case FIO_WARN_RANK_CAP: return "HSS rank cap reached";
    }
    return "unknown status";
}
