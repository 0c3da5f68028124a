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
#include "bf_apply.h"
#include "ddmath.h"

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>

namespace fio {

// ---------------------------------------------------------------------------
// geometry
fio_status bf_plan(const fio_bf_desc *d, fio_bf_s *bf) {
    if (d && d->dim == 2) return bf2d_plan(d, bf);
    if (!d || d->dim != 1) return d ? FIO_ERR_UNSUPPORTED : FIO_ERR_ARG;
    if (d->n < 64 || (d->n & (d->n - 1))) return FIO_ERR_ARG;
    int L = 0;
    while ((1L << L) < d->n) ++L;
    if (L % 2) return FIO_ERR_UNSUPPORTED;
    if (d->q < 2 || d->q > 16 || d->level_offset < 1) return FIO_ERR_ARG;
    if (d->phase_kind != FIO_PHASE2_ANISO) return FIO_ERR_UNSUPPORTED;   // 2D phases only
    if (d->amp_kind < FIO_AMP_ONE || d->amp_kind > FIO_AMP_HANKEL) return FIO_ERR_ARG;
    if (d->amp_kind == FIO_AMP_HANKEL) return FIO_ERR_UNSUPPORTED;       // 2D amplitude only
    const int terms = d->amp_kind == FIO_AMP_GAUSSIAN_SUM ? d->amp_terms : 0;
    if (d->amp_kind == FIO_AMP_GAUSSIAN_SUM &&
        (terms < 1 || terms > kMaxAmpTerms || !(d->amp_sigma2 > 0.0) || !d->amp_centers))
        return FIO_ERR_ARG;
    bf->desc = *d;
    bf->desc.amp_centers = nullptr;          // the handle keeps its own copy
    bf->amp.m = terms;
    bf->amp.s2 = terms > 0 ? d->amp_sigma2 : 1.0;
    for (int k = 0; k < terms; ++k) {
        bf->amp.x[k] = d->amp_centers[k];
        bf->amp.xi[k] = d->amp_centers[terms + k];
    }
    bf->N = d->n;
    bf->n1 = d->n;
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

static bool g_fused_off = false;
bool fused_disabled() { return g_fused_off; }
void set_fused_disabled(bool v) { g_fused_off = v; }
static bool g_leaf_fused_off = false;
bool leaf_fused_disabled() { return g_leaf_fused_off; }

size_t bf_tw_off(const fio_bf_s *bf, bool cside, int lev) {
    const size_t ntw = (size_t)(bf->N / 2) * 8 * bf->q;
    return ((cside ? bf->nl : 0) + (size_t)lev) * ntw;
}

size_t bf_coef_elems(const fio_bf_s *bf, int nrhs) { return (size_t)bf->N * bf->q * (size_t)nrhs; }

// factor evaluation (Section 2.2).  Every entry is formed from exact points (box centers are
// binary fractions or integers, Chebyshev points are center + (w/2) t_i with the nodes t_i to 106
// bits) in double-double arithmetic (ddmath.h): phase differences, their products with the
// frequencies and c(x) keep all their bits, the integer part of a phase is dropped exactly and
// the entry is rounded once.  Lagrange values are taken in the reference coordinate u of the
// point in its interpolation box, where p_t(u) is the same for every box.

// c(x) = c0 + c1 sin(2 pi x)
__device__ dd c_dd(const Geo &g, dd x) { return dd_add(dd_of(g.c0), dd_mul_d(dd_sinpi(dd_ldexp(x, 2.0)), g.c1)); }

__device__ __forceinline__ double2 scaled(double2 e, double v) { return zc(e.x * v, e.y * v); }

// V[sigma][tau][j][s] = exp(2 pi i (y + sgn c(y)) (xi_s - gamma_j)) q_j(xi_s)   (|xi| = sgn xi on the box)
__global__ void gen_V(Geo g, Nodes tn, double2 *out) {
    size_t n = (size_t)(1L << g.Lp) * g.nsl * g.q * g.b;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= n) return;
    int s = id % g.b;
    size_t r = id / g.b;
    int j = r % g.q;
    r /= g.q;
    int tau = r % g.nsl;
    long sigma = r / g.nsl;
    const double w = (double)g.b, hw = 0.5 * w;                  // frequency leaf width (8) and half width
    const double eta = -0.5 * g.N + (sigma + 0.5) * w;
    const double sgn = eta > 0 ? 1.0 : -1.0;
    const double y = (tau + 0.5) / g.nsl;
    const dd kap = dd_add(dd_of(y), dd_mul_d(c_dd(g, dd_of(y)), sgn));
    const dd dxi = dd_sub(dd_of(s - hw), dd_ldexp(tn.t(j), hw));  // xi_s - gamma_j
    const double qv = dd_lagrange(dd_of((s - hw) / hw), j, tn);
    out[id] = scaled(dd_expi2pi(dd_frac(dd_mul(kap, dxi))), qv);
}

// C^[l+1]: group (alpha at spatial level L-l-1, sigma at frequency level l)
__global__ void gen_C(Geo g, Nodes tn, int l, double2 *out) {
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
    const double y = (tau + 0.5) / (double)(1L << (g.L - l));
    const double ws = (double)g.N / (double)(1L << l), wb = 0.5 * ws;
    const double eta_s = -0.5 * g.N + (sigma + 0.5) * ws;
    const double sgn = eta_s > 0 ? 1.0 : -1.0;
    const dd kap = dd_add(dd_of(y), dd_mul_d(c_dd(g, dd_of(y)), sgn));
    // gamma_beta,t - gamma_sigma,j
    const dd dgam = dd_add(dd_of((cin - 0.5) * wb), dd_sub(dd_ldexp(tn.t(t), 0.5 * wb), dd_ldexp(tn.t(j), 0.5 * ws)));
    const dd u = dd_add(dd_of(cin - 0.5), dd_ldexp(tn.t(t), 0.5));
    out[id] = scaled(dd_expi2pi(dd_frac(dd_mul(kap, dgam))), dd_lagrange(u, j, tn));
}

// M[p][i][j] = k(z_tau,i, gamma_sigma,j), p = tau 2^h + sigma
// a(z, gamma) of Section 5.1 (1 when the amplitude has no terms)
__device__ double amp_at(const Amp &a, double z, double gam, double N) {
    if (a.m == 0) return 1.0;
    double s = 0.0;
    for (int k = 0; k < a.m; ++k) {
        const double dx = z - a.x[k], dxi = (gam - a.xi[k]) / N;
        s += exp(-(dx * dx + dxi * dxi) / a.s2);
    }
    return s;
}

__global__ void gen_M(Geo g, Nodes tn, Amp am, double2 *out) {
    const int q = g.q;
    size_t n = (size_t)g.N * q * q;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= n) return;
    int j = id % q, i = (id / q) % q;
    long p = id / ((size_t)q * q);
    long H = 1L << g.h;
    long tau = p / H, sigma = p % H;
    const double wsp = 1.0 / (double)H, wf = (double)g.N / (double)H;
    const dd z = dd_add(dd_of((tau + 0.5) * wsp), dd_ldexp(tn.t(i), 0.5 * wsp));
    const double eta = -0.5 * g.N + (sigma + 0.5) * wf;           // an integer (wf is even)
    const dd gam = dd_add(dd_of(eta), dd_ldexp(tn.t(j), 0.5 * wf));
    const double sgn = eta > 0 ? 1.0 : -1.0;                       // no level-h box straddles 0
    // Phi = z gamma + c(z) |gamma|, each product reduced modulo 1 before the sum
    const dd lin = dd_frac(dd_mul(z, gam));
    const dd nonlin = dd_frac(dd_mul(c_dd(g, z), dd_mul_d(gam, sgn)));
    const double av = amp_at(am, dd_val(z), dd_val(gam), (double)g.N);
    out[id] = scaled(dd_expi2pi(dd_add(lin, nonlin)), av);
}

// B^[l+1]: group (alpha at spatial level l, sigma at frequency level L-l-1)
//   exp(2 pi i ((z_tau,i - z_alpha,t) eta + (c(z_tau,i) - c(z_alpha,t)) |eta|)) p_t(u_i)
__global__ void gen_B(Geo g, Nodes tn, int l, double2 *out) {
    const int q = g.q, q2 = 2 * q;
    size_t n = (size_t)(g.N / 2) * q2 * q2;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= n) return;
    int col = id % q2, row = (id / q2) % q2;
    long grp = id / ((size_t)q2 * q2);
    long G = 1L << (g.L - l - 1);
    long alpha = grp / G, sigma = grp % G;
    int cout = row / q, i = row % q, cin = col / q, t = col % q;
    const double wa = 1.0 / (double)(1L << l), wt = 0.5 * wa;
    const double ya = (alpha + 0.5) * wa;
    const dd d1 = dd_add(dd_of((cout - 0.5) * wt), dd_ldexp(tn.t(i), 0.5 * wt));   // z_tau,i - y_alpha
    const dd d2 = dd_ldexp(tn.t(t), 0.5 * wa);                                       // z_alpha,t - y_alpha
    const long beta = 2 * sigma + cin;
    const double wf = (double)g.N / (double)(1L << (g.L - l));
    const double eta = -0.5 * g.N + (beta + 0.5) * wf;
    const dd dc = dd_sub(c_dd(g, dd_add(dd_of(ya), d1)), c_dd(g, dd_add(dd_of(ya), d2)));
    const dd ph = dd_add(dd_frac(dd_mul_d(dd_sub(d1, d2), eta)), dd_frac(dd_mul_d(dc, fabs(eta))));
    const dd u = dd_add(dd_of(cout - 0.5), dd_ldexp(tn.t(i), 0.5));
    out[id] = scaled(dd_expi2pi(ph), dd_lagrange(u, t, tn));
}

// U[tau][sigma][s][i] = exp(2 pi i ((x_s - z_tau,i) eta + (c(x_s) - c(z_tau,i)) |eta|)) p_i(x_s)
__global__ void gen_U(Geo g, Nodes tn, double2 *out) {
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
    const double w = 1.0 / (double)(1L << g.Lp), hb = 0.5 * g.b;
    const double y = (tau + 0.5) * w;
    const double x = (tau * g.b + s) / (double)g.N;                 // grid point, exact
    const dd dzt = dd_ldexp(tn.t(i), 0.5 * w);                      // z_tau,i - y
    const dd dx = dd_sub(dd_of((s - hb) / (double)g.N), dzt);     // x_s - z_tau,i
    const double eta = -0.5 * g.N + (sigma + 0.5) * ((double)g.N / g.nsl);
    const dd dc = dd_sub(c_dd(g, dd_of(x)), c_dd(g, dd_add(dd_of(y), dzt)));
    const dd ph = dd_add(dd_frac(dd_mul_d(dx, eta)), dd_frac(dd_mul_d(dc, fabs(eta))));
    out[id] = scaled(dd_expi2pi(ph), dd_lagrange(dd_of((s - hb) / hb), i, tn));
}

// Structured transfer factors: every 2q x 2q transfer block is, per (c_out, c_in) quadrant,
// diag(a) P diag(b) with P a Lagrange matrix shared by all groups of a side, and
//   B side: a = exp(2 pi i (Phi(z_tau,i, eta_beta) - Phi(y_alpha, eta_beta))),
//           b = exp(-2 pi i (Phi(z_alpha,t, eta_beta) - Phi(y_alpha, eta_beta))), P = P_cout(i, t);
//   C side: a = exp(-2 pi i (Phi(y_tau, gamma_sigma,j) - Phi(y_tau, eta_sigma))),
//           b = exp(2 pi i (Phi(y_tau, gamma_beta,t) - Phi(y_tau, eta_sigma))),   P = P_cin(t, j),
// with P_c(i, t) = p_t((c - 1/2) + t_i / 2) on the reference grid.  The products a P b are the
// entries of Section 2.2 (the common phase at the parent's center cancels).
// Layout per group: [c_out][4][q] = a(c_out, 0), a(c_out, 1), b(c_out, 0), b(c_out, 1).
__global__ void gen_TW_B(Geo g, Nodes tn, int l, double2 *out) {
    const int q = g.q;
    size_t n = (size_t)(g.N / 2) * 8 * q;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= n) return;
    const int i = id % q, kind = (id / q) % 4, cout = (id / (4 * q)) % 2;
    const long grp = id / (8 * q);
    const long G = 1L << (g.L - l - 1);
    const long alpha = grp / G, sigma = grp % G;
    const int cin = kind & 1;
    const double wa = 1.0 / (double)(1L << l), wt = 0.5 * wa;
    const double ya = (alpha + 0.5) * wa;
    const long beta = 2 * sigma + cin;
    const double wf = (double)g.N / (double)(1L << (g.L - l));
    const double eta = -0.5 * g.N + (beta + 0.5) * wf;
    // a: z_tau,i - y_alpha; b: z_alpha,i - y_alpha, conjugated
    const dd dz = kind < 2 ? dd_add(dd_of((cout - 0.5) * wt), dd_ldexp(tn.t(i), 0.5 * wt))
                           : dd_ldexp(tn.t(i), 0.5 * wa);
    const dd dc = dd_sub(c_dd(g, dd_add(dd_of(ya), dz)), c_dd(g, dd_of(ya)));
    const dd ph = dd_add(dd_frac(dd_mul_d(dz, eta)), dd_frac(dd_mul_d(dc, fabs(eta))));
    out[id] = dd_expi2pi(kind < 2 ? ph : dd_neg(ph));
}

__global__ void gen_TW_C(Geo g, Nodes tn, int l, double2 *out) {
    const int q = g.q;
    size_t n = (size_t)(g.N / 2) * 8 * q;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= n) return;
    const int i = id % q, kind = (id / q) % 4, cout = (id / (4 * q)) % 2;
    const long grp = id / (8 * q);
    const long G = 1L << l;
    const long alpha = grp / G, sigma = grp % G;
    const int cin = kind & 1;
    const long tau = 2 * alpha + cout;
    const double y = (tau + 0.5) / (double)(1L << (g.L - l));
    const double ws = (double)g.N / (double)(1L << l), wb = 0.5 * ws;
    const double eta_s = -0.5 * g.N + (sigma + 0.5) * ws;
    const double sgn = eta_s > 0 ? 1.0 : -1.0;
    const dd kap = dd_add(dd_of(y), dd_mul_d(c_dd(g, dd_of(y)), sgn));
    // a: -(gamma_sigma,j - eta_sigma); b: gamma_beta,t - eta_sigma
    const dd d = kind < 2 ? dd_neg(dd_ldexp(tn.t(i), 0.5 * ws))
                          : dd_add(dd_of((cin - 0.5) * wb), dd_ldexp(tn.t(i), 0.5 * wb));
    out[id] = dd_expi2pi(dd_frac(dd_mul(kap, d)));
}

__global__ void gen_Pchild(Nodes tn, double *out) {
    // out[c][i][t] = P_c(i, t) = p_t((c - 1/2) + t_i / 2)
    const int q = tn.q;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= 2 * q * q) return;
    const int t = id % q, i = (id / q) % q, c = id / (q * q);
    out[id] = dd_lagrange(dd_add(dd_of(c - 0.5), dd_ldexp(tn.t(i), 0.5)), t, tn);
}

__global__ void cvt_f64_f32(const double2 *in, float2 *out, size_t n) {
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id < n) {
        double2 v = in[id];
        out[id] = make_float2((float)v.x, (float)v.y);
    }
}

static void bf_generate(fio_bf_s *bf, hipStream_t s) {
    if (bf->dim == 2) return bf2d_generate(bf, s);
    Geo g = geo_of(bf);
    const Nodes tn = make_nodes(bf->q);
    double2 *base = bf->f64.as<double2>();
    const unsigned T = 256;
    size_t nV = (size_t)(1L << bf->Lp) * bf->nsl * bf->q * bf->b;
    gen_V<<<grid1d(nV, T), T, 0, s>>>(g, tn, base + bf->offV);
    size_t nT = (size_t)(bf->N / 2) * 4 * bf->q * bf->q;
    for (int lev = 0; lev < bf->nl; ++lev) {
        gen_C<<<grid1d(nT, T), T, 0, s>>>(g, tn, bf->h + lev, base + bf->offC[lev]);
        gen_B<<<grid1d(nT, T), T, 0, s>>>(g, tn, bf->h + lev, base + bf->offB[lev]);
    }
    size_t nM = (size_t)bf->N * bf->q * bf->q;
    gen_M<<<grid1d(nM, T), T, 0, s>>>(g, tn, bf->amp, base + bf->offM);
    gen_U<<<grid1d(nV, T), T, 0, s>>>(g, tn, base + bf->offU);
    FIO_HIP(hipGetLastError());
    // structured transfer twiddles and the shared Lagrange matrices
    if (bf->nl > 0) {
        const size_t ntw = (size_t)(bf->N / 2) * 8 * bf->q;
        bf->tw64.alloc(2 * bf->nl * ntw * sizeof(double2));
        for (int lev = 0; lev < bf->nl; ++lev) {
            gen_TW_B<<<grid1d(ntw, T), T, 0, s>>>(g, tn, bf->h + lev, bf->tw64.as<double2>() + bf_tw_off(bf, false, lev));
            gen_TW_C<<<grid1d(ntw, T), T, 0, s>>>(g, tn, bf->h + lev, bf->tw64.as<double2>() + bf_tw_off(bf, true, lev));
        }
        DevBuf pd(2 * bf->q * bf->q * sizeof(double));
        gen_Pchild<<<1, 2 * bf->q * bf->q, 0, s>>>(tn, pd.as<double>());
        FIO_HIP(hipGetLastError());
        FIO_HIP(hipMemcpyAsync(bf->Pchild, pd.p, 2 * bf->q * bf->q * sizeof(double), hipMemcpyDeviceToHost, s));
        FIO_HIP(hipStreamSynchronize(s));
        bf->structured = true;
    }
}

void bf_make_lowprec(fio_bf_s *bf, hipStream_t s);   // bf_lowprec.hip

static void bf_make_copies(fio_bf_s *bf, hipStream_t s) {
    const bool want16 = (bf->desc.prec_mask & (1u << FIO_PREC_SPLIT_FP16)) != 0;
    if (want16 && (bf->dim != 1 || bf->q != 9)) throw Err{FIO_ERR_UNSUPPORTED};
    if (bf->dim == 2) return bf2d_finish(bf, s);
    // the split-FP16 apply keeps leaf and middle factors in FP32
    if (bf->desc.prec_mask & ((1u << FIO_PREC_FP32) | (1u << FIO_PREC_SPLIT_FP16))) {
        bf->f32.alloc(bf->total * sizeof(float2));
        cvt_f64_f32<<<grid1d(bf->total, 256), 256, 0, s>>>(bf->f64.as<double2>(), bf->f32.as<float2>(),
                                                         bf->total);
        if (bf->structured) {
            const size_t ntw = 2 * bf->nl * (size_t)(bf->N / 2) * 8 * bf->q;
            bf->tw32.alloc(ntw * sizeof(float2));
            cvt_f64_f32<<<grid1d(ntw, 256), 256, 0, s>>>(bf->tw64.as<double2>(), bf->tw32.as<float2>(), ntw);
        }
        FIO_HIP(hipGetLastError());
    }
    if (want16) bf_make_lowprec(bf, s);
}

void bf_apply_f64(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                 const double2 *F, void *ws, hipStream_t s, const double2 *Ysub = nullptr, long ldsub = 0);
void bf_apply_f32(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                 const float2 *F, void *ws, hipStream_t s, bool split);

void bf_apply_split16(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                      void *ws, hipStream_t s);   // bf_lowprec.hip
size_t bf_ws_bytes_split16(const fio_bf_s *bf, int nrhs);

size_t bf_ws_bytes(const fio_bf_s *bf, int nrhs, fio_prec prec) {
    if (bf->dim == 2) return bf2d_ws_bytes(bf, nrhs, prec);
    size_t e = bf_coef_elems(bf, nrhs);
    switch (prec) {
        case FIO_PREC_FP64: return 2 * e * sizeof(double2);
        case FIO_PREC_FP32: return 2 * e * sizeof(float2);
        case FIO_PREC_SPLIT_FP16: return bf_ws_bytes_split16(bf, nrhs);
    }
    return 0;
}

int tile_key(bool adj, fio_prec prec, int nrhs) {
    int b = 0;
    while (b < 6 && (1 << b) < nrhs) ++b;
    return (adj ? 1 : 0) | ((int)prec << 1) | (b << 3);
}

TileCfg bf_tile(const fio_bf_s *bf, bool adj, fio_prec prec, int nrhs) {
    std::lock_guard<std::mutex> lk(bf->tune_mu);
    auto it = bf->tuned.find(tile_key(adj, prec, nrhs));
    return it == bf->tuned.end() ? TileCfg{} : it->second;
}

// candidate tile configurations of an apply (the first is the built-in default)
static std::vector<TileCfg> tile_candidates(const fio_bf_s *bf, fio_prec prec) {
    std::vector<TileCfg> c;
    c.push_back(TileCfg{});
    if (bf->dim == 2) {
        const long T = 1L << (2 * bf->lc);
        const int nmax = (int)(T < 16 ? T : 16);
        for (int kc : {8, 16})
            for (int ns : {4, 8, 16})
                if (ns <= nmax && T % ns == 0) c.push_back(TileCfg{kc, ns, 0});
    } else if (bf->nl > 0 && bf->q == 9) {
        // levels per fused pass; with 3, the first leaf factor folded in or run on its own; in
        // split precision, each of these with the transfer passes on the matrix cores (split
        // FP16) or on the vector units (FP32, the more accurate of the two)
        for (int valu : {0, 1}) {
            if (valu && prec != FIO_PREC_SPLIT_FP16) continue;
            for (int km : {1, 2, 3}) c.push_back(TileCfg{0, 0, km, 0, valu});
            c.push_back(TileCfg{0, 0, 3, 1, valu});
        }
    }
    return c;
}

static std::string tile_str(const TileCfg &c) {
    char buf[96];
    snprintf(buf, sizeof buf, "kc=%d nsplit=%d kmax=%d leaf_sep=%d valu=%d", c.kc, c.nsplit, c.kmax, c.leaf_sep,
             c.valu);
    return buf;
}

void bf_apply_impl(fio_bf_s *bf, bool adjoint, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                   fio_prec prec, void *ws, hipStream_t s, bool freq_internal) {
    if (nrhs <= 0) return;
    if (bf->dim == 2) {
        if ((prec == FIO_PREC_FP32 && !bf->f32.p) || prec == FIO_PREC_SPLIT_FP16) throw Err{FIO_ERR_ARG};
        return bf2d_apply(bf, adjoint, X, ldx, Y, ldy, nrhs, prec, ws, freq_internal, s);
    }
    switch (prec) {
        case FIO_PREC_FP64:
            bf_apply_f64(bf, adjoint, X, ldx, Y, ldy, nrhs, bf->f64.as<double2>(), ws, s);
            break;
        case FIO_PREC_FP32:
            if (!bf->f32.p) throw Err{FIO_ERR_ARG};
            bf_apply_f32(bf, adjoint, X, ldx, Y, ldy, nrhs, bf->f32.as<float2>(), ws, s, false);
            break;
        case FIO_PREC_SPLIT_FP16:
            if (!bf->split16) throw Err{FIO_ERR_ARG};
            bf_apply_split16(bf, adjoint, X, ldx, Y, ldy, nrhs, ws, s);
            break;
    }
}

// R = U - K~ X in FP64 with the subtraction done by the leaf kernel that writes K~ X (1D);
// returns false, doing nothing, where that form does not exist (2D)
bool bf_residual_f64(fio_bf_s *bf, const double2 *X, long ldx, const double2 *U, long ldu, double2 *R, long ldr,
                     int nrhs, void *ws, hipStream_t s) {
    if (bf->dim != 1) return false;
    if (nrhs > 0) bf_apply_f64(bf, false, X, ldx, R, ldr, nrhs, bf->f64.as<double2>(), ws, s, U, ldu);
    return true;
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
    if (prec == FIO_PREC_SPLIT_FP16 && !bf->split16) return FIO_ERR_ARG;
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

static bool tile_valid(const fio_bf_s *bf, const TileCfg &c) {
    if (!(c.kc == 0 || c.kc == 8 || c.kc == 16)) return false;
    if (!(c.kmax >= 0 && c.kmax <= 3 && c.nsplit >= 0)) return false;
    if (!(c.leaf_sep == 0 || c.leaf_sep == 1) || !(c.valu == 0 || c.valu == 1)) return false;
    if (bf->dim == 2 && c.nsplit > 0) {
        const long T = 1L << (2 * bf->lc);
        if (!(c.nsplit <= (T < 16 ? T : 16) && T % c.nsplit == 0)) return false;
    }
    return true;
}

extern "C" fio_status fio_bf_set_tile(fio_bf_t bf, int adj, fio_prec prec, int nrhs, int kc, int nsplit, int kmax) {
    fio_tile t{kc, nsplit, kmax, 0, 0};
    return fio_bf_set_tile_cfg(bf, adj, prec, nrhs, &t);
}

extern "C" fio_status fio_bf_set_tile_cfg(fio_bf_t bf, int adj, fio_prec prec, int nrhs, const fio_tile *t) {
    FIO_CHECK_ARG(bf && t && nrhs > 0 && prec >= FIO_PREC_FP64 && prec <= FIO_PREC_SPLIT_FP16);
    const TileCfg c{t->kc, t->nsplit, t->kmax, t->leaf_sep, t->valu};
    FIO_CHECK_ARG(tile_valid(bf, c));
    FIO_CHECK_ARG(c.valu == 0 || prec == FIO_PREC_SPLIT_FP16);
    std::lock_guard<std::mutex> lk(bf->tune_mu);
    bf->tuned[tile_key(adj != 0, prec, nrhs)] = c;
    return FIO_OK;
}

extern "C" fio_status fio_bf_get_tile_cfg(fio_bf_t bf, int adj, fio_prec prec, int nrhs, fio_tile *t) {
    FIO_CHECK_ARG(bf && t && nrhs > 0 && prec >= FIO_PREC_FP64 && prec <= FIO_PREC_SPLIT_FP16);
    const TileCfg c = bf_tile(bf, adj != 0, prec, nrhs);
    *t = fio_tile{c.kc, c.nsplit, c.kmax, c.leaf_sep, c.valu};
    return FIO_OK;
}

// The tuned table as text: one header line naming the operator shape, then one line per entry,
//   fiohss-tune 1 dim=<d> n=<n> q=<q> level_offset=<o>
//   adj=<0|1> prec=<p> cols=<bucket> kc=<kc> nsplit=<s> kmax=<k> leaf_sep=<0|1> valu=<0|1>
static std::string tune_text(const fio_bf_s *bf) {
    std::string out;
    char buf[256];
    snprintf(buf, sizeof buf, "fiohss-tune 1 dim=%d n=%ld q=%d level_offset=%d\n", bf->dim, (long)bf->desc.n,
             bf->q, bf->desc.level_offset);
    out += buf;
    for (const auto &kv : bf->tuned) {
        const int key = kv.first;
        const TileCfg &c = kv.second;
        snprintf(buf, sizeof buf, "adj=%d prec=%d cols=%d %s\n", key & 1, (key >> 1) & 3, 1 << (key >> 3),
                 tile_str(c).c_str());
        out += buf;
    }
    return out;
}

extern "C" fio_status fio_bf_tune_export(fio_bf_t bf, char *buf, size_t len, size_t *needed) {
    FIO_CHECK_ARG(bf);
    std::string t;
    {
        std::lock_guard<std::mutex> lk(bf->tune_mu);
        t = tune_text(bf);
    }
    if (needed) *needed = t.size() + 1;
    if (!buf) return FIO_OK;
    FIO_CHECK_ARG(len >= t.size() + 1);
    memcpy(buf, t.c_str(), t.size() + 1);
    return FIO_OK;
}

// value of "name=<int>" in a line (false when absent or malformed)
static bool field(const std::string &line, const char *name, long *v) {
    const std::string key = std::string(" ") + name + "=";
    const std::string l = " " + line;
    const size_t at = l.find(key);
    if (at == std::string::npos) return false;
    const char *p = l.c_str() + at + key.size();
    char *end = nullptr;
    const long x = strtol(p, &end, 10);
    if (end == p || (*end != 0 && *end != ' ' && *end != '\r')) return false;
    *v = x;
    return true;
}

extern "C" fio_status fio_bf_tune_import(fio_bf_t bf, const char *text) {
    FIO_CHECK_ARG(bf && text);
    std::vector<std::string> lines;
    {
        std::string cur;
        for (const char *p = text; *p; ++p) {
            if (*p == '\n') {
                lines.push_back(cur);
                cur.clear();
            } else {
                cur += *p;
            }
        }
        if (!cur.empty()) lines.push_back(cur);
    }
    FIO_CHECK_ARG(!lines.empty() && lines[0].rfind("fiohss-tune 1 ", 0) == 0);
    long d = 0, n = 0, q = 0, o = 0;
    FIO_CHECK_ARG(field(lines[0], "dim", &d) && field(lines[0], "n", &n) && field(lines[0], "q", &q) &&
                  field(lines[0], "level_offset", &o));
    // a table tuned for another operator shape is refused
    FIO_CHECK_ARG(d == bf->dim && n == (long)bf->desc.n && q == bf->q && o == bf->desc.level_offset);
    std::map<int, TileCfg> tab;
    for (size_t i = 1; i < lines.size(); ++i) {
        if (lines[i].empty()) continue;
        long adj, prec, cols, kc, ns, km, ls, va;
        FIO_CHECK_ARG(field(lines[i], "adj", &adj) && field(lines[i], "prec", &prec) && field(lines[i], "cols", &cols) &&
                      field(lines[i], "kc", &kc) && field(lines[i], "nsplit", &ns) && field(lines[i], "kmax", &km) &&
                      field(lines[i], "leaf_sep", &ls) && field(lines[i], "valu", &va));
        FIO_CHECK_ARG((adj == 0 || adj == 1) && prec >= FIO_PREC_FP64 && prec <= FIO_PREC_SPLIT_FP16);
        FIO_CHECK_ARG(cols >= 1 && cols <= 64 && (cols & (cols - 1)) == 0);
        const TileCfg c{(int)kc, (int)ns, (int)km, (int)ls, (int)va};
        FIO_CHECK_ARG(tile_valid(bf, c) && (c.valu == 0 || prec == FIO_PREC_SPLIT_FP16));
        tab[tile_key(adj != 0, (fio_prec)prec, (int)cols)] = c;
    }
    std::lock_guard<std::mutex> lk(bf->tune_mu);
    for (const auto &kv : tab) bf->tuned[kv.first] = kv.second;
    return FIO_OK;
}

extern "C" fio_status fio_bf_autotune(fio_bf_t bf, const void *X, long ldx, void *Y, long ldy, int nrhs,
                                     fio_prec prec, int reps, void *ws, size_t ws_bytes, void *stream, char *report,
                                     size_t report_len) {
    FIO_CHECK_ARG(bf && nrhs > 0 && reps > 0 && X && Y && ldx >= bf->N && ldy >= bf->N);
    FIO_CHECK_ARG(prec >= FIO_PREC_FP64 && prec <= FIO_PREC_SPLIT_FP16);
    if (prec == FIO_PREC_FP32 && !bf->f32.p) return FIO_ERR_ARG;
    if (prec == FIO_PREC_SPLIT_FP16 && !bf->split16) return FIO_ERR_ARG;
    if (bf->dim == 2 && prec == FIO_PREC_SPLIT_FP16) return FIO_ERR_ARG;
    const size_t need = bf_ws_bytes(bf, nrhs, prec);
    if (ws && ws_bytes < need) return FIO_ERR_ARG;
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        if (!ws) {
            std::lock_guard<std::mutex> lk(bf->ws_mu);
            if (bf->ws.bytes < need) {
                FIO_HIP(hipStreamSynchronize(s));
                bf->ws.alloc(need);
            }
            ws = bf->ws.p;
        }
        hipEvent_t e0, e1;
        FIO_HIP(hipEventCreate(&e0));
        FIO_HIP(hipEventCreate(&e1));
        std::string rep;
        const std::vector<TileCfg> cand = tile_candidates(bf, prec);
        for (int adj = 0; adj < 2; ++adj) {
            const int key = tile_key(adj != 0, prec, nrhs);
            float best = -1.f;
            TileCfg bc{};
            for (const TileCfg &c : cand) {
                {
                    std::lock_guard<std::mutex> lk(bf->tune_mu);
                    bf->tuned[key] = c;
                }
                bf_apply_impl(bf, adj != 0, (const double2 *)X, ldx, (double2 *)Y, ldy, nrhs, prec, ws, s);
                FIO_HIP(hipEventRecord(e0, s));
                for (int r = 0; r < reps; ++r)
                    bf_apply_impl(bf, adj != 0, (const double2 *)X, ldx, (double2 *)Y, ldy, nrhs, prec, ws, s);
                FIO_HIP(hipEventRecord(e1, s));
                FIO_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                FIO_HIP(hipEventElapsedTime(&ms, e0, e1));
                ms /= (float)reps;
                char buf[160];
                snprintf(buf, sizeof buf, "%s %s %.4f ms; ", adj ? "adj" : "fwd", tile_str(c).c_str(), ms);
                rep += buf;
                if (best < 0.f || ms < best) {
                    best = ms;
                    bc = c;
                }
            }
            std::lock_guard<std::mutex> lk(bf->tune_mu);
            bf->tuned[key] = bc;
            char buf[160];
            snprintf(buf, sizeof buf, "chosen %s %s; ", adj ? "adj" : "fwd", tile_str(bc).c_str());
            rep += buf;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (report && report_len) {
            const size_t n = rep.size() < report_len - 1 ? rep.size() : report_len - 1;
            memcpy(report, rep.data(), n);
            report[n] = 0;
        }
        return FIO_OK;
    });
}

extern "C" void fio_bf_destroy(fio_bf_t bf) { delete bf; }

extern "C" void fio_set_fused(int on) { set_fused_disabled(on == 0); }
extern "C" void fio_set_leaf_fused(int on) { g_leaf_fused_off = on == 0; }

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
