// Butterfly factorization of a 2D discrete FIO on gfx950 (Section 2.2 on a
// quadtree, the phases of Sections 5.2 and 5.3), for the levels where the outermost factors
// meet at the middle level (L' = h, no B or C factor): K~ = U M V.
//
// Trees: n = 2^L points per dimension, N = n^2, h = ceil(L/2), lc = L - h.
//   V side: pairs (tau' at spatial level lc, sigma at frequency level h),
//           pair index tau' * 4^h + sigma;
//   U side: pairs (tau at spatial level h, sigma' at frequency level lc),
//           pair index tau * 4^lc + sigma';
//   M couples U pair (tau, sigma') with the V pairs (parent^(h-lc)(tau), sigma)
//   for the rr = 4^(h-lc) frequency boxes sigma of level h inside sigma'.
// Box indices are Morton codes of the box coordinates (first coordinate on the
// odd bits), so the points of a box are contiguous in Morton order and the
// children of box v are 4v .. 4v+3.
//
// Factor layout (complex entries, column-major blocks; the import/export layout):
//   V: block p (V pair), q^2 x b^2, entry (i, s) at p q^2 b^2 + s q^2 + i
//   M: block u * 4^h + sigma (u, sigma at level h), q^2 x q^2, entry (i, j) at
//      blk q^4 + j q^2 + i
//   U: block p (U pair), b^2 x q^2, entry (s, i) at p q^2 b^2 + i b^2 + s
// with s the Morton index of a point inside its box and i = i1 q + i2 the
// tensor Chebyshev index.  The adjoint applies read conjugate-transposed copies
// (built on the device from the forward factors) so that every step streams its
// factor with consecutive lanes on consecutive rows:
//   Vadj block sigma * 4^lc + tau' = V_{tau',sigma}^*  (b^2 x q^2)
//   Madj block (tau' * 4^h + sigma) * rr + d = M_{tau' rr + d, sigma}^*  (q^2 x q^2)
//   Uadj block p = U_p^*  (q^2 x b^2)
//
// Apply: one kernel per factor.  A workgroup owns one output block (a pair's
// q^2 coefficients, or a leaf box's b^2 values) for a chunk of KC right-hand
// sides; lane r accumulates row r for the KC columns; the factor block streams
// from HBM once per chunk, the input coefficients are wave-uniform reads.  The
// leaf-box sums over 4^lc blocks are split over workgroups and reduced in a
// fixed order (deterministic results).
//
// Coefficient buffers: entry (pair p, coefficient i, column c) at
// (p q^2 + i) * ldc + c with ldc = nrhs rounded up to KC.
#include <cmath>

#include "bf.h"
#include "ddmath.h"
#include "timing.h"

namespace fio {

namespace {

struct G2 {
    int n, L, h, lc, b, hb, q, q2, b2;
    long S, T, rr;                // 4^h, 4^lc, 4^(h-lc)
    double a0, a1;                // phase parameters
    int iso;                      // Section 5.3's isotropic phase (c2 = c1)
    int hankel;                   // Section 5.3's amplitude
};

G2 g2_of(const fio_bf_s *bf) {
    G2 g;
    g.n = (int)bf->n1;
    g.L = bf->L;
    g.h = bf->h;
    g.lc = bf->lc;
    g.b = bf->b;
    g.hb = bf->hb;
    g.q = bf->q;
    g.q2 = bf->q * bf->q;
    g.b2 = bf->b * bf->b;
    g.S = 1L << (2 * bf->h);
    g.T = 1L << (2 * bf->lc);
    g.rr = g.S / g.T;
    g.a0 = bf->desc.c0;
    g.a1 = bf->desc.c1;
    g.iso = bf->desc.phase_kind == FIO_PHASE2_ISO;
    g.hankel = bf->desc.amp_kind == FIO_AMP_HANKEL;
    return g;
}

// --- geometry and phase (Sections 5.2 and 5.3) ---------------------------------------------
__device__ __forceinline__ void demorton(long m, int bits, int &j1, int &j2) {
    j1 = 0;
    j2 = 0;
    for (int k = 0; k < bits; ++k) {
        j1 |= (int)((m >> (2 * k + 1)) & 1) << k;
        j2 |= (int)((m >> (2 * k)) & 1) << k;
    }
}

// user (lexicographic) index of the point with Morton code m
__device__ __forceinline__ long lex_of(long m, int L, int n) {
    int j1, j2;
    demorton(m, L, j1, j2);
    return (long)j1 * n + j2;
}

// Phases are formed in double-double arithmetic from exact points (ddmath.h; box corners and
// grid points are binary fractions or integers, Chebyshev points are center + (w/2) t_i) and
// reduced modulo 1 before the single rounding of an entry; Lagrange values are taken in the
// reference coordinate of the point in its box.
__device__ dd rho2_dd(const G2 &g, dd x1, dd x2, dd k1, dd k2) {
    dd s1, co1, s2, co2;
    dd_sincospi(dd_ldexp(x1, 2.0), s1, co1);
    dd_sincospi(dd_ldexp(x2, 2.0), s2, co2);
    const dd c1 = dd_add(dd_of(g.a0), dd_mul_d(dd_mul(s1, s2), g.a1));
    const dd c2 = g.iso ? c1 : dd_add(dd_of(g.a0), dd_mul_d(dd_mul(co1, co2), g.a1));
    const dd t1 = dd_mul(c1, k1), t2 = dd_mul(c2, k2);
    return dd_sqrt(dd_add(dd_mul(t1, t1), dd_mul(t2, t2)));
}

// box geometry: spatial box j at level l is [j1 2^-l, (j1 + 1) 2^-l] x [..];
// frequency box j at level l is [-n/2 + j1 n 2^-l, ..] x [..]
__device__ __forceinline__ void s_box(int l, long box, double &lo1, double &lo2, double &w) {
    int j1, j2;
    demorton(box, l, j1, j2);
    w = ldexp(1.0, -l);
    lo1 = j1 * w;
    lo2 = j2 * w;
}

__device__ __forceinline__ void f_box(const G2 &g, int l, long box, double &lo1, double &lo2, double &w) {
    int j1, j2;
    demorton(box, l, j1, j2);
    w = ldexp((double)g.n, -l);
    lo1 = -0.5 * g.n + j1 * w;
    lo2 = -0.5 * g.n + j2 * w;
}

// --- factor generation ------------------------------------------------------------
// V(i, s) of pair p = tau' * S + sigma:
//   exp(2 pi i (y.(xi_s - gamma_i) + rho(y, xi_s) - rho(y, gamma_i))) q_i(xi_s)
__global__ void gen2_V(G2 g, Nodes tn, double2 *out) {
    const size_t nV = (size_t)g.T * g.S * g.q2 * g.b2;
    const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= nV) return;
    const int i = (int)(id % g.q2);
    const int s = (int)((id / g.q2) % g.b2);
    const long p = (long)(id / ((size_t)g.q2 * g.b2));
    const long tau = p / g.S, sigma = p % g.S;
    double y1, y2, ws, f1, f2, wf;
    s_box(g.lc, tau, y1, y2, ws);
    y1 += 0.5 * ws;
    y2 += 0.5 * ws;
    f_box(g, g.h, sigma, f1, f2, wf);
    int a1, a2;
    demorton(s, g.hb, a1, a2);
    const double k1 = f1 + a1, k2 = f2 + a2;                   // xi_s (integers)
    const int i1 = i / g.q, i2 = i % g.q;
    const double c1 = f1 + 0.5 * wf, c2 = f2 + 0.5 * wf, hw = 0.5 * wf;
    const dd g1 = dd_add(dd_of(c1), dd_ldexp(tn.t(i1), hw)), g2 = dd_add(dd_of(c2), dd_ldexp(tn.t(i2), hw));
    const dd lin = dd_add(dd_frac(dd_mul_d(dd_sub(dd_of(k1), g1), y1)), dd_frac(dd_mul_d(dd_sub(dd_of(k2), g2), y2)));
    const dd nl = dd_sub(rho2_dd(g, dd_of(y1), dd_of(y2), dd_of(k1), dd_of(k2)), rho2_dd(g, dd_of(y1), dd_of(y2), g1, g2));
    const double lag = dd_lagrange(dd_of((k1 - c1) / hw), i1, tn) * dd_lagrange(dd_of((k2 - c2) / hw), i2, tn);
    const double2 e = dd_expi2pi(dd_add(lin, dd_frac(nl)));
    out[id] = zc(e.x * lag, e.y * lag);
}

// M(i, j) of block u * S + sigma: k(z_u,i, gamma_sigma,j)
__global__ void gen2_M(G2 g, Nodes tn, double2 *out) {
    const size_t nM = (size_t)g.S * g.S * g.q2 * g.q2;
    const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= nM) return;
    const int i = (int)(id % g.q2);
    const int j = (int)((id / g.q2) % g.q2);
    const long blk = (long)(id / ((size_t)g.q2 * g.q2));
    const long u = blk / g.S, sigma = blk % g.S;
    double z1, z2, ws, f1, f2, wf;
    s_box(g.h, u, z1, z2, ws);
    f_box(g, g.h, sigma, f1, f2, wf);
    const double hs = 0.5 * ws, hf = 0.5 * wf;
    const dd x1 = dd_add(dd_of(z1 + hs), dd_ldexp(tn.t(i / g.q), hs));
    const dd x2 = dd_add(dd_of(z2 + hs), dd_ldexp(tn.t(i % g.q), hs));
    const dd k1 = dd_add(dd_of(f1 + hf), dd_ldexp(tn.t(j / g.q), hf));
    const dd k2 = dd_add(dd_of(f2 + hf), dd_ldexp(tn.t(j % g.q), hf));
    const dd r = rho2_dd(g, x1, x2, k1, k2);
    const dd lin = dd_add(dd_frac(dd_mul(x1, k1)), dd_frac(dd_mul(x2, k2)));
    const double2 e = dd_expi2pi(dd_add(lin, dd_frac(r)));
    if (!g.hankel) {
        out[id] = e;
        return;
    }
    // a = H0^(1)(t) exp(-i t), t = 2 pi rho (H0^(1) = J0 + i Y0): a is smooth in t, so t is taken
    // rounded once; the oscillation of H0^(1) cancels against exp(-i t) at the same t.
    // Chebyshev points never fall on xi = 0, so rho > 0 here.
    const double t = 2.0 * M_PI * dd_val(r);
    double st, ct;
    sincos(t, &st, &ct);
    const double jr = j0(t), yi = y0(t);
    const double ar = jr * ct + yi * st, ai = yi * ct - jr * st;    // (J0 + i Y0)(cos t - i sin t)
    out[id] = zc(ar * e.x - ai * e.y, ar * e.y + ai * e.x);
}

// U(s, i) of pair p = tau * T + sigma':
//   exp(2 pi i ((x_s - z_i).eta + rho(x_s, eta) - rho(z_i, eta))) p_i(x_s)
__global__ void gen2_U(G2 g, Nodes tn, double2 *out) {
    const size_t nU = (size_t)g.S * g.T * g.q2 * g.b2;
    const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= nU) return;
    const int s = (int)(id % g.b2);
    const int i = (int)((id / g.b2) % g.q2);
    const long p = (long)(id / ((size_t)g.q2 * g.b2));
    const long tau = p / g.T, sig = p % g.T;
    double t1, t2, ws, e1, e2, wf;
    s_box(g.h, tau, t1, t2, ws);
    f_box(g, g.lc, sig, e1, e2, wf);
    e1 += 0.5 * wf;
    e2 += 0.5 * wf;                                            // eta_sigma'
    int a1, a2;
    demorton(s, g.hb, a1, a2);
    const double hs = 0.5 * ws, c1 = t1 + hs, c2 = t2 + hs;
    const double x1 = t1 + a1 * (1.0 / g.n), x2 = t2 + a2 * (1.0 / g.n);   // grid points, exact
    const int i1 = i / g.q, i2 = i % g.q;
    const dd z1 = dd_add(dd_of(c1), dd_ldexp(tn.t(i1), hs)), z2 = dd_add(dd_of(c2), dd_ldexp(tn.t(i2), hs));
    const dd lin = dd_add(dd_frac(dd_mul_d(dd_sub(dd_of(x1), z1), e1)), dd_frac(dd_mul_d(dd_sub(dd_of(x2), z2), e2)));
    const dd nl = dd_sub(rho2_dd(g, dd_of(x1), dd_of(x2), dd_of(e1), dd_of(e2)), rho2_dd(g, z1, z2, dd_of(e1), dd_of(e2)));
    const double lag = dd_lagrange(dd_of((x1 - c1) / hs), i1, tn) * dd_lagrange(dd_of((x2 - c2) / hs), i2, tn);
    const double2 e = dd_expi2pi(dd_add(lin, dd_frac(nl)));
    out[id] = zc(e.x * lag, e.y * lag);
}

// conjugate-transposed copies of the three factors (layout in the file header)
__global__ void adj2_V(G2 g, const double2 *V, double2 *Va) {
    const size_t nV = (size_t)g.T * g.S * g.q2 * g.b2;
    const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= nV) return;
    // destination order: block sigma * T + tau, entry (s, i) at i b2 + s
    const int s = (int)(id % g.b2);
    const int i = (int)((id / g.b2) % g.q2);
    const long blk = (long)(id / ((size_t)g.q2 * g.b2));
    const long sigma = blk / g.T, tau = blk % g.T;
    const double2 v = V[((size_t)(tau * g.S + sigma) * g.b2 + s) * g.q2 + i];
    Va[id] = zc(v.x, -v.y);
}

__global__ void adj2_M(G2 g, const double2 *M, double2 *Ma) {
    const size_t nM = (size_t)g.S * g.S * g.q2 * g.q2;
    const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= nM) return;
    // destination block (tau' * S + sigma) * rr + d holds M_{tau' rr + d, sigma}^*: entry (j, i) at i q2 + j
    const int j = (int)(id % g.q2);
    const int i = (int)((id / g.q2) % g.q2);
    const long blk = (long)(id / ((size_t)g.q2 * g.q2));
    const long d = blk % g.rr, p = blk / g.rr;
    const long taup = p / g.S, sigma = p % g.S;
    const long u = taup * g.rr + d;
    const double2 v = M[((size_t)(u * g.S + sigma) * g.q2 + j) * g.q2 + i];
    Ma[id] = zc(v.x, -v.y);
}

__global__ void adj2_U(G2 g, const double2 *U, double2 *Ua) {
    const size_t nU = (size_t)g.S * g.T * g.q2 * g.b2;
    const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= nU) return;
    // destination: block p, entry (i, s) at s q2 + i
    const int i = (int)(id % g.q2);
    const int s = (int)((id / g.q2) % g.b2);
    const long p = (long)(id / ((size_t)g.q2 * g.b2));
    const double2 v = U[((size_t)p * g.q2 + i) * g.b2 + s];
    Ua[id] = zc(v.x, -v.y);
}

__global__ void cvt2_f32(const double2 *in, float2 *out, size_t n) {
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id < n) {
        double2 v = in[id];
        out[id] = make_float2((float)v.x, (float)v.y);
    }
}

// --- apply -------------------------------------------------------------------------
enum Step { VF, MF, UF, UA, MA, VA };

template <typename T> struct K2Args {
    G2 g;
    const cpx<T> *A;        // factor blocks of this step
    const cpx<T> *cin;      // input coefficients (MF, UF, MA, VA)
    const double2 *X;       // input vector (VF: frequency side, UA: spatial side)
    long ldx;
    cpx<T> *cout;           // output coefficients (VF, MF, UA, MA)
    double2 *Y;             // output vector (UF: spatial side, VA: frequency side), when nsplit == 1
    cpx<T> *part;           // split partial sums (UF, VA), when nsplit > 1
    long ldy;
    int nrhs, ldc;          // right-hand sides, coefficient row stride
    int nb, nsplit;         // blocks per output, splits of the block range
    int fint;               // frequency-side vectors in Morton order (no index map)
    long nout;              // output blocks (workgroup rows) of the launch
};

template <typename C> __device__ __forceinline__ C to_c(double2 v);
template <> __device__ __forceinline__ double2 to_c<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 to_c<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ double2 to_z(double2 v) { return v; }
__device__ __forceinline__ double2 to_z(float2 v) { return zc(v.x, v.y); }

// rows of one output block / columns of one factor block, per step
template <int STEP> __device__ __forceinline__ int rows_of(const G2 &g) {
    return (STEP == UF || STEP == VA) ? g.b2 : g.q2;
}
template <int STEP> __device__ __forceinline__ int cols_of(const G2 &g) {
    return (STEP == VF || STEP == UA) ? g.b2 : g.q2;
}

template <typename T, int KC, int STEP>
__global__ void __launch_bounds__(128) k2_step(K2Args<T> a) {
    using C = cpx<T>;
    const G2 &g = a.g;
    const int R = rows_of<STEP>(g), CC = cols_of<STEP>(g);
    const int r = threadIdx.x;
    // grid: x = column chunk (fastest, so the chunks of one output block run together and share
    // its factor blocks through L2), y (+ z) = output block, z = split for the leaf-box sums
    const bool splitk = STEP == UF || STEP == VA;
    const long o = splitk ? (long)blockIdx.y : (long)blockIdx.y + (long)blockIdx.z * gridDim.y;
    const int split = splitk ? (int)blockIdx.z : 0;
    const int c0 = blockIdx.x * KC;
    if (o >= a.nout) return;
    const int nc = min(KC, a.nrhs - c0);
    const bool act = r < R;
    C acc[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] = czero<C>();
    const int nbs = a.nb / a.nsplit;
    // lanes beyond the block's rows read its last row (no lane condition on the loads, which would
    // put each one in a block of its own and wait for it there) and store nothing
    const int rc = act ? r : R - 1;
    for (int bb = split * nbs; bb < (split + 1) * nbs; ++bb) {
        const C *Ab = a.A + ((size_t)o * a.nb + bb) * R * CC + rc;
        if (STEP == VF || STEP == UA) {
            // input from a user vector: the b^2 points of one leaf box
            const long base = (STEP == VF) ? (o % g.S) * g.b2 : (o / g.T) * g.b2;
            const bool internal = STEP == VF && a.fint;
            for (int j = 0; j < CC; ++j) {
                const C av = Ab[(size_t)j * R];
                const long m = base + j;
                const long row = internal ? m : lex_of(m, g.L, g.n);
                const double2 *xp = a.X + row + (size_t)c0 * a.ldx;
#pragma unroll
                for (int c = 0; c < KC; ++c) {
                    const C x = c < nc ? to_c<C>(xp[(size_t)c * a.ldx]) : czero<C>();
                    cfma(acc[c], av, x);
                }
            }
        } else {
            long srow;
            if (STEP == MF) {
                const long u = o / g.T, v = o % g.T;
                srow = (u / g.rr) * g.S + v * g.rr + bb;
            } else if (STEP == UF) {
                srow = o * g.T + bb;
            } else if (STEP == MA) {
                const long taup = o / g.S, sigma = o % g.S;
                srow = (taup * g.rr + bb) * g.T + sigma / g.rr;
            } else {   // VA
                srow = bb * g.S + o;
            }
            const C *xp = a.cin + (size_t)srow * g.q2 * a.ldc + c0;
#pragma unroll 3
            for (int j = 0; j < CC; ++j) {
                const C av = Ab[(size_t)j * R];
#pragma unroll
                for (int c = 0; c < KC; ++c) cfma(acc[c], av, xp[(size_t)j * a.ldc + c]);
            }
        }
    }
    if (!act) return;
    if (STEP == UF || STEP == VA) {
        if (a.nsplit > 1) {
            C *pp = a.part + (((size_t)split * a.nout + o) * R + r) * a.ldc + c0;
#pragma unroll
            for (int c = 0; c < KC; ++c) pp[c] = acc[c];
        } else {
            const long m = o * g.b2 + r;
            const long row = (STEP == VA && a.fint) ? m : lex_of(m, g.L, g.n);
            double2 *yp = a.Y + row + (size_t)c0 * a.ldy;
#pragma unroll
            for (int c = 0; c < KC; ++c)
                if (c < nc) yp[(size_t)c * a.ldy] = to_z(acc[c]);
        }
    } else {
        C *cp = a.cout + ((size_t)o * g.q2 + r) * a.ldc + c0;
#pragma unroll
        for (int c = 0; c < KC; ++c) cp[c] = acc[c];
    }
}

// VF / UA: the input is the user vector on one leaf box (b^2 points, gathered through the
// index map), shared by G consecutive output pairs of the workgroup: it is staged once in
// LDS and read back as wave-uniform broadcasts, while the G factor blocks stream from HBM.
//   VF: box sigma, outputs (tau' = t0 + g) * S + sigma;  UA: box tau, outputs tau * T + v0 + g.
template <typename T, int KC, int STEP, int G>
__global__ void __launch_bounds__(128) k2_leaf_in(K2Args<T> a) {
    using C = cpx<T>;
    const G2 &g = a.g;
    constexpr int MAXB2 = 128;
    __shared__ C xs[MAXB2 * KC];
    const int R = g.q2, CC = g.b2;
    const int r = threadIdx.x;
    const long groups = g.T / G;
    const long wg = (long)blockIdx.y + (long)blockIdx.z * gridDim.y;   // x = column chunk (fastest)
    if (wg >= a.nout) return;
    const long box = wg / groups;
    const long first = (wg % groups) * G;
    const int c0 = blockIdx.x * KC;
    const int nc = min(KC, a.nrhs - c0);
    const bool internal = STEP == VF && a.fint;
    for (int e = threadIdx.x; e < CC * KC; e += blockDim.x) {
        const int j = e / KC, c = e % KC;
        const long m = box * g.b2 + j;
        const long row = internal ? m : lex_of(m, g.L, g.n);
        xs[e] = c < nc ? to_c<C>(a.X[row + (size_t)(c0 + c) * a.ldx]) : czero<C>();
    }
    __syncthreads();
    if (r >= R) return;
    for (int gg = 0; gg < G; ++gg) {
        const long o = STEP == VF ? (first + gg) * g.S + box : box * g.T + first + gg;
        const C *Ab = a.A + (size_t)o * R * CC + r;
        C acc[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) acc[c] = czero<C>();
#pragma unroll 4
        for (int j = 0; j < CC; ++j) {
            const C av = Ab[(size_t)j * R];
#pragma unroll
            for (int c = 0; c < KC; ++c) cfma(acc[c], av, xs[j * KC + c]);
        }
        C *cp = a.cout + ((size_t)o * g.q2 + r) * a.ldc + c0;
#pragma unroll
        for (int c = 0; c < KC; ++c) cp[c] = acc[c];
    }
}

// fixed-order sum of the split partials, scattered to the user vector
template <typename T>
__global__ void k2_reduce(G2 g, const cpx<T> *part, int nsplit, long nout, int ldc, int nrhs, int frequency,
                          int fint, double2 *Y, long ldy) {
    const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t tot = (size_t)nout * g.b2 * nrhs;
    if (id >= tot) return;
    const int c = (int)(id % nrhs);
    const long m = (long)(id / nrhs);               // o * b2 + r
    cpx<T> s = czero<cpx<T>>();
    for (int k = 0; k < nsplit; ++k) s = cadd(s, part[((size_t)k * nout * g.b2 + m) * ldc + c]);
    const long row = (frequency && fint) ? m : lex_of(m, g.L, g.n);
    Y[row + (size_t)c * ldy] = to_z(s);
}

__global__ void k_perm2(int n, int L, int to_int, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs) {
    const size_t N = (size_t)n * n;
    const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= N * nrhs) return;
    const long m = (long)(id % N);
    const size_t c = id / N;
    const long l = lex_of(m, L, n);
    if (to_int)
        Y[m + c * ldy] = X[l + c * ldx];
    else
        Y[l + c * ldy] = X[m + c * ldx];
}


int nsplit_of(long nb) { return (int)(nb < 16 ? nb : 16); }

// output pairs per workgroup of the leaf-input steps: 8 when the box has that many partners
// grid for `n` workgroup rows with the column chunks fastest: (chunks, min(n, 32768), rest)
dim3 grid_rows(unsigned chunks, long n) {
    const long gy = n < 32768 ? n : 32768;
    return dim3(chunks, (unsigned)gy, (unsigned)((n + gy - 1) / gy));
}

template <typename T, int KC, int STEP>
void launch_leaf_in(const K2Args<T> &a_in, const G2 &g, unsigned chunks, unsigned blk, hipStream_t s) {
    K2Args<T> a = a_in;
    const long G = g.T >= 8 ? 8 : 1;
    a.nout = g.S * (g.T / G);
    if (G == 8)
        k2_leaf_in<T, KC, STEP, 8><<<grid_rows(chunks, a.nout), blk, 0, s>>>(a);
    else
        k2_leaf_in<T, KC, STEP, 1><<<grid_rows(chunks, a.nout), blk, 0, s>>>(a);
}

// KC columns per workgroup: 8 for few right-hand sides, 16 for wide blocks (the HSS sample
// blocks), which halves how often the factors stream while the FMAs per factor entry double
template <typename T, int KC>
void apply2k(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs, const cpx<T> *F,
             const cpx<T> *Fa, void *ws, bool fint, int nsplit, hipStream_t s) {
    using C = cpx<T>;
    const G2 g = g2_of(bf);
    const int ldc = (nrhs + KC - 1) / KC * KC;
    const size_t ncoef = (size_t)bf->N * g.q2 * ldc;
    C *c1 = reinterpret_cast<C *>(ws);
    C *c2 = c1 + ncoef;
    C *part = c2 + ncoef;
    const unsigned chunks = (unsigned)(ldc / KC);
    const bool f64 = sizeof(T) == 8;
    const unsigned blkq = 64 * ((g.q2 + 63) / 64), blkb = 64 * ((g.b2 + 63) / 64);
    const long NP = bf->N;                            // pairs on either side
    // reduction split of the U / V^* steps: a power of two dividing the T partner blocks, at most
    // nsplit_of(T) (the workspace holds that many partial sums)
    int nsp = nsplit_of(g.T);
    if (nsplit > 0 && nsplit < nsp && g.T % nsplit == 0) nsp = nsplit;
    K2Args<T> a{};
    a.g = g;
    a.nrhs = nrhs;
    a.ldc = ldc;
    a.fint = fint ? 1 : 0;
    if (!adj) {
        const C *V = F + bf->offV, *M = F + bf->offM, *U = F + bf->offU;
        {
            FIO_TIMED(f64 ? "bf2_V_f64" : "bf2_V_f32", s);
            K2Args<T> v = a;
            v.A = V; v.X = X; v.ldx = ldx; v.cout = c1; v.nb = 1; v.nsplit = 1;
            launch_leaf_in<T, KC, VF>(v, g, chunks, blkq, s);
        }
        {
            FIO_TIMED(f64 ? "bf2_M_f64" : "bf2_M_f32", s);
            K2Args<T> m = a;
            m.A = M; m.cin = c1; m.cout = c2; m.nb = (int)g.rr; m.nsplit = 1;
            m.nout = NP;
            k2_step<T, KC, MF><<<grid_rows(chunks, NP), blkq, 0, s>>>(m);
        }
        {
            FIO_TIMED(f64 ? "bf2_U_f64" : "bf2_U_f32", s);
            K2Args<T> u = a;
            u.A = U; u.cin = c2; u.Y = Y; u.ldy = ldy; u.part = part; u.nb = (int)g.T; u.nsplit = nsp;
            u.nout = g.S;
            k2_step<T, KC, UF><<<dim3(chunks, (unsigned)g.S, nsp), blkb, 0, s>>>(u);
            if (nsp > 1) {
                const size_t tot = (size_t)g.S * g.b2 * nrhs;
                k2_reduce<T><<<grid1d(tot, 256), 256, 0, s>>>(g, part, nsp, g.S, ldc, nrhs, 0, 0, Y, ldy);
            }
        }
    } else {
        const C *Va = Fa + bf->offV, *Ma = Fa + bf->offM, *Ua = Fa + bf->offU;
        {
            FIO_TIMED(f64 ? "bf2_U_f64" : "bf2_U_f32", s);
            K2Args<T> u = a;
            u.A = Ua; u.X = X; u.ldx = ldx; u.cout = c2; u.nb = 1; u.nsplit = 1;
            launch_leaf_in<T, KC, UA>(u, g, chunks, blkq, s);
        }
        {
            FIO_TIMED(f64 ? "bf2_M_f64" : "bf2_M_f32", s);
            K2Args<T> m = a;
            m.A = Ma; m.cin = c2; m.cout = c1; m.nb = (int)g.rr; m.nsplit = 1;
            m.nout = NP;
            k2_step<T, KC, MA><<<grid_rows(chunks, NP), blkq, 0, s>>>(m);
        }
        {
            FIO_TIMED(f64 ? "bf2_V_f64" : "bf2_V_f32", s);
            K2Args<T> v = a;
            v.A = Va; v.cin = c1; v.Y = Y; v.ldy = ldy; v.part = part; v.nb = (int)g.T; v.nsplit = nsp;
            v.nout = g.S;
            k2_step<T, KC, VA><<<dim3(chunks, (unsigned)g.S, nsp), blkb, 0, s>>>(v);
            if (nsp > 1) {
                const size_t tot = (size_t)g.S * g.b2 * nrhs;
                k2_reduce<T><<<grid1d(tot, 256), 256, 0, s>>>(g, part, nsp, g.S, ldc, nrhs, 1, a.fint, Y, ldy);
            }
        }
    }
    FIO_HIP(hipGetLastError());
}

template <typename T>
void apply2(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs, const cpx<T> *F,
            const cpx<T> *Fa, void *ws, bool fint, hipStream_t s) {
    // column chunk and reduction split: tuned (fio_bf_autotune) or 16 columns for wide blocks
    const TileCfg c = bf_tile(bf, adj, sizeof(T) == 8 ? FIO_PREC_FP64 : FIO_PREC_FP32, nrhs);
    const int kc = c.kc ? c.kc : (nrhs >= 16 ? 16 : 8);
    if (kc == 16)
        apply2k<T, 16>(bf, adj, X, ldx, Y, ldy, nrhs, F, Fa, ws, fint, c.nsplit, s);
    else
        apply2k<T, 8>(bf, adj, X, ldx, Y, ldy, nrhs, F, Fa, ws, fint, c.nsplit, s);
}

}  // namespace

// ---------------------------------------------------------------------------
fio_status bf2d_plan(const fio_bf_desc *d, fio_bf_s *bf) {
    if (d->n < 4 || d->n > (1L << 15) || (d->n & (d->n - 1))) return FIO_ERR_ARG;
    if (d->phase_kind < FIO_PHASE2_ANISO || d->phase_kind > FIO_PHASE2_ISO) return FIO_ERR_ARG;
    if (d->amp_kind < FIO_AMP_ONE || d->amp_kind > FIO_AMP_HANKEL) return FIO_ERR_ARG;
    if (d->amp_kind == FIO_AMP_GAUSSIAN_SUM) return FIO_ERR_UNSUPPORTED;   // 1D amplitude only
    if (d->q < 2 || d->q > 16 || d->level_offset < 1) return FIO_ERR_ARG;
    int L = 0;
    while ((1L << L) < d->n) ++L;
    const int h = (L + 1) / 2;
    if (L - d->level_offset > h) return FIO_ERR_UNSUPPORTED;   // transfer levels are not built in 2D
    const int b = (int)(d->n >> h);
    if (b * b > 128) return FIO_ERR_UNSUPPORTED;                // a leaf box must fit one workgroup
    if (h > 7) return FIO_ERR_UNSUPPORTED;                      // 4^h leaf boxes on one grid axis
    if (d->q * d->q > 128) return FIO_ERR_UNSUPPORTED;
    bf->desc = *d;
    bf->desc.amp_centers = nullptr;          // not used in 2D
    bf->dim = 2;
    bf->n1 = d->n;
    bf->N = d->n * d->n;
    bf->L = L;
    bf->h = h;
    bf->lc = L - h;
    bf->Lp = h;
    bf->nl = 0;
    bf->q = d->q;
    bf->b = b;
    bf->hb = 0;
    while ((1 << bf->hb) < b) ++bf->hb;
    const size_t q2 = (size_t)d->q * d->q, b2 = (size_t)b * b;
    const size_t S = 1UL << (2 * h), T = 1UL << (2 * bf->lc);
    bf->offV = 0;
    bf->offM = T * S * q2 * b2;
    bf->offU = bf->offM + S * S * q2 * q2;
    bf->total = bf->offU + S * T * q2 * b2;
    return FIO_OK;
}

size_t bf2d_ws_bytes(const fio_bf_s *bf, int nrhs, fio_prec prec) {
    if (prec == FIO_PREC_SPLIT_FP16) return 0;
    const size_t es = prec == FIO_PREC_FP64 ? sizeof(double2) : sizeof(float2);
    const size_t ldc = (size_t)(nrhs + 15) / 16 * 16;     // the larger of the two column chunkings
    const size_t T = 1UL << (2 * bf->lc);
    const size_t ns = (size_t)nsplit_of((long)T);
    return (2 * (size_t)bf->N * bf->q * bf->q * ldc + (ns > 1 ? ns * (size_t)bf->N * ldc : 0)) * es;
}

void bf2d_generate(fio_bf_s *bf, hipStream_t s) {
    const G2 g = g2_of(bf);
    double2 *base = bf->f64.as<double2>();
    const size_t nV = bf->offM - bf->offV, nM = bf->offU - bf->offM, nU = bf->total - bf->offU;
    const Nodes tn = make_nodes(bf->q);
    gen2_V<<<grid1d(nV, 256), 256, 0, s>>>(g, tn, base + bf->offV);
    gen2_M<<<grid1d(nM, 256), 256, 0, s>>>(g, tn, base + bf->offM);
    gen2_U<<<grid1d(nU, 256), 256, 0, s>>>(g, tn, base + bf->offU);
    FIO_HIP(hipGetLastError());
}

// adjoint copies and the single-precision copies of both
void bf2d_finish(fio_bf_s *bf, hipStream_t s) {
    const G2 g = g2_of(bf);
    const size_t nV = bf->offM - bf->offV, nM = bf->offU - bf->offM, nU = bf->total - bf->offU;
    bf->adj64.alloc(bf->total * sizeof(double2));
    const double2 *F = bf->f64.as<double2>();
    double2 *A = bf->adj64.as<double2>();
    adj2_V<<<grid1d(nV, 256), 256, 0, s>>>(g, F + bf->offV, A + bf->offV);
    adj2_M<<<grid1d(nM, 256), 256, 0, s>>>(g, F + bf->offM, A + bf->offM);
    adj2_U<<<grid1d(nU, 256), 256, 0, s>>>(g, F + bf->offU, A + bf->offU);
    if (bf->desc.prec_mask & (1u << FIO_PREC_FP32)) {
        bf->f32.alloc(bf->total * sizeof(float2));
        bf->adj32.alloc(bf->total * sizeof(float2));
        cvt2_f32<<<grid1d(bf->total, 256), 256, 0, s>>>(F, bf->f32.as<float2>(), bf->total);
        cvt2_f32<<<grid1d(bf->total, 256), 256, 0, s>>>(A, bf->adj32.as<float2>(), bf->total);
    }
    FIO_HIP(hipGetLastError());
}

void bf2d_apply(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs, fio_prec prec,
                void *ws, bool fint, hipStream_t s) {
    if (prec == FIO_PREC_FP64)
        apply2<double>(bf, adj, X, ldx, Y, ldy, nrhs, bf->f64.as<double2>(), bf->adj64.as<double2>(), ws, fint, s);
    else if (prec == FIO_PREC_FP32)
        apply2<float>(bf, adj, X, ldx, Y, ldy, nrhs, bf->f32.as<float2>(), bf->adj32.as<float2>(), ws, fint, s);
    else
        throw Err{FIO_ERR_UNSUPPORTED};
}

void permute2d(int n, bool to_internal, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs, hipStream_t s) {
    int L = 0;
    while ((1 << L) < n) ++L;
    const size_t tot = (size_t)n * n * nrhs;
    if (tot == 0) return;
    k_perm2<<<grid1d(tot, 256), 256, 0, s>>>(n, L, to_internal ? 1 : 0, X, ldx, Y, ldy, nrhs);
    FIO_HIP(hipGetLastError());
}

}  // namespace fio

extern "C" fio_status fio_permute2d(long n, int to_internal, const void *X, long ldx, void *Y, long ldy, int nrhs,
                                    void *stream) {
    FIO_CHECK_ARG(n >= 1 && n <= (1L << 15) && (n & (n - 1)) == 0 && nrhs >= 0);
    if (nrhs == 0) return FIO_OK;
    FIO_CHECK_ARG(X && Y && X != Y && ldx >= n * n && ldy >= n * n);
    return fio::guarded([&] {
        fio::permute2d((int)n, to_internal != 0, (const double2 *)X, ldx, (double2 *)Y, ldy, nrhs,
                       fio::as_stream(stream));
        return FIO_OK;
    });
}
