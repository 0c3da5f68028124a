// Randomized black-box HSS construction (Section 3) on gfx950.
//
// The level loop runs on the host because every level's sizes depend on the
// ranks found below it; everything else runs on the device:
//   * basis lift / projection of the test and sample matrices: batched GEMMs;
//   * the sampling matvec: the caller's callback (the FIO path passes K~^* K~);
//   * the per-node algebra of Section 3.1: one workgroup per node — full
//     Householder QR of Omega_tau^*, Y_tau Q, column-pivoted QR of Y_tau Gamma_tau
//     (truncated at the tolerance), U_tau, Y_tau Omega_tau^+, the residual block;
//   * the postprocessing of Section 3.3: one workgroup per child node.
// Householder convention and pivot rule (shared reading with the oracle):
//   beta = -(x0/|x0|) ||x||, v = (x - beta e0)/(x0 - beta), tau = 1 + |x0|/||x||;
//   QRCP takes the remaining column of largest norm (recomputed every step),
//   lowest index on ties.
#include "hss.h"

#include <cmath>

namespace fio {

constexpr int kMaxM = 2048;     // largest effective leaf size handled by the node kernel
constexpr int kMaxNW = 2304;    // largest number of sample columns beyond m

// Node kernels run one workgroup per node; nodes of the upper levels of 2D trees are
// large (hundreds to thousands of rows), so their workgroups get 16 waves instead of 4.
inline unsigned node_threads(int m) { return m >= 192 ? 1024u : 256u; }

// ---------------------------------------------------------------------------
// workgroup helpers (blockDim.x == 256, four waves)
__device__ __forceinline__ double wg_sum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    return t;
}

// Householder vector of x[0..n) (stride 1) in place: x[0] <- beta, x[1..] <- v[1..].
// Returns tau; every thread gets the same value.
__device__ double wg_house(double2 *x, int n, double *sh, double *beta_abs) {
    const double2 a0 = x[0];
    double part = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) part += x[i].x * x[i].x + x[i].y * x[i].y;
    const double sigma = sqrt(wg_sum(part, sh));
    if (sigma == 0.0) {
        if (beta_abs) *beta_abs = 0.0;
        __syncthreads();
        if (threadIdx.x == 0) x[0] = zc(0.0, 0.0);
        __syncthreads();
        return 0.0;
    }
    const double aa = sqrt(a0.x * a0.x + a0.y * a0.y);
    double2 ph = aa > 0.0 ? zc(a0.x / aa, a0.y / aa) : zc(1.0, 0.0);
    double2 beta = zc(-ph.x * sigma, -ph.y * sigma);
    double2 den = csub(a0, beta);                         // = ph (|a0| + sigma)
    double dn = den.x * den.x + den.y * den.y;
    double2 inv = zc(den.x / dn, -den.y / dn);
    for (int i = 1 + threadIdx.x; i < n; i += blockDim.x) x[i] = cmul(x[i], inv);
    __syncthreads();
    if (threadIdx.x == 0) x[0] = beta;
    if (beta_abs) *beta_abs = sigma;
    __syncthreads();
    return 1.0 + aa / sigma;
}

// A[0..n, 0..nc) -= tau v (v^* A), v = [1; vt[0..n-1)] (vt = v[1..]); A column-major (lda).
__device__ void wg_house_left(const double2 *vt, int n, double tau, double2 *A, int lda, int nc) {
    if (tau == 0.0) return;
    const int sub = threadIdx.x & 3;
    for (int c0 = 0; c0 < nc; c0 += (int)(blockDim.x >> 2)) {
        const int c = c0 + (threadIdx.x >> 2);
        double2 w = zc(0.0, 0.0);
        double2 *col = A + (size_t)(c < nc ? c : 0) * lda;
        if (c < nc) {
            for (int i = sub; i < n; i += 4) {
                double2 vi = i == 0 ? zc(1.0, 0.0) : vt[i - 1];
                cfmac(w, vi, col[i]);
            }
        }
        w.x += __shfl_xor(w.x, 1);
        w.y += __shfl_xor(w.y, 1);
        w.x += __shfl_xor(w.x, 2);
        w.y += __shfl_xor(w.y, 2);
        if (c < nc) {
            double2 tw = zc(tau * w.x, tau * w.y);
            for (int i = sub; i < n; i += 4) {
                double2 vi = i == 0 ? zc(1.0, 0.0) : vt[i - 1];
                col[i] = csub(col[i], cmul(vi, tw));
            }
        }
    }
    __syncthreads();
}

// Z[0..mr, 0..n) <- Z (I - tau v v^*), v = [1; vt]; Z column-major (ldz).
__device__ void wg_house_right(const double2 *vt, int n, double tau, double2 *Z, int ldz, int mr) {
    if (tau == 0.0) return;
    const int sub = threadIdx.x & 3;
    for (int r0 = 0; r0 < mr; r0 += (int)(blockDim.x >> 2)) {
        const int r = r0 + (threadIdx.x >> 2);
        double2 w = zc(0.0, 0.0);
        if (r < mr) {
            for (int l = sub; l < n; l += 4) {
                double2 vl = l == 0 ? zc(1.0, 0.0) : vt[l - 1];
                cfma(w, Z[r + (size_t)l * ldz], vl);
            }
        }
        w.x += __shfl_xor(w.x, 1);
        w.y += __shfl_xor(w.y, 1);
        w.x += __shfl_xor(w.x, 2);
        w.y += __shfl_xor(w.y, 2);
        if (r < mr) {
            double2 tw = zc(tau * w.x, tau * w.y);
            for (int l = sub; l < n; l += 4) {
                double2 vl = l == 0 ? zc(1.0, 0.0) : vt[l - 1];
                double2 &z = Z[r + (size_t)l * ldz];
                // z -= tw conj(vl)
                z.x -= tw.x * vl.x + tw.y * vl.y;
                z.y -= tw.y * vl.x - tw.x * vl.y;
            }
        }
    }
    __syncthreads();
}

struct NodeArgs {
    const double2 *Om;     // test matrix, rows of the level x s, ld = ldR
    const double2 *Y;      // sample matrix, same layout
    long ldR;
    const long *moff;      // first row of each node
    const int *msz;        // effective leaf size of each node
    int s;                 // samples
    double tol_abs;
    int cap;               // rank cap
    double2 *scratch;
    size_t stride;         // scratch entries per node
    int *rank_out;
    double2 *Uslot;        // U_tau slot (m x m) of every node
    const size_t *uoff;
    double2 *Dres;         // residual block slot (m x m) of every node
    const size_t *doff;
    int root;              // 1: only H0 = Y Omega^+ (made Hermitian) into Dres
};

// Section 3.1 for one node (blockIdx.x), or the root solve of Section 3.2, in two phases
// around the dense products of D-breve, which run as batched GEMMs over the level:
//   k_node_basis: null space of Omega_tau (QR of Omega_tau^*), W = Y_tau Gamma (QRCP, rank,
//            U_tau), T = Y_tau Omega_tau^+ = Z1 R^{-*}; at the root H0 = (T + T^*)/2 and done;
//   (batched GEMMs: X = T - U U^* T, then D-breve = X + U (X U)^*, in place in T)
//   k_node_finish: out = (D-breve + D-breve^*)/2 and U_tau to its slot.
// Scratch of a node (leading dimensions m): A (s x m), Z (m x s, T = its first m columns),
// U (m x m slot), P (m x m slot), X (m x m slot).
__global__ void __launch_bounds__(1024) k_node_basis(NodeArgs a) {
    __shared__ double sh[16];
    __shared__ double s_tau[kMaxM];
    __shared__ double s_tauw[kMaxM];
    __shared__ double s_nrm[kMaxNW];
    __shared__ int s_piv;
    __shared__ double s_max;
    const int node = blockIdx.x;
    const int m = a.msz[node], s = a.s;
    const int tid = threadIdx.x, nt = blockDim.x;
    double2 *out = a.Dres + a.doff[node];
    if (m == 0) {
        if (tid == 0 && !a.root) a.rank_out[node] = 0;
        return;
    }
    double2 *A = a.scratch + a.stride * node;       // s x m : Omega_tau^*, then reflectors / R
    double2 *Z = A + (size_t)s * m;                  // m x s : Y_tau Q
    double2 *U = Z + (size_t)m * s;                  // m x m slot (first r columns used)
    const double2 *Om = a.Om + a.moff[node];
    const double2 *Yt = a.Y + a.moff[node];
    for (int e = tid; e < s * m; e += nt) {
        int i = e % s, j = e / s;                    // A(i, j) = conj(Om(j, i))
        double2 v = Om[j + (size_t)i * a.ldR];
        A[e] = zc(v.x, -v.y);
    }
    for (int e = tid; e < m * s; e += nt) {
        int i = e % m, j = e / m;
        Z[e] = Yt[i + (size_t)j * a.ldR];
    }
    __syncthreads();
    // full Householder QR of Omega_tau^* (s x m)
    for (int j = 0; j < m; ++j) {
        double2 *col = A + j + (size_t)j * s;
        double tau = wg_house(col, s - j, sh, nullptr);
        if (tid == 0) s_tau[j] = tau;
        wg_house_left(col + 1, s - j, tau, col + s, s, m - j - 1);
    }
    __syncthreads();
    // Z = Y_tau Q, Q = H_0 ... H_{m-1}
    for (int j = 0; j < m; ++j) {
        wg_house_right(A + j + 1 + (size_t)j * s, s - j, s_tau[j], Z + (size_t)j * m, m, m);
    }
    int r = 0;
    if (!a.root) {
        // QRCP of W = Z[:, m:s]  (m x nw)
        double2 *W = Z + (size_t)m * m;
        const int nw = s - m;
        int kmax = m < nw ? m : nw;
        if (a.cap > 0 && a.cap < kmax) kmax = a.cap;
        for (int j = 0; j < kmax; ++j) {
            const int sub = tid & 3;
            for (int c0 = j; c0 < nw; c0 += nt >> 2) {
                int c = c0 + (tid >> 2);
                double p = 0.0;
                if (c < nw)
                    for (int i = j + sub; i < m; i += 4) {
                        double2 v = W[i + (size_t)c * m];
                        p += v.x * v.x + v.y * v.y;
                    }
                p += __shfl_xor(p, 1);
                p += __shfl_xor(p, 2);
                if (c < nw && sub == 0) s_nrm[c] = sqrt(p);
            }
            __syncthreads();
            if (tid == 0) {
                int best = j;
                double bv = s_nrm[j];
                for (int c = j + 1; c < nw; ++c)
                    if (s_nrm[c] > bv) {
                        bv = s_nrm[c];
                        best = c;
                    }
                s_piv = best;
                s_max = bv;
            }
            __syncthreads();
            if (!(s_max > a.tol_abs)) break;
            const int pc = s_piv;
            if (pc != j) {
                for (int i = tid; i < m; i += nt) {
                    double2 t = W[i + (size_t)j * m];
                    W[i + (size_t)j * m] = W[i + (size_t)pc * m];
                    W[i + (size_t)pc * m] = t;
                }
                __syncthreads();
            }
            double2 *col = W + j + (size_t)j * m;
            double tau = wg_house(col, m - j, sh, nullptr);
            if (tid == 0) s_tauw[j] = tau;
            wg_house_left(col + 1, m - j, tau, col + m, m, nw - j - 1);
            r = j + 1;
        }
        __syncthreads();
        // U = H_0 ... H_{r-1} [I_r; 0]
        for (int e = tid; e < m * r; e += nt) {
            int i = e % m, j = e / m;
            U[e] = zc(i == j ? 1.0 : 0.0, 0.0);
        }
        __syncthreads();
        for (int j = r - 1; j >= 0; --j)
            wg_house_left(W + j + 1 + (size_t)j * m, m - j, s_tauw[j], U + j, m, r);
        if (tid == 0) a.rank_out[node] = r;
    }
    // T = Z1 R^{-*} (R = upper m x m of A): solve T R^* = Z1 row by row, in place in Z[:, 0:m]
    for (int i = tid; i < m; i += nt) {
        for (int j = m - 1; j >= 0; --j) {
            double2 acc = Z[i + (size_t)j * m];
            for (int k = j + 1; k < m; ++k) {
                double2 rjk = A[j + (size_t)k * s];
                double2 t = Z[i + (size_t)k * m];
                // acc -= t conj(rjk)
                acc.x -= t.x * rjk.x + t.y * rjk.y;
                acc.y -= t.y * rjk.x - t.x * rjk.y;
            }
            double2 rjj = A[j + (size_t)j * s];
            double d = rjj.x * rjj.x + rjj.y * rjj.y;
            // acc / conj(rjj) = acc rjj / |rjj|^2
            Z[i + (size_t)j * m] = zc((acc.x * rjj.x - acc.y * rjj.y) / d, (acc.x * rjj.y + acc.y * rjj.x) / d);
        }
    }
    __syncthreads();
    const double2 *T = Z;
    if (a.root) {
        for (int e = tid; e < m * m; e += nt) {
            int i = e % m, j = e / m;
            double2 x = T[i + (size_t)j * m], y = T[j + (size_t)i * m];
            out[e] = zc(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
        }
    }
}

__global__ void __launch_bounds__(1024) k_node_finish(NodeArgs a) {
    const int node = blockIdx.x;
    const int m = a.msz[node], s = a.s;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (m == 0) return;
    const int r = a.rank_out[node];
    double2 *out = a.Dres + a.doff[node];
    const double2 *Z = a.scratch + a.stride * node + (size_t)s * m;   // D-breve in Z[:, 0:m]
    const double2 *U = Z + (size_t)m * s;
    for (int e = tid; e < m * m; e += nt) {
        int i = e % m, j = e / m;
        double2 x = Z[i + (size_t)j * m], y = Z[j + (size_t)i * m];
        out[e] = zc(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
    }
    double2 *Uo = a.Uslot + a.uoff[node];
    for (int e = tid; e < m * r; e += nt) Uo[e] = U[e];
}

// ---------------------------------------------------------------------------
// Large nodes (the upper levels of 2D trees, hundreds to thousands of rows, few nodes per
// level): the same Section 3.1 steps as k_node_basis, one reflector or pivot step per
// launch, each launch spread over many workgroups (grid.y = node, grid.x = column or row
// chunk).  The reflector and pivot arithmetic is k_node_basis's; only the work split differs.
struct BigArgs {
    NodeArgs n;
    double *tauA, *tauW;   // reflector scalars per node (kMaxM each)
    double *nrm;           // column norms per node (ldn each)
    int ldn;
    int *done;             // 1 once the node's QRCP has stopped
};

// columns (or rows) per workgroup of the apply kernels, four lanes each: small workgroups, so
// that the few large nodes of a level still spread over most of the GPU
constexpr int kBigChunk = 16, kBigThreads = 4 * kBigChunk;

__global__ void k_big_init(BigArgs b) {
    const NodeArgs &a = b.n;
    const int node = blockIdx.y, m = a.msz[node], s = a.s;
    if (m == 0) return;
    double2 *A = a.scratch + a.stride * node, *Z = A + (size_t)s * m;
    const double2 *Om = a.Om + a.moff[node], *Yt = a.Y + a.moff[node];
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)s * m; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e % s), j = (int)(e / s);
        const double2 v = Om[j + (size_t)i * a.ldR];
        A[e] = zc(v.x, -v.y);
        const int zi = (int)(e % m), zj = (int)(e / m);
        Z[e] = Yt[zi + (size_t)zj * a.ldR];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (!a.root) a.rank_out[node] = 0;
        b.done[node] = 0;
    }
}

// Householder vector of column j of A (rows j..s-1)
__global__ void __launch_bounds__(1024) k_big_house_A(BigArgs b, int j) {
    __shared__ double sh[16];
    const NodeArgs &a = b.n;
    const int node = blockIdx.y, m = a.msz[node], s = a.s;
    if (j >= m) return;
    double2 *A = a.scratch + a.stride * node;
    const double tau = wg_house(A + j + (size_t)j * s, s - j, sh, nullptr);
    if (threadIdx.x == 0) b.tauA[(size_t)node * kMaxM + j] = tau;
}

// H_j applied to columns j+1.. of A
__global__ void __launch_bounds__(256) k_big_left_A(BigArgs b, int j) {
    const NodeArgs &a = b.n;
    const int node = blockIdx.y, m = a.msz[node], s = a.s;
    const int c0 = j + 1 + blockIdx.x * kBigChunk;
    if (j >= m || c0 >= m) return;
    double2 *A = a.scratch + a.stride * node;
    const int nc = m - c0 < kBigChunk ? m - c0 : kBigChunk;
    wg_house_left(A + j + 1 + (size_t)j * s, s - j, b.tauA[(size_t)node * kMaxM + j], A + j + (size_t)c0 * s, s, nc);
}

// Z <- Z H_j on a chunk of Z's rows
__global__ void __launch_bounds__(256) k_big_right_Z(BigArgs b, int j) {
    const NodeArgs &a = b.n;
    const int node = blockIdx.y, m = a.msz[node], s = a.s;
    const int r0 = blockIdx.x * kBigChunk;
    if (j >= m || r0 >= m) return;
    double2 *A = a.scratch + a.stride * node, *Z = A + (size_t)s * m;
    const int nr = m - r0 < kBigChunk ? m - r0 : kBigChunk;
    wg_house_right(A + j + 1 + (size_t)j * s, s - j, b.tauA[(size_t)node * kMaxM + j], Z + r0 + (size_t)j * m, m, nr);
}

__device__ __forceinline__ int big_kmax(const NodeArgs &a, int m) {
    const int nw = a.s - m;
    int kmax = m < nw ? m : nw;
    if (a.cap > 0 && a.cap < kmax) kmax = a.cap;
    return kmax;
}

// QRCP step j: norms of the remaining columns of W (rows j..m-1), 4 lanes per column
__global__ void __launch_bounds__(256) k_big_norms(BigArgs b, int j) {
    const NodeArgs &a = b.n;
    const int node = blockIdx.y, m = a.msz[node], s = a.s;
    if (m == 0 || b.done[node] || j >= big_kmax(a, m)) return;
    const int nw = s - m;
    const double2 *W = a.scratch + a.stride * node + (size_t)s * m + (size_t)m * m;
    const int sub = threadIdx.x & 3;
    const int c = j + blockIdx.x * kBigChunk + (threadIdx.x >> 2);
    double p = 0.0;
    if (c < nw)
        for (int i = j + sub; i < m; i += 4) {
            const double2 v = W[i + (size_t)c * m];
            p += v.x * v.x + v.y * v.y;
        }
    p += __shfl_xor(p, 1);
    p += __shfl_xor(p, 2);
    if (c < nw && sub == 0) b.nrm[(size_t)node * b.ldn + c] = sqrt(p);
}

// QRCP step j: pivot (largest norm, lowest index on ties), stop test, swap, reflector
__global__ void __launch_bounds__(1024) k_big_pivot(BigArgs b, int j) {
    __shared__ double sh[16];
    __shared__ int s_piv;
    __shared__ double s_max;
    const NodeArgs &a = b.n;
    const int node = blockIdx.y, m = a.msz[node], s = a.s;
    if (m == 0 || b.done[node]) return;
    if (j >= big_kmax(a, m)) {
        if (threadIdx.x == 0) b.done[node] = 1;
        return;
    }
    const int nw = s - m;
    double2 *W = a.scratch + a.stride * node + (size_t)s * m + (size_t)m * m;
    const double *nrm = b.nrm + (size_t)node * b.ldn;
    if (threadIdx.x == 0) {
        int best = j;
        double bv = nrm[j];
        for (int c = j + 1; c < nw; ++c)
            if (nrm[c] > bv) {
                bv = nrm[c];
                best = c;
            }
        s_piv = best;
        s_max = bv;
    }
    __syncthreads();
    if (!(s_max > a.tol_abs)) {
        if (threadIdx.x == 0) b.done[node] = 1;
        return;
    }
    const int pc = s_piv;
    if (pc != j) {
        for (int i = threadIdx.x; i < m; i += blockDim.x) {
            const double2 t = W[i + (size_t)j * m];
            W[i + (size_t)j * m] = W[i + (size_t)pc * m];
            W[i + (size_t)pc * m] = t;
        }
        __syncthreads();
    }
    const double tau = wg_house(W + j + (size_t)j * m, m - j, sh, nullptr);
    if (threadIdx.x == 0) {
        b.tauW[(size_t)node * kMaxM + j] = tau;
        a.rank_out[node] = j + 1;
    }
}

// QRCP step j: H_j applied to columns j+1.. of W
__global__ void __launch_bounds__(256) k_big_left_W(BigArgs b, int j) {
    const NodeArgs &a = b.n;
    const int node = blockIdx.y, m = a.msz[node], s = a.s;
    if (m == 0 || b.done[node]) return;
    const int nw = s - m;
    const int c0 = j + 1 + blockIdx.x * kBigChunk;
    if (c0 >= nw) return;
    double2 *W = a.scratch + a.stride * node + (size_t)s * m + (size_t)m * m;
    const int nc = nw - c0 < kBigChunk ? nw - c0 : kBigChunk;
    wg_house_left(W + j + 1 + (size_t)j * m, m - j, b.tauW[(size_t)node * kMaxM + j], W + j + (size_t)c0 * m, m, nc);
}

// U = [I_r; 0]
__global__ void k_big_uinit(BigArgs b) {
    const NodeArgs &a = b.n;
    const int node = blockIdx.y, m = a.msz[node], s = a.s;
    if (m == 0) return;
    const int r = a.rank_out[node];
    double2 *U = a.scratch + a.stride * node + (size_t)s * m + (size_t)m * s;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)m * r; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e % m), jj = (int)(e / m);
        U[e] = zc(i == jj ? 1.0 : 0.0, 0.0);
    }
}

// U <- H_j U (rows j..m-1) on a chunk of U's r columns
__global__ void __launch_bounds__(256) k_big_left_U(BigArgs b, int j) {
    const NodeArgs &a = b.n;
    const int node = blockIdx.y, m = a.msz[node], s = a.s;
    if (m == 0) return;
    const int r = a.rank_out[node];
    const int c0 = blockIdx.x * kBigChunk;
    if (j >= r || c0 >= r) return;
    double2 *Z = a.scratch + a.stride * node + (size_t)s * m;
    double2 *W = Z + (size_t)m * m, *U = Z + (size_t)m * s;
    const int nc = r - c0 < kBigChunk ? r - c0 : kBigChunk;
    wg_house_left(W + j + 1 + (size_t)j * m, m - j, b.tauW[(size_t)node * kMaxM + j], U + j + (size_t)c0 * m, m, nc);
}

// T = Z1 R^{-*} (R = upper m x m of A), one lane per row; at the root also H0 = (T + T^*)/2
__global__ void __launch_bounds__(256) k_big_tsolve(BigArgs b) {
    const NodeArgs &a = b.n;
    const int node = blockIdx.y, m = a.msz[node], s = a.s;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (m == 0 || i >= m) return;
    const double2 *A = a.scratch + a.stride * node;
    double2 *Z = const_cast<double2 *>(A) + (size_t)s * m;
    for (int j = m - 1; j >= 0; --j) {
        double2 acc = Z[i + (size_t)j * m];
        for (int k = j + 1; k < m; ++k) {
            const double2 rjk = A[j + (size_t)k * s];
            const double2 t = Z[i + (size_t)k * m];
            acc.x -= t.x * rjk.x + t.y * rjk.y;
            acc.y -= t.y * rjk.x - t.x * rjk.y;
        }
        const double2 rjj = A[j + (size_t)j * s];
        const double d = rjj.x * rjj.x + rjj.y * rjj.y;
        Z[i + (size_t)j * m] = zc((acc.x * rjj.x - acc.y * rjj.y) / d, (acc.x * rjj.y + acc.y * rjj.x) / d);
    }
}

__global__ void k_big_root_out(BigArgs b) {
    const NodeArgs &a = b.n;
    const int node = blockIdx.y, m = a.msz[node], s = a.s;
    const double2 *Z = a.scratch + a.stride * node + (size_t)s * m;
    double2 *out = a.Dres + a.doff[node];
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)m * m; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e % m), j = (int)(e / m);
        const double2 x = Z[i + (size_t)j * m], y = Z[j + (size_t)i * m];
        out[e] = zc(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
    }
}

// P(a, c) = conj(Y(c, a)) for a < r, c < m, Y = X U in the X slot, P in the P slot of each node
__global__ void k_node_conj_transpose(NodeArgs a) {
    const int node = blockIdx.y;
    const int m = a.msz[node], s = a.s;
    if (m == 0) return;
    const int r = a.rank_out[node];
    const double2 *Z = a.scratch + a.stride * node + (size_t)s * m;
    double2 *P = const_cast<double2 *>(Z) + (size_t)m * s + (size_t)m * m;
    const double2 *Y = P + (size_t)m * m;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)r * m; e += (long)gridDim.x * blockDim.x) {
        const int aa = (int)(e % r), c = (int)(e / r);
        const double2 y = Y[c + (size_t)aa * m];
        P[aa + (size_t)c * m] = zc(y.x, -y.y);
    }
}

struct PostArgs {
    const double2 *Dpar;   // parent diagonal blocks (m_par x m_par slots)
    const size_t *dpoff;
    const int *mpar;       // parent sizes
    const int *rch;        // child ranks (level l+1)
    const double2 *Dres;   // child residual slots
    const size_t *droff;
    const int *mch;        // child sizes
    const double2 *Uslot;  // child U slots
    const size_t *uoff;
    double2 *Dout;         // child D slots
    const size_t *dooff;
    double2 *Bout;         // B of the parents
    const size_t *boff;
    double2 *tmp;          // scratch per child: T (m_ch x r_ch), then U_c^* (r_ch x m_ch)
    size_t tstride;
};

// Section 3.3 for the two children of every node of level l (one workgroup per child c),
// around two batched GEMMs over the level:
//   k_post_prep: B_{a2,a1} = A_21 of the parent's block (written by the first child),
//                D_c <- D_res_c, and the conjugate transpose U_c^* next to T in the scratch;
//   GEMMs: T = U_c A (A = the child's diagonal block of D^[l]_parent), D_c += T U_c^*.
__global__ void __launch_bounds__(1024) k_post_prep(PostArgs a) {
    const int c = blockIdx.x, par = c >> 1, tid = threadIdx.x, nt = blockDim.x;
    const int mp = a.mpar[par], mc = a.mch[c], r = a.rch[c];
    const int r1 = a.rch[par * 2];
    const double2 *Dp = a.Dpar + a.dpoff[par];
    if ((c & 1) == 0) {
        const int r2 = a.rch[par * 2 + 1];
        double2 *Bo = a.Bout + a.boff[par];
        for (int e = tid; e < r2 * r1; e += nt) {
            int i = e % r2, j = e / r2;
            Bo[e] = Dp[(r1 + i) + (size_t)j * mp];
        }
    }
    const double2 *Uc = a.Uslot + a.uoff[c];
    double2 *UcH = a.tmp + a.tstride * c + (size_t)mc * r;
    for (int e = tid; e < r * mc; e += nt) {
        int i = e % r, j = e / r;
        const double2 u = Uc[j + (size_t)i * mc];
        UcH[i + (size_t)j * r] = zc(u.x, -u.y);
    }
    const double2 *Dr = a.Dres + a.droff[c];
    double2 *Do = a.Dout + a.dooff[c];
    for (int e = tid; e < mc * mc; e += nt) Do[e] = Dr[e];
}

__global__ void k_sumsq_partial(const double2 *x, size_t n, double *part) {
    __shared__ double sh[8];
    double p = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p += x[i].x * x[i].x + x[i].y * x[i].y;
    double t = wg_sum(p, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// deterministic sum of squares of n complex entries
static double sumsq(const double2 *x, size_t n, hipStream_t s) {
    const int nb = 512;
    DevBuf part(nb * sizeof(double));
    k_sumsq_partial<<<nb, 256, 0, s>>>(x, n, part.as<double>());
    FIO_HIP(hipGetLastError());
    std::vector<double> hp(nb);
    FIO_HIP(hipMemcpyAsync(hp.data(), part.p, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    FIO_HIP(hipStreamSynchronize(s));
    double t = 0.0;
    for (double v : hp) t += v;
    return t;
}

template <typename T> static DevBuf *upload(const std::vector<T> &v, hipStream_t s) {
    DevBuf *b = new DevBuf(v.size() * sizeof(T) + 8);
    FIO_HIP(hipMemcpyAsync(b->p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return b;
}

// Section 3.1 on a level of large nodes, one reflector or pivot step per launch (see BigArgs).
static int g_big_node = 256;       // levels whose largest node has at least this many rows take this path

static unsigned cdiv(long a, long b) { return (unsigned)(a <= 0 ? 0 : (a + b - 1) / b); }

static void basis_big(const NodeArgs &na, const std::vector<int> &ms, int nn, int mmax, int sl, bool root,
                      hipStream_t s) {
    DevBuf tauA((size_t)nn * kMaxM * sizeof(double)), tauW((size_t)nn * kMaxM * sizeof(double)),
        nrm((size_t)nn * sl * sizeof(double)), done((size_t)nn * sizeof(int));
    BigArgs b;
    b.n = na;
    b.tauA = tauA.as<double>();
    b.tauW = tauW.as<double>();
    b.nrm = nrm.as<double>();
    b.ldn = sl;
    b.done = done.as<int>();
    const unsigned y = (unsigned)nn;
    k_big_init<<<dim3(256, y), 256, 0, s>>>(b);
    // full Householder QR of Omega_tau^* (s x m), then Z = Y_tau H_0 ... H_{m-1}
    for (int j = 0; j < mmax; ++j) {
        k_big_house_A<<<dim3(1, y), 1024, 0, s>>>(b, j);
        if (mmax - 1 - j > 0) k_big_left_A<<<dim3(cdiv(mmax - 1 - j, kBigChunk), y), kBigThreads, 0, s>>>(b, j);
    }
    for (int j = 0; j < mmax; ++j) k_big_right_Z<<<dim3(cdiv(mmax, kBigChunk), y), kBigThreads, 0, s>>>(b, j);
    FIO_HIP(hipGetLastError());
    if (!root) {
        // QRCP of W = Z[:, m:s]; every 32 steps the host stops once every node has stopped
        int mmin = mmax, kcap = 0;
        for (int v : ms)
            if (v > 0) mmin = v < mmin ? v : mmin;
        for (int v : ms) {
            if (v == 0) continue;
            int k = v < sl - v ? v : sl - v;
            if (na.cap > 0 && na.cap < k) k = na.cap;
            kcap = k > kcap ? k : kcap;
        }
        const int nwmax = sl - mmin;
        std::vector<int> hd(nn);
        for (int j = 0; j < kcap; ++j) {
            k_big_norms<<<dim3(cdiv(nwmax - j, kBigChunk), y), kBigThreads, 0, s>>>(b, j);
            k_big_pivot<<<dim3(1, y), 1024, 0, s>>>(b, j);
            if (nwmax - j - 1 > 0) k_big_left_W<<<dim3(cdiv(nwmax - j - 1, kBigChunk), y), kBigThreads, 0, s>>>(b, j);
            if ((j & 31) == 31) {
                FIO_HIP(hipMemcpyAsync(hd.data(), done.p, nn * sizeof(int), hipMemcpyDeviceToHost, s));
                FIO_HIP(hipStreamSynchronize(s));
                bool all = true;
                for (int k = 0; k < nn; ++k) all = all && (hd[k] || ms[k] == 0);
                if (all) break;
            }
        }
        std::vector<int> rk(nn);
        FIO_HIP(hipMemcpyAsync(rk.data(), na.rank_out, nn * sizeof(int), hipMemcpyDeviceToHost, s));
        FIO_HIP(hipStreamSynchronize(s));
        int rmax = 0;
        for (int v : rk) rmax = v > rmax ? v : rmax;
        // U = H_0 ... H_{r-1} [I_r; 0]
        k_big_uinit<<<dim3(64, y), 256, 0, s>>>(b);
        for (int j = rmax - 1; j >= 0; --j) k_big_left_U<<<dim3(cdiv(rmax, kBigChunk), y), kBigThreads, 0, s>>>(b, j);
    }
    k_big_tsolve<<<dim3(cdiv(mmax, 256), y), 256, 0, s>>>(b);
    if (root) k_big_root_out<<<dim3(64, y), 256, 0, s>>>(b);
    FIO_HIP(hipGetLastError());
    FIO_HIP(hipStreamSynchronize(s));    // the work arrays are released here
}

void hss_layout_level(hss_s *h, int l) {
    const int nn = h->nodes(l);
    h->m[l].assign(nn, 0);
    h->uoff[l].assign(nn, 0);
    size_t off = 0;
    for (int j = 0; j < nn; ++j) {
        h->m[l][j] = (l == h->Lh) ? h->leaf : h->rank[l + 1][2 * j] + h->rank[l + 1][2 * j + 1];
        h->uoff[l][j] = off;
        off += (size_t)h->m[l][j] * h->m[l][j];
    }
    if (h->Ubuf[l]) delete h->Ubuf[l];
    h->Ubuf[l] = new DevBuf(off * sizeof(double2) + 16);
}

void hss_layout_B(hss_s *h) {
    size_t off = 0;
    h->boff.assign(h->Lh, {});
    for (int l = 0; l < h->Lh; ++l) {
        h->boff[l].assign(h->nodes(l), 0);
        for (int j = 0; j < h->nodes(l); ++j) {
            h->boff[l][j] = off;
            off += (size_t)h->rank[l + 1][2 * j] * h->rank[l + 1][2 * j + 1];
        }
    }
    h->Bbuf.alloc(off * sizeof(double2) + 16);
    h->Dbuf.alloc((size_t)h->nodes(h->Lh) * h->leaf * h->leaf * sizeof(double2));
}

// X_out (rows sum m_lv) = diag(U_(lv,j)) X_in (rows sum r_lv), or the projection with U^*.
static void lift_level(hss_s *h, int lv, const double2 *in, long ldin, double2 *out, long ldout, int ncols,
                       bool project, hipStream_t s) {
    ZgemmBatch zb;
    long ro = 0, mo = 0;
    for (int j = 0; j < h->nodes(lv); ++j) {
        int m = h->m[lv][j], r = h->rank[lv][j];
        if (!project)
            zb.add(h->U(lv, j), m, in + ro, ldin, out + mo, ldout, m, ncols, r);
        else
            zb.add(h->U(lv, j), m, in + mo, ldin, out + ro, ldout, r, ncols, m);
        ro += r;
        mo += m;
    }
    zb.upload(s);
    zb.run(project, zc(1.0), zc(0.0), s);
    FIO_HIP(hipStreamSynchronize(s));   // the descriptor list is freed on return
}

static long level_rows_m(const hss_s *h, int lv) {
    long t = 0;
    for (int v : h->m[lv]) t += v;
    return t;
}
static long level_rows_r(const hss_s *h, int lv) {
    long t = 0;
    for (int v : h->rank[lv]) t += v;
    return t;
}

// Omega_big = U^[Lh] ... U^[l+1] Omega (N x ncols); Y = U^[l+1]* ... U^[Lh]* Y_big.
static void lift_all(hss_s *h, int l, const double2 *Om, long R, double2 *t0, double2 *t1, double2 *out, int ncols,
                     hipStream_t s) {
    if (l == h->Lh) {
        FIO_HIP(hipMemcpyAsync(out, Om, (size_t)R * ncols * sizeof(double2), hipMemcpyDeviceToDevice, s));
        return;
    }
    const double2 *cur = Om;
    long ldc = R;
    for (int lv = l + 1; lv <= h->Lh; ++lv) {
        long rows = level_rows_m(h, lv);
        double2 *dst = (lv == h->Lh) ? out : ((lv - l) % 2 ? t0 : t1);
        lift_level(h, lv, cur, ldc, dst, rows, ncols, false, s);
        cur = dst;
        ldc = rows;
    }
}

static void project_all(hss_s *h, int l, const double2 *Yb, double2 *t0, double2 *t1, double2 *out, long R,
                        int ncols, hipStream_t s) {
    if (l == h->Lh) {
        FIO_HIP(hipMemcpyAsync(out, Yb, (size_t)R * ncols * sizeof(double2), hipMemcpyDeviceToDevice, s));
        return;
    }
    const double2 *cur = Yb;
    long ldc = h->N;
    for (int lv = h->Lh; lv >= l + 1; --lv) {
        long rows = level_rows_r(h, lv);
        double2 *dst = (lv == l + 1) ? out : ((h->Lh - lv) % 2 ? t1 : t0);
        lift_level(h, lv, cur, ldc, dst, rows, ncols, true, s);
        cur = dst;
        ldc = rows;
    }
}

struct Sampler {
    hss_matvec_fn matvec;
    void *mctx;
    hss_omega_fn omega;
    void *octx;
};

static fio_status build_impl(long n, const hss_opts *o, const Sampler &sm, hipStream_t s, hss_t *out) {
    FIO_CHECK_ARG(o && out && sm.matvec && sm.omega);
    FIO_CHECK_ARG(o->leaf >= 1 && o->p >= 0 && o->tol >= 0.0);
    int Lh = 0;
    while (((long)o->leaf << Lh) < n) ++Lh;
    FIO_CHECK_ARG(((long)o->leaf << Lh) == n && Lh >= 1);
    FIO_CHECK_ARG(o->leaf <= kMaxM);
    hss_s *h = new hss_s();
    h->N = n;
    h->leaf = o->leaf;
    h->Lh = Lh;
    h->rank.assign(Lh + 1, {});
    h->m.assign(Lh + 1, {});
    h->uoff.assign(Lh + 1, {});
    h->Ubuf.assign(Lh + 1, nullptr);
    h->samples.assign(Lh + 1, 0);
    h->drawn.assign(Lh + 1, 0);
    std::vector<DevBuf *> Dres(Lh + 1, nullptr);
    std::vector<std::vector<size_t>> doff(Lh + 1);
    fio_status st = guarded([&] {
        double g = o->norm_est;
        DevBuf Om, Ob, Yb, Y, t0, t1, scratch;
        for (int l = Lh; l >= 0; --l) {
            const bool root = (l == 0);
            if (!root) hss_layout_level(h, l);
            const int nn = root ? 1 : h->nodes(l);
            std::vector<int> ms(nn);
            std::vector<long> mo(nn);
            long R = 0;
            int mmax = 0;
            for (int j = 0; j < nn; ++j) {
                ms[j] = root ? h->rank[1][0] + h->rank[1][1] : h->m[l][j];
                mo[j] = R;
                R += ms[j];
                mmax = ms[j] > mmax ? ms[j] : mmax;
            }
            if (root) h->m[0] = {ms[0]};
            doff[l].assign(nn, 0);
            size_t dtot = 0;
            for (int j = 0; j < nn; ++j) {
                doff[l][j] = dtot;
                dtot += (size_t)ms[j] * ms[j];
            }
            Dres[l] = new DevBuf(dtot * sizeof(double2) + 16);
            if (mmax == 0) {
                h->rank[l].assign(nn, 0);
                continue;
            }
            if (mmax > kMaxM) throw Err{FIO_ERR_UNSUPPORTED};
            // Section 3.1: s_l = m_l + r_l + p.  The level's rank is not known before it is built:
            // the guess is rhat (or m_max); adaptive, a nonleaf level guesses the largest rank of
            // the level below and is sampled again with the guess m_max (always sufficient) when a
            // node's rank exceeds the guess
            int guess = root ? 0 : (o->rhat > 0 ? o->rhat : mmax);
            if (o->adaptive && !root && l < Lh) {
                int rb = 0;
                for (int v : h->rank[l + 1]) rb = v > rb ? v : rb;
                guess = rb < mmax ? rb : mmax;
            }
            for (;;) {
                const int sl = mmax + guess + o->p;
                // the one-workgroup node kernel keeps the norms of all s - m sample columns in LDS
                int mmin = mmax;
                for (int v : ms)
                    if (v > 0) mmin = v < mmin ? v : mmin;
                if (!root && mmax < g_big_node && sl - mmin > kMaxNW) throw Err{FIO_ERR_UNSUPPORTED};
                h->samples[l] = sl;
                Om.ensure((size_t)R * sl * sizeof(double2));
                if (sm.omega(sm.octx, l, R, sl, Om.p, s) != 0) throw Err{FIO_ERR_CALLBACK};
                const size_t big = (size_t)n * sl * sizeof(double2);
                Ob.ensure(big);
                Yb.ensure(big);
                t0.ensure(big);
                t1.ensure(big);
                Y.ensure((size_t)R * sl * sizeof(double2));
                lift_all(h, l, Om.as<double2>(), R, t0.as<double2>(), t1.as<double2>(), Ob.as<double2>(), sl, s);
                if (sm.matvec(sm.mctx, Ob.p, n, Yb.p, n, sl, s) != 0) throw Err{FIO_ERR_CALLBACK};
                project_all(h, l, Yb.as<double2>(), t0.as<double2>(), t1.as<double2>(), Y.as<double2>(), R, sl, s);
                if (l == Lh && !(o->norm_est > 0.0)) {
                    double ny = sumsq(Y.as<double2>(), (size_t)R * sl, s);
                    double no = sumsq(Om.as<double2>(), (size_t)R * sl, s);
                    g = sqrt(ny) / sqrt(no);
                }
                // per-node algebra
                size_t stride = (size_t)2 * sl * mmax + (size_t)3 * mmax * mmax;
                scratch.ensure(stride * nn * sizeof(double2));
                std::vector<size_t> uo(nn, 0);
                if (!root) uo = h->uoff[l];
                DevBuf *dmo = upload(mo, s), *dms = upload(ms, s), *duo = upload(uo, s), *ddo = upload(doff[l], s);
                DevBuf rk(nn * sizeof(int));
                NodeArgs na;
                na.Om = Om.as<double2>();
                na.Y = Y.as<double2>();
                na.ldR = R;
                na.moff = dmo->as<long>();
                na.msz = dms->as<int>();
                na.s = sl;
                na.tol_abs = o->tol * g;
                na.cap = o->rank_cap;
                na.scratch = scratch.as<double2>();
                na.stride = stride;
                na.rank_out = rk.as<int>();
                na.Uslot = root ? nullptr : h->Ubuf[l]->as<double2>();
                na.uoff = duo->as<size_t>();
                na.Dres = Dres[l]->as<double2>();
                na.doff = ddo->as<size_t>();
                na.root = root ? 1 : 0;
                if (mmax < g_big_node) {
                    k_node_basis<<<nn, node_threads(mmax), 0, s>>>(na);
                    FIO_HIP(hipGetLastError());
                } else {
                    basis_big(na, ms, nn, mmax, sl, root, s);
                }
                if (!root) {
                    h->rank[l].assign(nn, 0);
                    FIO_HIP(hipMemcpyAsync(h->rank[l].data(), rk.p, nn * sizeof(int), hipMemcpyDeviceToHost, s));
                    FIO_HIP(hipStreamSynchronize(s));
                    // D-breve = X + U (X U)^*, X = T - U (U^* T), for all nodes of the level
                    ZgemmBatch g1, g2, g3, g4;
                    double2 *sc = scratch.as<double2>();
                    int rmax = 0;
                    for (int j = 0; j < nn; ++j) {
                        const int m = ms[j], r = h->rank[l][j];
                        if (m == 0) continue;
                        rmax = r > rmax ? r : rmax;
                        double2 *T = sc + stride * j + (size_t)sl * m;
                        double2 *U = T + (size_t)m * sl, *P = U + (size_t)m * m, *X = P + (size_t)m * m;
                        g1.add(U, m, T, m, P, m, r, m, m);        // P = U^* T      (r x m)
                        g2.add(U, m, P, m, T, m, m, m, r);        // T -= U P       (X, m x m)
                        g3.add(T, m, U, m, X, m, m, r, m);        // X slot = X U   (m x r)
                        g4.add(U, m, P, m, T, m, m, m, r);        // T += U (X U)^* (D-breve)
                    }
                    g1.upload(s);
                    g2.upload(s);
                    g3.upload(s);
                    g4.upload(s);
                    g1.run(true, zc(1.0, 0.0), zc(0.0, 0.0), s);
                    g2.run(false, zc(-1.0, 0.0), zc(1.0, 0.0), s);
                    g3.run(false, zc(1.0, 0.0), zc(0.0, 0.0), s);
                    if (rmax > 0) {
                        dim3 gct((unsigned)((rmax * (size_t)mmax + 255) / 256), (unsigned)nn);
                        k_node_conj_transpose<<<gct, 256, 0, s>>>(na);
                    }
                    g4.run(false, zc(1.0, 0.0), zc(1.0, 0.0), s);
                    k_node_finish<<<nn, node_threads(mmax), 0, s>>>(na);
                    FIO_HIP(hipGetLastError());
                    FIO_HIP(hipStreamSynchronize(s));   // the descriptor lists are released here
                }
                FIO_HIP(hipStreamSynchronize(s));
                delete dmo;
                delete dms;
                delete duo;
                delete ddo;
                h->drawn[l] += sl;
                if (root || !o->adaptive || guess >= mmax) break;
                int rl = 0;
                for (int v : h->rank[l]) rl = v > rl ? v : rl;
                if (rl <= guess) break;
                guess = mmax;
            }
            if (!root && o->rank_cap > 0)
                for (int v : h->rank[l])
                    if (v >= o->rank_cap) h->rank_capped = true;
        }
        h->gain = g;
        // postprocessing (Section 3.3), top down
        hss_layout_B(h);
        DevBuf Dcur, Dnext, tmp;
        // level-0 "D" is H0, stored in Dres[0]
        const double2 *dpar = Dres[0]->as<double2>();
        std::vector<size_t> dpoff = {0};
        std::vector<int> mpar = {h->m[0][0]};
        for (int l = 0; l < Lh; ++l) {
            const int nc = h->nodes(l + 1);
            std::vector<size_t> dooff(nc);
            size_t tot = 0, tmax = 0;
            for (int c = 0; c < nc; ++c) {
                dooff[c] = tot;
                tot += (size_t)h->m[l + 1][c] * h->m[l + 1][c];
                size_t tt = (size_t)h->m[l + 1][c] * h->rank[l + 1][c];
                tmax = tt > tmax ? tt : tmax;
            }
            double2 *dout;
            if (l + 1 == Lh) {
                dout = h->Dbuf.as<double2>();
            } else {
                Dnext.alloc(tot * sizeof(double2) + 16);
                dout = Dnext.as<double2>();
            }
            tmp.ensure(2 * tmax * nc * sizeof(double2) + 16);
            std::vector<size_t> bo = h->boff[l];
            DevBuf *d1 = upload(dpoff, s), *d2 = upload(mpar, s), *d3 = upload(h->rank[l + 1], s),
                   *d4 = upload(doff[l + 1], s), *d5 = upload(h->m[l + 1], s), *d6 = upload(h->uoff[l + 1], s),
                   *d7 = upload(dooff, s), *d8 = upload(bo, s);
            PostArgs pa;
            pa.Dpar = dpar;
            pa.dpoff = d1->as<size_t>();
            pa.mpar = d2->as<int>();
            pa.rch = d3->as<int>();
            pa.Dres = Dres[l + 1]->as<double2>();
            pa.droff = d4->as<size_t>();
            pa.mch = d5->as<int>();
            pa.Uslot = h->Ubuf[l + 1]->as<double2>();
            pa.uoff = d6->as<size_t>();
            pa.Dout = dout;
            pa.dooff = d7->as<size_t>();
            pa.Bout = h->Bbuf.as<double2>();
            pa.boff = d8->as<size_t>();
            pa.tmp = tmp.as<double2>();
            pa.tstride = 2 * tmax;
            int mcmax = 0;
            for (int c = 0; c < nc; ++c) mcmax = h->m[l + 1][c] > mcmax ? h->m[l + 1][c] : mcmax;
            k_post_prep<<<nc, node_threads(mcmax), 0, s>>>(pa);
            FIO_HIP(hipGetLastError());
            ZgemmBatch g1, g2;
            for (int c = 0; c < nc; ++c) {
                const int par = c >> 1, mc = h->m[l + 1][c], r = h->rank[l + 1][c], mp = mpar[par];
                if (mc == 0 || r == 0) continue;
                const int o = (c & 1) ? h->rank[l + 1][par * 2] : 0;
                double2 *T = tmp.as<double2>() + pa.tstride * c, *UcH = T + (size_t)mc * r;
                const double2 *Uc = h->Ubuf[l + 1]->as<double2>() + h->uoff[l + 1][c];
                g1.add(Uc, mc, dpar + dpoff[par] + o + (size_t)o * mp, mp, T, mc, mc, r, r);   // T = U_c A
                g2.add(T, mc, UcH, r, dout + dooff[c], mc, mc, mc, r);                         // D_c += T U_c^*
            }
            g1.upload(s);
            g2.upload(s);
            g1.run(false, zc(1.0, 0.0), zc(0.0, 0.0), s);
            g2.run(false, zc(1.0, 0.0), zc(1.0, 0.0), s);
            FIO_HIP(hipStreamSynchronize(s));
            for (DevBuf *d : {d1, d2, d3, d4, d5, d6, d7, d8}) delete d;
            Dcur.swap(Dnext);
            dpar = Dcur.as<double2>();
            dpoff = dooff;
            mpar = h->m[l + 1];
        }
        return h->rank_capped ? FIO_WARN_RANK_CAP : FIO_OK;
    });
    for (auto *d : Dres) delete d;
    if (st < 0) {
        delete h;
        return st;
    }
    *out = h;
    return st;
}

}  // namespace fio

using namespace fio;

extern "C" fio_status hss_build_from_samples(long n, const hss_opts *opts, hss_matvec_fn matvec, void *matvec_ctx,
                                             hss_omega_fn omega, void *omega_ctx, void *stream, hss_t *out) {
    Sampler sm{matvec, matvec_ctx, omega, omega_ctx};
    return build_impl(n, opts, sm, as_stream(stream), out);
}

// ---------------------------------------------------------------------------
#include "bf.h"

namespace {
struct BfGram {
    fio_bf_s *bf;
    fio_prec prec;           // precision of the sample applies
    DevBuf ws, tmp;
};
int bf_gram_matvec(void *ctx, const void *X, long ldx, void *Y, long ldy, int ncols, void *stream) {
    BfGram *g = static_cast<BfGram *>(ctx);
    fio_status st = guarded([&] {
        hipStream_t s = as_stream(stream);
        // 2D: the HSS tree runs over the Morton order of the frequencies, and the sample
        // blocks are applied in chunks of 64 columns (the 2D coefficient buffers hold
        // 81 N entries per column)
        const bool fint = g->bf->dim == 2;
        const int chunk = fint ? 64 : ncols;
        const int c1 = ncols < chunk ? ncols : chunk;
        g->ws.ensure(bf_ws_bytes(g->bf, c1, g->prec));
        g->tmp.ensure((size_t)g->bf->N * c1 * sizeof(double2));
        for (int c0 = 0; c0 < ncols; c0 += chunk) {
            const int nc = ncols - c0 < chunk ? ncols - c0 : chunk;
            bf_apply_impl(g->bf, false, (const double2 *)X + (size_t)c0 * ldx, ldx, g->tmp.as<double2>(), g->bf->N,
                          nc, g->prec, g->ws.p, s, fint);
            bf_apply_impl(g->bf, true, g->tmp.as<double2>(), g->bf->N, (double2 *)Y + (size_t)c0 * ldy, ldy, nc,
                          g->prec, g->ws.p, s, fint);
        }
        return FIO_OK;
    });
    return st == FIO_OK ? 0 : 1;
}
}  // namespace

extern "C" fio_status fio_hss_build(fio_bf_t bf, const hss_opts *opts, hss_omega_fn omega, void *omega_ctx,
                                    void *stream, hss_t *out) {
    FIO_CHECK_ARG(bf && opts);
    FIO_CHECK_ARG(opts->sample_prec == FIO_PREC_FP64 || (opts->sample_prec == FIO_PREC_FP32 && bf->f32.p));
    BfGram g;
    g.bf = bf;
    g.prec = (fio_prec)opts->sample_prec;
    Sampler sm{bf_gram_matvec, &g, omega, omega_ctx};
    return build_impl(bf->N, opts, sm, as_stream(stream), out);
}

extern "C" fio_status hss_shape(hss_t h, int *levels, int *leaf, long *n, int *ranks, size_t nranks) {
    FIO_CHECK_ARG(h);
    if (levels) *levels = h->Lh;
    if (leaf) *leaf = h->leaf;
    if (n) *n = h->N;
    if (ranks) {
        size_t need = ((size_t)2 << h->Lh) - 2;
        FIO_CHECK_ARG(nranks >= need);
        size_t k = 0;
        for (int l = 1; l <= h->Lh; ++l)
            for (int v : h->rank[l]) ranks[k++] = v;
    }
    return FIO_OK;
}

extern "C" size_t hss_generator_count(long n, int leaf, const int *ranks) {
    if (!ranks || leaf <= 0) return 0;
    int Lh = 0;
    while (((long)leaf << Lh) < n) ++Lh;
    std::vector<std::vector<int>> r(Lh + 1);
    size_t k = 0;
    for (int l = 1; l <= Lh; ++l)
        for (int j = 0; j < (1 << l); ++j) r[l].push_back(ranks[k++]);
    size_t tot = 0;
    for (int l = 1; l <= Lh; ++l)
        for (int j = 0; j < (1 << l); ++j) {
            int m = (l == Lh) ? leaf : r[l + 1][2 * j] + r[l + 1][2 * j + 1];
            tot += (size_t)m * r[l][j];
        }
    for (int l = 0; l < Lh; ++l)
        for (int j = 0; j < (1 << l); ++j) tot += (size_t)r[l + 1][2 * j] * r[l + 1][2 * j + 1];
    tot += (size_t)(1 << Lh) * leaf * leaf;
    return tot;
}

extern "C" fio_status hss_export(hss_t h, void *host_out, size_t count, void *stream) {
    FIO_CHECK_ARG(h && host_out);
    std::vector<int> ranks;
    for (int l = 1; l <= h->Lh; ++l)
        for (int v : h->rank[l]) ranks.push_back(v);
    FIO_CHECK_ARG(count == hss_generator_count(h->N, h->leaf, ranks.data()));
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        double2 *o = (double2 *)host_out;
        for (int l = 1; l <= h->Lh; ++l)
            for (int j = 0; j < h->nodes(l); ++j) {
                size_t e = (size_t)h->m[l][j] * h->rank[l][j];
                if (e) FIO_HIP(hipMemcpyAsync(o, h->U(l, j), e * sizeof(double2), hipMemcpyDeviceToHost, s));
                o += e;
            }
        size_t nb = 0;
        for (int l = 0; l < h->Lh; ++l)
            for (int j = 0; j < h->nodes(l); ++j) nb += (size_t)h->rank[l + 1][2 * j] * h->rank[l + 1][2 * j + 1];
        if (nb) FIO_HIP(hipMemcpyAsync(o, h->Bbuf.p, nb * sizeof(double2), hipMemcpyDeviceToHost, s));
        o += nb;
        size_t nd = (size_t)h->nodes(h->Lh) * h->leaf * h->leaf;
        FIO_HIP(hipMemcpyAsync(o, h->Dbuf.p, nd * sizeof(double2), hipMemcpyDeviceToHost, s));
        FIO_HIP(hipStreamSynchronize(s));
        return FIO_OK;
    });
}

extern "C" fio_status hss_import(long n, int leaf, const int *ranks, const void *host_gen, size_t count, void *stream,
                                 hss_t *out) {
    FIO_CHECK_ARG(ranks && host_gen && out && leaf >= 1 && leaf <= kMaxM);
    int Lh = 0;
    while (((long)leaf << Lh) < n) ++Lh;
    FIO_CHECK_ARG(((long)leaf << Lh) == n && Lh >= 1);
    FIO_CHECK_ARG(count == hss_generator_count(n, leaf, ranks));
    hss_s *h = new hss_s();
    h->N = n;
    h->leaf = leaf;
    h->Lh = Lh;
    h->rank.assign(Lh + 1, {});
    h->m.assign(Lh + 1, {});
    h->uoff.assign(Lh + 1, {});
    h->Ubuf.assign(Lh + 1, nullptr);
    size_t k = 0;
    for (int l = 1; l <= Lh; ++l)
        for (int j = 0; j < (1 << l); ++j) h->rank[l].push_back(ranks[k++]);
    fio_status st = guarded([&] {
        hipStream_t s = as_stream(stream);
        for (int l = Lh; l >= 1; --l) hss_layout_level(h, l);
        h->m[0] = {h->rank[1][0] + h->rank[1][1]};
        for (int l = 1; l <= Lh; ++l)
            for (int j = 0; j < h->nodes(l); ++j)
                if (h->m[l][j] > kMaxM || h->rank[l][j] > h->m[l][j] || h->rank[l][j] < 0) return FIO_ERR_ARG;
        hss_layout_B(h);
        const double2 *in = (const double2 *)host_gen;
        for (int l = 1; l <= Lh; ++l)
            for (int j = 0; j < h->nodes(l); ++j) {
                size_t e = (size_t)h->m[l][j] * h->rank[l][j];
                if (e) FIO_HIP(hipMemcpyAsync(h->U(l, j), in, e * sizeof(double2), hipMemcpyHostToDevice, s));
                in += e;
            }
        size_t nb = 0;
        for (int l = 0; l < Lh; ++l)
            for (int j = 0; j < h->nodes(l); ++j) nb += (size_t)h->rank[l + 1][2 * j] * h->rank[l + 1][2 * j + 1];
        if (nb) FIO_HIP(hipMemcpyAsync(h->Bbuf.p, in, nb * sizeof(double2), hipMemcpyHostToDevice, s));
        in += nb;
        size_t nd = (size_t)h->nodes(Lh) * leaf * leaf;
        FIO_HIP(hipMemcpyAsync(h->Dbuf.p, in, nd * sizeof(double2), hipMemcpyHostToDevice, s));
        FIO_HIP(hipStreamSynchronize(s));
        return FIO_OK;
    });
    if (st != FIO_OK) {
        delete h;
        return st;
    }
    *out = h;
    return FIO_OK;
}

// Y = H X by the telescoping form: upward xhat = U^* x, downward yhat from B and the
// parent's yhat, leaves y = D x + U yhat.  All steps are batched GEMMs.
extern "C" fio_status hss_matvec(hss_t h, const void *X, long ldx, void *Y, long ldy, int nrhs, void *stream) {
    FIO_CHECK_ARG(h && X && Y && ldx >= h->N && ldy >= h->N && nrhs >= 0);
    if (nrhs == 0) return FIO_OK;
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        const int Lh = h->Lh;
        std::vector<long> rtot(Lh + 1, 0);
        for (int l = 1; l <= Lh; ++l) rtot[l] = level_rows_r(h, l);
        std::vector<DevBuf *> xh(Lh + 1, nullptr), yh(Lh + 1, nullptr);
        for (int l = 1; l <= Lh; ++l) {
            xh[l] = new DevBuf((size_t)(rtot[l] + 1) * nrhs * sizeof(double2));
            yh[l] = new DevBuf((size_t)(rtot[l] + 1) * nrhs * sizeof(double2));
        }
        const double2 *x = (const double2 *)X;
        double2 *y = (double2 *)Y;
        // upward
        lift_level(h, Lh, x, ldx, xh[Lh]->as<double2>(), rtot[Lh], nrhs, true, s);
        for (int l = Lh - 1; l >= 1; --l)
            lift_level(h, l, xh[l + 1]->as<double2>(), rtot[l + 1], xh[l]->as<double2>(), rtot[l], nrhs, true, s);
        // downward: children of level l
        for (int l = 0; l < Lh; ++l) {
            double2 *yc = yh[l + 1]->as<double2>();
            const double2 *xc = xh[l + 1]->as<double2>();
            long ldc = rtot[l + 1];
            if (l > 0) lift_level(h, l, yh[l]->as<double2>(), rtot[l], yc, ldc, nrhs, false, s);
            ZgemmBatch b1, b2;
            long ro = 0;
            for (int j = 0; j < h->nodes(l); ++j) {
                int r1 = h->rank[l + 1][2 * j], r2 = h->rank[l + 1][2 * j + 1];
                // y_a2 += B x_a1 ; y_a1 += B^* x_a2
                b1.add(h->B(l, j), r2, xc + ro, ldc, yc + ro + r1, ldc, r2, nrhs, r1);
                b2.add(h->B(l, j), r2, xc + ro + r1, ldc, yc + ro, ldc, r1, nrhs, r2);
                ro += r1 + r2;
            }
            double2 beta = l > 0 ? zc(1.0) : zc(0.0);
            if (l == 0) {
                FIO_HIP(hipMemsetAsync(yc, 0, (size_t)ldc * nrhs * sizeof(double2), s));
                beta = zc(1.0);
            }
            b1.upload(s);
            b1.run(false, zc(1.0), beta, s);
            b2.upload(s);
            b2.run(true, zc(1.0), beta, s);
            FIO_HIP(hipStreamSynchronize(s));
        }
        // leaves: y = D x + U yhat
        ZgemmBatch bd, bu;
        long ro = 0;
        for (int j = 0; j < h->nodes(Lh); ++j) {
            int r = h->rank[Lh][j];
            bd.add(h->D(j), h->leaf, x + (size_t)j * h->leaf, ldx, y + (size_t)j * h->leaf, ldy, h->leaf, nrhs, h->leaf);
            bu.add(h->U(Lh, j), h->leaf, yh[Lh]->as<double2>() + ro, rtot[Lh], y + (size_t)j * h->leaf, ldy, h->leaf,
                   nrhs, r);
            ro += r;
        }
        bd.upload(s);
        bd.run(false, zc(1.0), zc(0.0), s);
        bu.upload(s);
        bu.run(false, zc(1.0), zc(1.0), s);
        FIO_HIP(hipStreamSynchronize(s));
        for (int l = 1; l <= Lh; ++l) {
            delete xh[l];
            delete yh[l];
        }
        return FIO_OK;
    });
}

extern "C" void hss_destroy(hss_t h) { delete h; }

extern "C" void fio_hss_set_big_node(int rows) { fio::g_big_node = rows > 0 ? rows : 256; }
