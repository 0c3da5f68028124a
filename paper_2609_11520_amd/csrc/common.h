// Shared device/host helpers of the fiohss HIP library (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/fiohss.h"

namespace fio {

// ---------------------------------------------------------------------------
// complex arithmetic on HIP vector types (double2 / float2 = (re, im))
template <typename T> struct cplx;
template <> struct cplx<double> { using type = double2; };
template <> struct cplx<float> { using type = float2; };
template <typename T> using cpx = typename cplx<T>::type;

template <typename C> __host__ __device__ __forceinline__ C cmake(decltype(C{}.x) re, decltype(C{}.x) im) {
    C c; c.x = re; c.y = im; return c;
}
template <typename C> __device__ __forceinline__ C czero() { C c; c.x = 0; c.y = 0; return c; }
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc += a * b
template <typename C> __device__ __forceinline__ void cfma(C &acc, C a, C b) {
    acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename C> __device__ __forceinline__ void cfmac(C &acc, C a, C b) {
    acc.x = fma(a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmake<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C{}.x) s) { return cmake<C>(a.x * s, a.y * s); }

__host__ __device__ inline double2 zc(double re, double im = 0.0) {
    double2 c;
    c.x = re;
    c.y = im;
    return c;
}

// ---------------------------------------------------------------------------
struct Err {
    fio_status st;
};

#define FIO_HIP(call)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) {                                                                 \
            fprintf(stderr, "fiohss: %s failed at %s:%d: %s\n", #call, __FILE__, __LINE__,      \
                    hipGetErrorString(e_));                                                     \
            throw ::fio::Err{e_ == hipErrorOutOfMemory ? FIO_ERR_OOM : FIO_ERR_HIP};            \
        }                                                                                       \
    } while (0)

#define FIO_CHECK_ARG(cond)                                                                     \
    do {                                                                                        \
        if (!(cond)) {                                                                          \
            fprintf(stderr, "fiohss: invalid argument: %s (%s:%d)\n", #cond, __FILE__, __LINE__); \
            return FIO_ERR_ARG;                                                                 \
        }                                                                                       \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline unsigned grid1d(size_t threads, unsigned block) {
    return (unsigned)((threads + block - 1) / block);
}

// RAII device buffer
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    explicit DevBuf(size_t b) { alloc(b); }
    void alloc(size_t b) {
        release();
        if (b) FIO_HIP(hipMalloc(&p, b));
        bytes = b;
    }
    void ensure(size_t b) {
        if (b > bytes) alloc(b);
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
    void swap(DevBuf &o) {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
    }
};

// Runs f() and maps library exceptions to status codes.
template <typename F> fio_status guarded(F &&f) {
    try {
        return f();
    } catch (const Err &e) {
        return e.st;
    } catch (const std::bad_alloc &) {
        return FIO_ERR_OOM;
    }
}

// ---------------------------------------------------------------------------
// batched variable-size complex GEMM (gemm.hip):
//   C_b = alpha op(A_b) B_b + beta C_b,  op(A) = A or A^* (conjugate transpose).
// All matrices column-major, entries complex128.
struct ZgemmDesc {
    const double2 *A;
    const double2 *B;
    double2 *C;
    int M, N, K;
    int lda, ldb, ldc;
};
void zgemm_vbatched(const ZgemmDesc *d_descs, int count, int maxM, int maxN, bool conjA, double2 alpha,
                    double2 beta, hipStream_t s);
// a single GEMM whose descriptor travels as a kernel argument (no device copy needed)
void zgemm_one(const ZgemmDesc &d, bool conjA, double2 alpha, double2 beta, hipStream_t s);

// Host-side helper that keeps a device copy of a descriptor list.
struct ZgemmBatch {
    std::vector<ZgemmDesc> h;
    DevBuf d;
    int maxM = 0, maxN = 0;
    void add(const double2 *A, int lda, const double2 *B, int ldb, double2 *C, int ldc, int M, int N, int K) {
        if (M <= 0 || N <= 0) return;
        h.push_back(ZgemmDesc{A, B, C, M, N, K, lda, ldb, ldc});
        if (M > maxM) maxM = M;
        if (N > maxN) maxN = N;
    }
    void upload(hipStream_t s) {
        if (h.empty()) return;
        d.ensure(h.size() * sizeof(ZgemmDesc));
        FIO_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(ZgemmDesc), hipMemcpyHostToDevice, s));
    }
    void run(bool conjA, double2 alpha, double2 beta, hipStream_t s) {
        if (h.empty()) return;
        zgemm_vbatched(d.as<ZgemmDesc>(), (int)h.size(), maxM, maxN, conjA, alpha, beta, s);
    }
};

}  // namespace fio

// Opaque handle bodies (declared here so that every translation unit sees them).
struct fio_bf_s;
struct hss_s;
struct hss_ulv_s;
