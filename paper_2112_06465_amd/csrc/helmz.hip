// Host side of the helmz C-ABI: argument checks, workspace carving, launch
// geometry and the BiCGStab driver.  All arithmetic runs in the kernels of
// hz_kernels.hpp; the host only sequences launches and polls a done flag.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>

#include "helmz.h"
#include "hz_kernels.hpp"

using hz::cx;
using hz::Geom;
using hz::kBlock;
using hz::kMaxGrid;
using hz::kParts;
using hz::SolverScal;

struct hz_handle {
    int device;
    double* part;          // kParts * kMaxGrid partials for standalone reductions
    int* dflag;            // device word for CSR validation
    unsigned long long* dcount;  // device counter for the locality test
    unsigned long long* hcount;  // pinned host copy
    int* hflag;            // pinned host word
    SolverScal* hsc;       // pinned host copy of the solver scalars
    SolverScal* hsc2;      // pinned host copy of the refinement's outer scalars
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool misaligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) != 0; }

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}

#define HZ_HIP(call)                                  \
    do {                                              \
        if ((call) != hipSuccess) return HZ_ERR_HIP;  \
    } while (0)

// Lanes per row for the vector-CSR kernels: the smallest power of two not
// below half the mean row length, in [2, 64], so each lane holds about two
// entries of a row.  HZ_SPMV_LANES overrides (tuning).
int pick_lanes(int n, int64_t nnz) {
    if (const char* env = std::getenv("HZ_SPMV_LANES")) {
        int v = std::atoi(env);
        if (v == 2 || v == 4 || v == 8 || v == 16 || v == 32 || v == 64) return v;
    }
    const double mean = n > 0 ? double(nnz) / double(n) : 1.0;
    int L = 2;
    while (L < 64 && 2 * L < mean) L *= 2;
    return L;
}

// Contiguous chunks of rows per block (see hz_kernels.hpp): G <= kMaxGrid
// blocks, a multiple of 8 when there are at least 8, chunk = ceil(n / G).
Geom geom_for(int n, int step) {
    const int64_t steps = (int64_t(n) + step - 1) / step;
    int64_t G = steps < kMaxGrid ? steps : kMaxGrid;
    if (G < 1) G = 1;
    if (G >= hz::kXcd) G -= G % hz::kXcd;
    const int64_t chunk = (int64_t(n) + G - 1) / G;
    return Geom{int(G), int(chunk > 0 ? chunk : 1)};
}

inline dim3 grid1(int64_t n) { return dim3(unsigned((n + kBlock - 1) / kBlock)); }

// Entries per lane batch: U independent loads of each kind per lane.
constexpr int batch_for(int L) { return L >= 16 ? 1 : 2; }

// Calls f.template operator()<L, U>() for the lane width chosen at run time.
template <typename F> void with_lanes(int L, F&& f) {
    switch (L) {
        case 2: f.template operator()<2, batch_for(2)>(); break;
        case 4: f.template operator()<4, batch_for(4)>(); break;
        case 8: f.template operator()<8, batch_for(8)>(); break;
        case 16: f.template operator()<16, batch_for(16)>(); break;
        case 32: f.template operator()<32, batch_for(32)>(); break;
        default: f.template operator()<64, batch_for(64)>(); break;
    }
}

template <typename T, int EPI>
void launch_spmv(int L, const hz::SpmvArgs<T>& a, hipStream_t s) {
    with_lanes(L, [&]<int LL, int UU>() {
        hipLaunchKernelGGL((hz::k_spmv<T, LL, UU, EPI>), dim3(a.geo.G), dim3(kBlock), 0, s, a);
    });
}

template <typename T>
hz::SpmvArgs<T> spmv_args(int n, Geom geo, const int* rp, const int* ci, const cx<T>* v, const cx<T>* x, cx<T>* y,
                          const cx<T>* w, double* part) {
    hz::SpmvArgs<T> a;
    a.n = n;
    a.geo = geo;
    a.row_ptr = rp;
    a.col_idx = ci;
    a.vals = v;
    a.x = x;
    a.y = y;
    a.w = w;
    a.part = part;
    return a;
}

// Device CSR structure check; synchronises the stream.
int validate_csr(hz_handle* h, hipStream_t s, int n, int nnz, const int* rp, const int* ci) {
    HZ_HIP(hipMemsetAsync(h->dflag, 0, sizeof(int), s));
    hipLaunchKernelGGL(hz::k_validate, grid1(int64_t(n) + 1), dim3(kBlock), 0, s, n, nnz, rp, ci, h->dflag);
    HZ_HIP(hipGetLastError());
    HZ_HIP(hipMemcpyAsync(h->hflag, h->dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    return *h->hflag ? HZ_ERR_INVALID : HZ_OK;
}

// Enqueue the locality count: entries with |col - row| > kFarRows.  Read
// *h->hcount after the next stream synchronisation.
constexpr int kFarRows = 32768;  // 512 KiB of complex128 x on either side of the row
int enqueue_far_count(hz_handle* h, hipStream_t s, int n, const int* rp, const int* ci) {
    HZ_HIP(hipMemsetAsync(h->dcount, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(hz::k_far_count, grid1(n), dim3(kBlock), 0, s, n, rp, ci, kFarRows, h->dcount);
    HZ_HIP(hipGetLastError());
    HZ_HIP(hipMemcpyAsync(h->hcount, h->dcount, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    return HZ_OK;
}

// Fused iteration (p and s formed per gathered column) unless more than 5 %
// of the entries lie far from the diagonal; HZ_FUSED=0/1 overrides.
bool choose_fused(const hz_handle* h, int64_t nnz) {
    if (const char* env = std::getenv("HZ_FUSED")) return std::atoi(env) != 0;
    return double(*h->hcount) <= 0.05 * double(nnz);
}

int check_csr_args(int n, int nnz, const int* rp, const int* ci, const void* vals) {
    if (n < 0 || nnz < 0) return HZ_ERR_INVALID;
    if (n > 0 && rp == nullptr) return HZ_ERR_INVALID;
    if (nnz > 0 && (ci == nullptr || vals == nullptr)) return HZ_ERR_INVALID;
    if (misaligned(rp, 4) || misaligned(ci, 4)) return HZ_ERR_INVALID;
    return HZ_OK;
}

// ------------------------------------------------------------------ solver workspace

struct SolveWs {
    SolverScal* sc;
    double* part;
    void* vec[8];  // r, rhat, p0, p1, v0, v1, s, t
    void* dinv;
    void* ahat;
};

template <typename T>
size_t ws_layout(int n, int64_t nnz, bool jacobi, char* base, SolveWs* out) {
    const size_t vb = align_up(sizeof(cx<T>) * size_t(n > 0 ? n : 1));
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    SolveWs w{};
    w.sc = static_cast<SolverScal*>(take(sizeof(SolverScal)));
    w.part = static_cast<double*>(take(sizeof(double) * kParts * kMaxGrid));
    for (auto& v : w.vec) v = take(vb);
    w.dinv = jacobi ? take(vb) : nullptr;
    w.ahat = jacobi ? take(sizeof(cx<T>) * size_t(nnz > 0 ? nnz : 1)) : nullptr;
    if (out) *out = w;
    return off;
}

// Arguments shared by the three kernels of an iteration.
template <typename T>
hz::BicgArgs<T> bicg_args(int n, Geom geo, const int* rp, const int* ci, const cx<T>* av, cx<T>* x, const SolveWs& w) {
    hz::BicgArgs<T> a;
    a.n = n;
    a.geo = geo;
    a.row_ptr = rp;
    a.col_idx = ci;
    a.vals = av;
    a.r = static_cast<cx<T>*>(w.vec[0]);
    a.rh = static_cast<const cx<T>*>(w.vec[1]);
    a.p[0] = static_cast<cx<T>*>(w.vec[2]);
    a.p[1] = static_cast<cx<T>*>(w.vec[3]);
    a.v[0] = static_cast<cx<T>*>(w.vec[4]);
    a.v[1] = static_cast<cx<T>*>(w.vec[5]);
    a.s = static_cast<cx<T>*>(w.vec[6]);
    a.t = static_cast<cx<T>*>(w.vec[7]);
    a.x = x;
    a.part = w.part;
    a.sc = w.sc;
    return a;
}

// The iteration loop of BiCGStab on the (possibly column-scaled) matrix
// `av`.  On entry r, rhat and the scalars are initialised (k_fin_init ran).
// Launches at most maxiter iterations of three kernels, then one more
// A-kernel that concludes the last iteration; polls sc->done between
// chunks of 8, 16, ..., 64 iterations.  x holds the iterate (the scaled one,
// y, under Jacobi).
template <typename T>
int iterate(hz_handle* h, hipStream_t s, int n, int L, Geom geo, const int* rp, const int* ci, const cx<T>* av,
            cx<T>* x, const SolveWs& w, int maxiter, bool fused) {
    const hz::BicgArgs<T> a = bicg_args<T>(n, geo, rp, ci, av, x, w);
    const dim3 G(geo.G), B(kBlock);
    int launched = 0, poll = 8;
    with_lanes(L, [&]<int LL, int UU>() {
        while (launched < maxiter) {
            const int m = (maxiter - launched) < poll ? (maxiter - launched) : poll;
            for (int k = 0; k < m; ++k) {
                if (fused) {
                    hipLaunchKernelGGL((hz::k_bicg_A<T, LL, UU>), G, B, 0, s, a);
                    hipLaunchKernelGGL((hz::k_bicg_B<T, LL, UU>), G, B, 0, s, a);
                } else {
                    hipLaunchKernelGGL((hz::k_bicg_P<T>), G, B, 0, s, a);
                    hipLaunchKernelGGL((hz::k_bicg_A1<T, LL, UU>), G, B, 0, s, a);
                    hipLaunchKernelGGL((hz::k_bicg_S<T>), G, B, 0, s, a);
                    hipLaunchKernelGGL((hz::k_bicg_B1<T, LL, UU>), G, B, 0, s, a);
                }
                hipLaunchKernelGGL((hz::k_bicg_C<T>), G, B, 0, s, a);
            }
            launched += m;
            if (launched == maxiter) hipLaunchKernelGGL((hz::k_bicg_P<T>), G, B, 0, s, a);
            if (hipGetLastError() != hipSuccess) return;
            if (hipMemcpyAsync(h->hflag, &w.sc->done, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return;
            if (hipStreamSynchronize(s) != hipSuccess) return;
            if (*h->hflag) break;
            if (poll < 64) poll *= 2;
        }
    });
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}


// Mixed refinement workspace: outer scalars, the complex64 solver's own
// workspace (vectors, partials, scalars, D^{-1}, demoted matrix), the FP64
// residual and the complex64 right-hand side and correction.
struct MixedWs {
    SolverScal* outer;
    SolveWs in;
    double2* r64;
    float2* b32;
    float2* d32;
};

size_t mixed_layout(int n, int64_t nnz, bool jacobi, char* base, MixedWs* out) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    const size_t nn = size_t(n > 0 ? n : 1);
    MixedWs m{};
    m.outer = static_cast<SolverScal*>(take(sizeof(SolverScal)));
    m.in.sc = static_cast<SolverScal*>(take(sizeof(SolverScal)));
    m.in.part = static_cast<double*>(take(sizeof(double) * kParts * kMaxGrid));
    for (auto& v : m.in.vec) v = take(sizeof(float2) * nn);
    m.in.dinv = jacobi ? take(sizeof(float2) * nn) : nullptr;
    m.in.ahat = take(sizeof(float2) * size_t(nnz > 0 ? nnz : 1));
    m.r64 = static_cast<double2*>(take(sizeof(double2) * nn));
    m.b32 = static_cast<float2*>(take(sizeof(float2) * nn));
    m.d32 = static_cast<float2*>(take(sizeof(float2) * nn));
    if (out) *out = m;
    return off;
}

}  // namespace

// ====================================================================== C-ABI

extern "C" {

const char* hz_strerror(int code) {
    switch (code) {
        case HZ_OK: return "ok";
        case HZ_NOT_CONVERGED: return "not converged: iteration limit reached";
        case HZ_BREAKDOWN: return "breakdown: a BiCGStab denominator became exactly zero";
        case HZ_NONFINITE: return "non-finite scalar (NaN or Inf) in the iteration";
        case HZ_ERR_INVALID: return "invalid argument or malformed CSR";
        case HZ_ERR_HIP: return "HIP runtime error";
        case HZ_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
        default: return "unknown helmz status";
    }
}

int hz_handle_create(hz_handle** out) {
    if (out == nullptr) return HZ_ERR_INVALID;
    *out = nullptr;
    hz_handle* h = new (std::nothrow) hz_handle();
    if (h == nullptr) return HZ_ERR_HIP;
    if (hipGetDevice(&h->device) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&h->part), sizeof(double) * kParts * kMaxGrid) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&h->dflag), sizeof(int)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&h->dcount), sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&h->hcount), sizeof(unsigned long long), hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&h->hflag), sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&h->hsc), sizeof(SolverScal), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&h->hsc2), sizeof(SolverScal), hipHostMallocDefault) != hipSuccess) {
        hz_handle_destroy(h);
        return HZ_ERR_HIP;
    }
    *out = h;
    return HZ_OK;
}

int hz_handle_destroy(hz_handle* h) {
    if (h == nullptr) return HZ_OK;
    if (h->part) (void)hipFree(h->part);
    if (h->dflag) (void)hipFree(h->dflag);
    if (h->dcount) (void)hipFree(h->dcount);
    if (h->hcount) (void)hipHostFree(h->hcount);
    if (h->hflag) (void)hipHostFree(h->hflag);
    if (h->hsc) (void)hipHostFree(h->hsc);
    if (h->hsc2) (void)hipHostFree(h->hsc2);
    delete h;
    return HZ_OK;
}

static int spmv_common_checks(hz_handle* h, int n, int nnz, const int* rp, const int* ci, const void* vals,
                              const void* x, void* y, size_t esz) {
    if (h == nullptr) return HZ_ERR_INVALID;
    int rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (n > 0 && (x == nullptr || y == nullptr)) return HZ_ERR_INVALID;
    if (misaligned(x, esz) || misaligned(y, esz) || misaligned(vals, esz)) return HZ_ERR_INVALID;
    if (n > 0 && overlap(x, esz * size_t(n), y, esz * size_t(n))) return HZ_ERR_INVALID;
    return HZ_OK;
}

int csr_zspmv(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci, const hz_c128* vals,
              const hz_c128* x, hz_c128* y) {
    int rc = spmv_common_checks(h, n, nnz, rp, ci, vals, x, y, sizeof(hz_c128));
    if (rc || n == 0) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int L = pick_lanes(n, nnz);
    const Geom geo = geom_for(n, kBlock / L);
    auto a = spmv_args<double>(n, geo, rp, ci, reinterpret_cast<const double2*>(vals),
                               reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), nullptr, nullptr);
    launch_spmv<double, hz::EPI_NONE>(L, a, s);
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

int csr_cspmv(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci, const hz_c64* vals,
              const hz_c64* x, hz_c64* y) {
    int rc = spmv_common_checks(h, n, nnz, rp, ci, vals, x, y, sizeof(hz_c64));
    if (rc || n == 0) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int L = pick_lanes(n, nnz);
    const Geom geo = geom_for(n, kBlock / L);
    auto a = spmv_args<float>(n, geo, rp, ci, reinterpret_cast<const float2*>(vals), reinterpret_cast<const float2*>(x),
                              reinterpret_cast<float2*>(y), nullptr, nullptr);
    launch_spmv<float, hz::EPI_NONE>(L, a, s);
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

int zdotc(hz_handle* h, hz_stream stream, int n, const hz_c128* x, const hz_c128* y, hz_c128* out) {
    if (h == nullptr || n < 0 || out == nullptr) return HZ_ERR_INVALID;
    if (n > 0 && (x == nullptr || y == nullptr)) return HZ_ERR_INVALID;
    if (misaligned(x, 16) || misaligned(y, 16) || misaligned(out, 16)) return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Geom geo = geom_for(n > 0 ? n : 1, kBlock);
    hipLaunchKernelGGL(hz::k_dot_part<0>, dim3(geo.G), dim3(kBlock), 0, s, n, geo,
                       reinterpret_cast<const double2*>(x), reinterpret_cast<const double2*>(y), h->part);
    hipLaunchKernelGGL(hz::k_dot_fin<0>, dim3(1), dim3(kBlock), 0, s, h->part, geo.G, static_cast<void*>(out));
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

int dznrm2(hz_handle* h, hz_stream stream, int n, const hz_c128* x, double* out) {
    if (h == nullptr || n < 0 || out == nullptr) return HZ_ERR_INVALID;
    if (n > 0 && x == nullptr) return HZ_ERR_INVALID;
    if (misaligned(x, 16) || misaligned(out, 8)) return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Geom geo = geom_for(n > 0 ? n : 1, kBlock);
    hipLaunchKernelGGL(hz::k_dot_part<1>, dim3(geo.G), dim3(kBlock), 0, s, n, geo,
                       reinterpret_cast<const double2*>(x), nullptr, h->part);
    hipLaunchKernelGGL(hz::k_dot_fin<1>, dim3(1), dim3(kBlock), 0, s, h->part, geo.G, static_cast<void*>(out));
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

int zaxpy(hz_handle* h, hz_stream stream, int n, hz_c128 alpha, const hz_c128* x, hz_c128* y) {
    if (h == nullptr || n < 0) return HZ_ERR_INVALID;
    if (n == 0) return HZ_OK;
    if (x == nullptr || y == nullptr || misaligned(x, 16) || misaligned(y, 16)) return HZ_ERR_INVALID;
    if (x != y && overlap(x, 16 * size_t(n), y, 16 * size_t(n))) return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double2 a;
    a.x = alpha.re;
    a.y = alpha.im;
    int64_t blocks = (int64_t(n) + kBlock - 1) / kBlock;
    if (blocks > 8 * kMaxGrid) blocks = 8 * kMaxGrid;
    hipLaunchKernelGGL(hz::k_zaxpy, dim3(unsigned(blocks)), dim3(kBlock), 0, s, int64_t(n), a,
                       reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y));
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

size_t zbicgstab_workspace_bytes(int n, int nnz, int flags) {
    if (n < 0 || nnz < 0) return 0;
    return ws_layout<double>(n, nnz, (flags & HZ_PRECOND_JACOBI) != 0, nullptr, nullptr);
}

int zbicgstab_solve(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci, const hz_c128* vals,
                    const hz_c128* b, hz_c128* x, double rtol, int maxiter, int flags, void* ws, size_t ws_bytes,
                    hz_solve_info* info) {
    if (info) std::memset(info, 0, sizeof(*info));
    if (h == nullptr || info == nullptr) return HZ_ERR_INVALID;
    int rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (!(rtol >= 0.0) || maxiter < 0) return HZ_ERR_INVALID;
    if (n == 0) return HZ_OK;
    if (b == nullptr || x == nullptr || misaligned(b, 16) || misaligned(x, 16) || misaligned(vals, 16))
        return HZ_ERR_INVALID;
    if (overlap(b, 16 * size_t(n), x, 16 * size_t(n))) return HZ_ERR_INVALID;
    const bool jacobi = (flags & HZ_PRECOND_JACOBI) != 0;
    SolveWs w;
    const size_t need = ws_layout<double>(n, nnz, jacobi, static_cast<char*>(ws), &w);
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;

    hipStream_t s = static_cast<hipStream_t>(stream);
    if (flags & HZ_VALIDATE) {
        rc = validate_csr(h, s, n, nnz, rp, ci);
        if (rc) return rc;
    }
    const int L = pick_lanes(n, nnz);
    const Geom geo = geom_for(n, kBlock / L);
    const double2* A = reinterpret_cast<const double2*>(vals);
    const double2* bd = reinterpret_cast<const double2*>(b);
    double2* xd = reinterpret_cast<double2*>(x);
    double2* r = static_cast<double2*>(w.vec[0]);
    double2* rh = static_cast<double2*>(w.vec[1]);
    double2* t = static_cast<double2*>(w.vec[7]);
    double2* dinv = static_cast<double2*>(w.dinv);

    SolverScal* hs = h->hsc;
    hipLaunchKernelGGL(hz::k_sc_init, dim3(1), dim3(64), 0, s, w.sc, rtol, maxiter);

    const double2* Aop = A;
    if (jacobi) {
        hipLaunchKernelGGL(hz::k_jacobi_diag<double>, grid1(n), dim3(kBlock), 0, s, n, rp, ci, A, dinv, w.sc);
        double2* ah = static_cast<double2*>(w.ahat);
        if (nnz > 0)
            hipLaunchKernelGGL(hz::k_colscale<double>, grid1(nnz), dim3(kBlock), 0, s, int64_t(nnz), ci, A,
                               static_cast<const double2*>(dinv), ah);
        Aop = ah;
    }
    // initial iterate (y = D x0 under Jacobi) and residual
    const double2* rsrc = bd;
    if (flags & HZ_X0_ZERO) {
        HZ_HIP(hipMemsetAsync(xd, 0, 16 * size_t(n), s));
    } else {
        if (jacobi) hipLaunchKernelGGL(hz::k_diag_apply<double>, grid1(n), dim3(kBlock), 0, s, n, dinv, xd, 1);
        launch_spmv<double, hz::EPI_RESID>(L, spmv_args<double>(n, geo, rp, ci, Aop, xd, r, bd, w.part + hz::kPartI * kMaxGrid), s);
        rsrc = r;
    }
    hipLaunchKernelGGL(hz::k_init<double>, dim3(geo.G), dim3(kBlock), 0, s, n, geo, bd, rsrc, r, rh, w.part);
    hipLaunchKernelGGL(hz::k_fin_init, dim3(1), dim3(kBlock), 0, s, w.part, geo.G, w.sc);
    HZ_HIP(hipGetLastError());
    rc = enqueue_far_count(h, s, n, rp, ci);
    if (rc) return rc;
    HZ_HIP(hipMemcpyAsync(hs, w.sc, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    if (hs->bad_diag) return HZ_ERR_INVALID;

    if (!hs->done) {
        rc = iterate<double>(h, s, n, L, geo, rp, ci, Aop, xd, w, maxiter, choose_fused(h, nnz));
        if (rc) return rc;
    }
    hipLaunchKernelGGL(hz::k_zero_if<double>, grid1(n), dim3(kBlock), 0, s, n, w.sc, xd);
    if (jacobi) hipLaunchKernelGGL(hz::k_diag_apply<double>, grid1(n), dim3(kBlock), 0, s, n, dinv, xd, 0);
    // true residual with the caller's matrix
    launch_spmv<double, hz::EPI_RESID>(L, spmv_args<double>(n, geo, rp, ci, A, xd, t, bd, w.part + hz::kPartI * kMaxGrid), s);
    hipLaunchKernelGGL(hz::k_fin_true, dim3(1), dim3(kBlock), 0, s, w.part, geo.G, w.sc);
    HZ_HIP(hipGetLastError());
    HZ_HIP(hipMemcpyAsync(hs, w.sc, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    info->status = hs->status;
    info->iterations = hs->iters;
    info->outer_steps = 0;
    info->relres_recursive = hs->relres;
    info->relres_true = hs->relres_true;
    return hs->status;
}


size_t zbicgstab_mixed_workspace_bytes(int n, int nnz, int flags) {
    if (n < 0 || nnz < 0) return 0;
    return mixed_layout(n, nnz, (flags & HZ_PRECOND_JACOBI) != 0, nullptr, nullptr);
}

int zbicgstab_solve_mixed(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci,
                          const hz_c128* vals, const hz_c128* b, hz_c128* x, double rtol, double inner_rtol,
                          int maxiter, int max_outer, int flags, void* ws, size_t ws_bytes, hz_solve_info* info) {
    if (info) std::memset(info, 0, sizeof(*info));
    if (h == nullptr || info == nullptr) return HZ_ERR_INVALID;
    int rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (!(rtol >= 0.0) || !(inner_rtol > 0.0) || maxiter < 0 || max_outer < 0) return HZ_ERR_INVALID;
    if (n == 0) return HZ_OK;
    if (b == nullptr || x == nullptr || misaligned(b, 16) || misaligned(x, 16) || misaligned(vals, 16))
        return HZ_ERR_INVALID;
    if (overlap(b, 16 * size_t(n), x, 16 * size_t(n))) return HZ_ERR_INVALID;
    const bool jacobi = (flags & HZ_PRECOND_JACOBI) != 0;
    MixedWs m;
    const size_t need = mixed_layout(n, nnz, jacobi, static_cast<char*>(ws), &m);
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;

    hipStream_t s = static_cast<hipStream_t>(stream);
    if (flags & HZ_VALIDATE) {
        rc = validate_csr(h, s, n, nnz, rp, ci);
        if (rc) return rc;
    }
    const int L = pick_lanes(n, nnz);
    const Geom geo = geom_for(n, kBlock / L);
    const double2* A = reinterpret_cast<const double2*>(vals);
    const double2* bd = reinterpret_cast<const double2*>(b);
    double2* xd = reinterpret_cast<double2*>(x);
    float2* r32 = static_cast<float2*>(m.in.vec[0]);
    float2* rh32 = static_cast<float2*>(m.in.vec[1]);
    const dim3 one(1), B(kBlock);

    hipLaunchKernelGGL(hz::k_sc_init, one, dim3(64), 0, s, m.outer, rtol, max_outer);
    hipLaunchKernelGGL(hz::k_sc_init, one, dim3(64), 0, s, m.in.sc, inner_rtol, maxiter);
    // complex64 copy of the (column-scaled) matrix; r64 holds the FP64 D^{-1} meanwhile
    const double2* dinv64 = nullptr;
    if (jacobi) {
        hipLaunchKernelGGL(hz::k_jacobi_diag<double>, grid1(n), B, 0, s, n, rp, ci, A, m.r64, m.outer);
        hipLaunchKernelGGL(hz::k_demote_vec, grid1(n), B, 0, s, n, static_cast<const double2*>(m.r64),
                           static_cast<float2*>(m.in.dinv));
        dinv64 = m.r64;
    }
    if (nnz > 0)
        hipLaunchKernelGGL(hz::k_demote_vals, grid1(nnz), B, 0, s, int64_t(nnz), ci, A, dinv64,
                           static_cast<float2*>(m.in.ahat));
    if (flags & HZ_X0_ZERO) HZ_HIP(hipMemsetAsync(xd, 0, 16 * size_t(n), s));
    double* partI = m.in.part + hz::kPartI * kMaxGrid;
    hipLaunchKernelGGL(hz::k_dot_part<1>, dim3(geo.G), B, 0, s, n, geo, bd, nullptr, partI);
    hipLaunchKernelGGL(hz::k_fin_bnorm, one, B, 0, s, partI, geo.G, m.outer);
    HZ_HIP(hipGetLastError());
    rc = enqueue_far_count(h, s, n, rp, ci);
    if (rc) return rc;
    SolverScal* ho = h->hsc2;
    SolverScal* hi = h->hsc;
    HZ_HIP(hipMemcpyAsync(ho, m.outer, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    if (ho->bad_diag) return HZ_ERR_INVALID;
    const bool fused = choose_fused(h, nnz);

    const float2* dinv32 = jacobi ? static_cast<const float2*>(m.in.dinv) : nullptr;
    int inner_total = 0, outer = 0;
    for (;; ++outer) {
        // r = b - A x in FP64, and the outer decision
        launch_spmv<double, hz::EPI_RESID>(L, spmv_args<double>(n, geo, rp, ci, A, xd, m.r64, bd, partI), s);
        hipLaunchKernelGGL(hz::k_fin_outer, one, B, 0, s, partI, geo.G, m.outer, outer, max_outer);
        HZ_HIP(hipGetLastError());
        HZ_HIP(hipMemcpyAsync(ho, m.outer, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
        HZ_HIP(hipStreamSynchronize(s));
        if (ho->done) break;
        // inner complex64 solve of A d = r / ||r|| from d = 0
        hipLaunchKernelGGL(hz::k_demote_scaled, grid1(n), B, 0, s, n, static_cast<const double2*>(m.r64), m.outer,
                           m.b32);
        HZ_HIP(hipMemsetAsync(m.d32, 0, 8 * size_t(n), s));
        hipLaunchKernelGGL(hz::k_sc_init, one, dim3(64), 0, s, m.in.sc, inner_rtol, maxiter);
        hipLaunchKernelGGL(hz::k_init<float>, dim3(geo.G), B, 0, s, n, geo, static_cast<const float2*>(m.b32),
                           static_cast<const float2*>(m.b32), r32, rh32, m.in.part);
        hipLaunchKernelGGL(hz::k_fin_init, one, B, 0, s, m.in.part, geo.G, m.in.sc);
        HZ_HIP(hipGetLastError());
        rc = iterate<float>(h, s, n, L, geo, rp, ci, static_cast<const float2*>(m.in.ahat), m.d32, m.in, maxiter,
                            fused);
        if (rc) return rc;
        HZ_HIP(hipMemcpyAsync(hi, m.in.sc, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
        HZ_HIP(hipStreamSynchronize(s));
        inner_total += hi->iters;
        if (hi->status == HZ_NONFINITE) {
            info->status = HZ_NONFINITE;
            info->iterations = inner_total;
            info->outer_steps = outer + 1;
            return HZ_NONFINITE;
        }
        hipLaunchKernelGGL(hz::k_promote_add, grid1(n), B, 0, s, n, static_cast<const float2*>(m.d32), dinv32,
                           static_cast<const SolverScal*>(m.outer), xd);
    }
    hipLaunchKernelGGL(hz::k_zero_if<double>, grid1(n), B, 0, s, n, static_cast<const SolverScal*>(m.outer), xd);
    HZ_HIP(hipGetLastError());
    HZ_HIP(hipStreamSynchronize(s));
    info->status = ho->status;
    info->iterations = inner_total;
    info->outer_steps = outer;
    info->relres_recursive = ho->relres;
    info->relres_true = ho->relres_true;
    return ho->status;
}

}  // extern "C"
