// Host side of the helmz C-ABI: argument checks, workspace carving, launch
// geometry and the BiCGStab driver.  All arithmetic runs in the kernels of
// hz_kernels.hpp; the host only sequences launches and polls a done flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "helmz.h"
#include "hz_kernels.hpp"
#include "hz_adjoint.hpp"
#include "hz_reorder.hpp"
#include "hz_multi.hpp"
#include "hz_reliable.hpp"
#include "hz_spmv.hpp"
#include "hz_soltile.hpp"
#include "hz_bicgstabl.hpp"
#include "hz_tfqmr.hpp"
#include "hz_formats.hpp"
#include "hz_stream.hpp"
#include "hz_blas1.hpp"

using hz::cx;
using hz::Geom;
using hz::kBlock;
using hz::kMaxGrid;
using hz::kParts;
using hz::SolverScal;

// Form of a standalone row product (hz_spmv.hpp).
enum SpForm : int { SP_PIPE = HZ_SPMV_FORM_ROWS, SP_TILE = HZ_SPMV_FORM_TILES };
struct SpPlan {
    int form;  // SP_PIPE or SP_TILE
    int L;     // lanes per row of SP_PIPE
};

// What hz_autotune_spmv picked for one matrix (by its index arrays): the lane
// count of the solver kernels' row products and the standalone product's plan.
struct TuneEntry {
    const int* rp;
    const int* ci;
    int n;
    int64_t nnz;
    int L;
    SpPlan sp;
};

// An instantiated graph of one chunk of solver iterations, keyed by the
// kernel family, lane count, chunk length and the kernels' argument bytes.
// `last` is recorded on the launch stream after every launch of the graph, so
// evicting it can first wait for a launch that may still be queued (the
// asynchronous solve enqueues chunks without waiting).
struct GraphEntry {
    std::vector<unsigned char> key;
    hipGraphExec_t exec;
    hipEvent_t last;
};

// Static scratch of the allocation-free solve (zbicgstab_solve_noalloc): one
// copy per GPU the library runs on, held from module load until the process
// ends.  Host code never passes `scratch` itself to a kernel (on the host it
// is only a stand-in symbol): it uses the device address that
// hz_handle_create obtains with hipGetSymbolAddress, with the handle's device
// current, and keeps in the handle.
constexpr size_t kScratchBytes = size_t(96) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct hz_handle {
    int device;
    void* scratch_dev;     // device address of `scratch` on this handle's device
    std::vector<TuneEntry> tune;  // autotuned lanes per row, newest last
    hipStream_t cap;                 // stream the iteration graphs are captured on (never runs work)
    std::vector<GraphEntry> graphs;  // cached iteration graphs, newest last
    double* part;          // kParts * kMaxGrid partials for standalone reductions
    hz::B1Slots b1;        // zdotc / dznrm2 slots, armed at creation
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

// ------------------------------------------------------------------ iteration graphs

constexpr size_t kMaxGraphs = 32;  // instantiated chunks kept per handle

bool graphs_on() {
    const char* e = std::getenv("HZ_NO_GRAPH");
    return !(e != nullptr && e[0] == '1');
}

// Key of a chunk: family, lane count, chunk length, whether the concluding
// kernel is appended, and the bytes of the kernels' argument struct (the
// structs are value-initialised, so padding bytes are zero).
template <typename A>
std::vector<unsigned char> chunk_key(int family, int lanes, int k, int tail, const A& args) {
    const int hdr[4] = {family, lanes, k, tail};
    std::vector<unsigned char> key(sizeof(hdr) + sizeof(A));
    std::memcpy(key.data(), hdr, sizeof(hdr));
    std::memcpy(key.data() + sizeof(hdr), &args, sizeof(A));
    return key;
}

// Enqueues a chunk of solver iterations on s: record(q) issues the chunk's
// kernels on stream q.  The chunk is captured once into a graph on the
// handle's capture stream, instantiated and cached under `key`; later chunks
// with the same key replay it with one hipGraphLaunch.  With HZ_NO_GRAPH=1,
// or if capture or instantiation fails, the kernels are launched directly.
// The cache keeps kMaxGraphs graphs; the oldest is evicted only after its
// last launch has completed (its event), since the asynchronous solve leaves
// chunks queued on the caller's stream.
int graph_launch(GraphEntry& g, hipStream_t s) {
    if (hipGraphLaunch(g.exec, s) != hipSuccess) return HZ_ERR_HIP;
    return hipEventRecord(g.last, s) == hipSuccess ? HZ_OK : HZ_ERR_HIP;
}

void graph_release(GraphEntry& g) {
    (void)hipEventSynchronize(g.last);
    (void)hipGraphExecDestroy(g.exec);
    (void)hipEventDestroy(g.last);
}

template <typename F>
int launch_chunk(hz_handle* h, hipStream_t s, const std::vector<unsigned char>& key, F&& record) {
    if (graphs_on() && h->cap != nullptr) {
        for (GraphEntry& g : h->graphs)
            if (g.key == key) return graph_launch(g, s);
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipEvent_t last = nullptr;
        if (hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            record(h->cap);
            hipError_t e = hipStreamEndCapture(h->cap, &graph);
            if (e == hipSuccess && graph != nullptr) e = hipGraphInstantiateWithFlags(&exec, graph, 0);
            if (graph != nullptr) (void)hipGraphDestroy(graph);
            if (e == hipSuccess && exec != nullptr) e = hipEventCreateWithFlags(&last, hipEventDisableTiming);
            if (e == hipSuccess && exec != nullptr && last != nullptr) {
                if (h->graphs.size() >= kMaxGraphs) {
                    graph_release(h->graphs.front());
                    h->graphs.erase(h->graphs.begin());
                }
                h->graphs.push_back(GraphEntry{key, exec, last});
                return graph_launch(h->graphs.back(), s);
            }
            if (exec != nullptr) (void)hipGraphExecDestroy(exec);
        }
        (void)hipGetLastError();  // a failed capture leaves its error; launch directly instead
    }
    record(s);
    return hipGetLastError() == hipSuccess ? HZ_OK : HZ_ERR_HIP;
}

// Lanes per row for the vector-CSR kernels: the smallest power of two not
// below half the mean row length, in [2, 64], so each lane holds about two
// entries of a row.  HZ_SPMV_LANES overrides (tuning).
int rule_lanes(int n, int64_t nnz) {
    const double mean = n > 0 ? double(nnz) / double(n) : 1.0;
    int L = 2;
    while (L < 64 && 2 * L < mean) L *= 2;
    return L;
}

// The lane count for a matrix: HZ_SPMV_LANES if set, else the handle's
// autotuned choice for these index arrays, else the rule above.
int pick_lanes(const hz_handle* h, const int* rp, const int* ci, int n, int64_t nnz) {
    if (const char* env = std::getenv("HZ_SPMV_LANES")) {
        int v = std::atoi(env);
        if (v == 1 || v == 2 || v == 4 || v == 8 || v == 16 || v == 32 || v == 64) return v;
    }
    if (h != nullptr)
        for (auto it = h->tune.rbegin(); it != h->tune.rend(); ++it)
            if (it->rp == rp && it->ci == ci && it->n == n && it->nnz == nnz) return it->L;
    return rule_lanes(n, nnz);
}

// The lane count of a one-system FP64 solve: pick_lanes, except that a
// matrix whose values exceed half of the 256 MB Infinity Cache (so that every
// product streams them from HBM) runs the block-tile row loop (L = 1) unless
// HZ_SPMV_LANES or the autotuner decided for these arrays.  Measured on the
// 291 MB cabin: 241 against 254 us per BiCGStab iteration, 490 against 556 ms
// for TFQMR to 1e-10; on the 49 MB cylinder, which stays in the cache, vector
// rows are faster (48 against 63 us), and complex64 products stay on rows.
constexpr int64_t kTileSolveBytes = int64_t(128) << 20;
int solve_lanes(const hz_handle* h, const int* rp, const int* ci, int n, int64_t nnz) {
    bool decided = std::getenv("HZ_SPMV_LANES") != nullptr;
    if (!decided && h != nullptr)
        for (const TuneEntry& t : h->tune)
            if (t.rp == rp && t.ci == ci && t.n == n && t.nnz == nnz) decided = true;
    if (!decided && 16 * nnz > kTileSolveBytes) return 1;
    return pick_lanes(h, rp, ci, n, nnz);
}

// The standalone product's plan without tuning: block tiles when a tile of
// mean rows fits the LDS buffer (at most kTileCap / kTileRows = 16 entries per
// row on average), else pipelined rows with the lane rule.  Measured cold:
// tiles 70-74 against 97 us on the renumbered cabin, 287 against 297 us in its
// random numbering, 13.5 against 17.1 us on the cylinder.
SpPlan default_sp(int n, int64_t nnz) {
    const bool tiles = nnz > 0 && nnz <= int64_t(hz::kTileCap / hz::kTileRows) * n;
    return tiles ? SpPlan{SP_TILE, hz::kTileLanes} : SpPlan{SP_PIPE, rule_lanes(n, nnz)};
}

// The standalone product's plan: HZ_SPMV_FORM ("rows" / "tiles") and
// HZ_SPMV_LANES if set, else the autotuned plan, else default_sp.
SpPlan pick_sp(const hz_handle* h, const int* rp, const int* ci, int n, int64_t nnz) {
    SpPlan p = default_sp(n, nnz);
    bool tuned = false;
    if (h != nullptr)
        for (auto it = h->tune.rbegin(); it != h->tune.rend(); ++it)
            if (it->rp == rp && it->ci == ci && it->n == n && it->nnz == nnz) {
                p = it->sp;
                tuned = true;
                break;
            }
    if (const char* env = std::getenv("HZ_SPMV_LANES")) {
        const int v = std::atoi(env);
        if (v == 2 || v == 4 || v == 8 || v == 16 || v == 32 || v == 64) {
            p.L = v;
            if (!tuned) p.form = SP_PIPE;
        }
    }
    if (const char* env = std::getenv("HZ_SPMV_FORM")) {
        if (std::strcmp(env, "rows") == 0) p.form = SP_PIPE;
        if (std::strcmp(env, "tiles") == 0) p.form = SP_TILE;
    }
    return p;
}

// Blocks of a launch over n rows taken `step` rows at a time: G <= kMaxGrid,
// a multiple of 8 when there are at least 8 (one group per XCD, struct Rows).
Geom geom_for(int n, int step) {
    const int64_t steps = (int64_t(n) + step - 1) / step;
    int64_t G = steps < kMaxGrid ? steps : kMaxGrid;
    if (G < 1) G = 1;
    if (G >= hz::kXcd) G -= G % hz::kXcd;
    return Geom{int(G)};
}

inline dim3 grid1(int64_t n) { return dim3(unsigned((n + kBlock - 1) / kBlock)); }

// Entries per lane batch: U independent loads of each kind per lane.
constexpr int batch_for(int L) { return L >= 16 ? 1 : 2; }

// Calls f.template operator()<L, U>() for the lane width chosen at run time.
// L = 1 selects the block-tile form of the solver kernels' row loop (for_tiles).
template <typename F> void with_lanes(int L, F&& f) {
    switch (L) {
        case 1: f.template operator()<1, 1>(); break;
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

// Entries per lane in the first batch of a pipelined row (16 slots up to L = 8).
constexpr int pipe_batch(int L) { return L <= 4 ? 4 : (L == 8 ? 2 : 1); }

// Blocks of a standalone product over n rows, `rows` per block step.
Geom geom_sp(int n, int rows) {
    const int64_t steps = (int64_t(n) + rows - 1) / rows;
    int64_t G = steps < hz::kSpMaxGrid ? steps : hz::kSpMaxGrid;
    if (G < 1) G = 1;
    if (G >= hz::kXcd) G -= G % hz::kXcd;
    return Geom{int(G)};
}

// y = A x on m rows in the plan's form (nnz >= 1 and at least one x element).
template <typename T>
void launch_sp(const SpPlan& p, int m, int nnz, const int* rp, const int* ci, const cx<T>* v, const cx<T>* x,
               cx<T>* y, hipStream_t s) {
    hz::SpArgs<T> a{m, nnz, Geom{1}, rp, ci, v, x, y};
    if (p.form == SP_TILE) {
        a.geo = geom_sp(m, hz::kTileRows);
        if (a.geo.G >= hz::kSpMaxGrid) {  // blocks loop over the tiles: results through the LDS ring
            a.geo.G = hz::kSpTileGrid;
            hipLaunchKernelGGL((hz::k_spmv_tile<T>), dim3(a.geo.G), dim3(hz::kSpBlock), 0, s, a);
        } else {
            hipLaunchKernelGGL((hz::k_spmv_tile1<T>), dim3(a.geo.G), dim3(hz::kSpBlock), 0, s, a);
        }
        return;
    }
    auto go = [&]<int L>() {
        a.geo = geom_sp(m, hz::kSpBlock / L);
        hipLaunchKernelGGL((hz::k_spmv_pipe<T, L, pipe_batch(L)>), dim3(a.geo.G), dim3(hz::kSpBlock), 0, s, a);
    };
    switch (p.L) {
        case 2: go.template operator()<2>(); break;
        case 4: go.template operator()<4>(); break;
        case 8: go.template operator()<8>(); break;
        case 16: go.template operator()<16>(); break;
        case 32: go.template operator()<32>(); break;
        default: go.template operator()<64>(); break;
    }
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

// The standalone product y = A x (m rows, at least one x element): the plan's
// form, or the vector rows of the solver kernels for a matrix without entries.
template <typename T>
void standalone_spmv(const hz_handle* h, int m, int nnz, const int* rp, const int* ci, const cx<T>* v, const cx<T>* x,
                     cx<T>* y, hipStream_t s) {
    if (nnz > 0) {
        launch_sp<T>(pick_sp(h, rp, ci, m, nnz), m, nnz, rp, ci, v, x, y, s);
        return;
    }
    const int L = pick_lanes(h, rp, ci, m, nnz);
    launch_spmv<T, hz::EPI_NONE>(L, spmv_args<T>(m, geom_for(m, kBlock / L), rp, ci, v, x, y, nullptr, nullptr), s);
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

// Which iteration: the gather-light one (p and s materialised, one gathered
// vector per product, five kernels) or the fused one (p and s formed per
// gathered column, three gathered vectors, three kernels).  On large systems
// the extra gathers cost more than the two launches they save: 1.05x on the
// cylinder (n = 210k), 1.6x on the renumbered cabin, 2.4x on the randomly
// numbered one, a tie at n = 262k.  Up to about 10^5 rows every gathered
// vector sits in L2 and the iteration is launch-bound, so the fused one wins
// (20^3 cube 24.1 -> 21.0 us, 48^3 cube 32.4 -> 30.6 us per iteration).
// `rows` is the total over the systems of a launch.  HZ_FUSED=0/1 overrides.
constexpr int64_t kFusedMaxRows = 131072;
bool choose_fused(const hz_handle*, int64_t rows) {
    if (const char* env = std::getenv("HZ_FUSED")) return std::atoi(env) != 0;
    return rows <= kFusedMaxRows;
}

int check_csr_args(int n, int nnz, const int* rp, const int* ci, const void* vals) {
    if (n < 0 || nnz < 0) return HZ_ERR_INVALID;
    if (n > 0 && rp == nullptr) return HZ_ERR_INVALID;
    if (nnz > 0 && (ci == nullptr || vals == nullptr)) return HZ_ERR_INVALID;
    if (misaligned(rp, 4) || misaligned(ci, 4)) return HZ_ERR_INVALID;
    return HZ_OK;
}

// ------------------------------------------------------------------ solver work map and workspace

using hz::BlockMap;
using hz::SysMap;

// Work map of a solver launch over nsys systems with host row offsets
// row_off[0..nsys].  One system: the G <= kMaxGrid blocks of geom_for in 8
// groups (one per XCD) that deal their eighth of the rows out in tiles.
// Several systems: every system gets ceil(n_j / R) blocks (R rows per
// block, chosen so the whole launch has about kMaxGrid blocks), each with a
// contiguous chunk of its system, blocks of one system are consecutive, and
// the total is padded to a multiple of 8 with empty blocks.
struct WorkMap {
    int nsys = 0, G = 0, stride = 0;
    std::vector<BlockMap> blocks;
    std::vector<SysMap> systems;
};

WorkMap build_map(int nsys, const int* row_off, int L) {
    WorkMap m;
    m.nsys = nsys;
    const int64_t N = int64_t(row_off[nsys]) - row_off[0];
    if (nsys == 1) {
        // one group of blocks per XCD, each group's blocks taking its rows' tiles in turn (struct Rows)
        const Geom geo = geom_for(int(N), kBlock / L);
        const int groups = (geo.G % hz::kXcd == 0) ? hz::kXcd : 1, K = geo.G / groups;
        for (int b = 0; b < geo.G; ++b) {
            const int x = b / K;
            const int64_t x0 = N * x / groups, x1 = N * (x + 1) / groups;
            m.blocks.push_back(BlockMap{0, int(row_off[0] + x0), int(row_off[0] + x1), b % K, K, b});
        }
        m.systems.push_back(SysMap{0, geo.G, row_off[0], row_off[1]});
    } else {
        const int64_t R = std::max<int64_t>(kBlock / L, (N + kMaxGrid - 1) / kMaxGrid);
        for (int j = 0; j < nsys; ++j) {
            const int64_t nj = int64_t(row_off[j + 1]) - row_off[j];
            const int64_t gj = std::max<int64_t>(1, (nj + R - 1) / R);
            const int64_t chunk = std::max<int64_t>(1, (nj + gj - 1) / gj);
            m.systems.push_back(SysMap{int(m.blocks.size()), int(gj), row_off[j], row_off[j + 1]});
            for (int64_t b = 0; b < gj; ++b) {
                const int64_t r0 = std::min<int64_t>(nj, b * chunk), r1 = std::min<int64_t>(nj, r0 + chunk);
                m.blocks.push_back(BlockMap{j, int(row_off[j] + r0), int(row_off[j] + r1), 0, 1, int(b)});
            }
        }
        while (m.blocks.size() >= size_t(hz::kXcd) && m.blocks.size() % hz::kXcd != 0)
            m.blocks.push_back(BlockMap{-1, 0, 0, 0, 1, 0});
    }
    m.G = int(m.blocks.size());
    m.stride = std::max(m.G, kMaxGrid);
    return m;
}

// Solver workspace: per-system scalars, partials, the work map, a done
// counter, eight vectors (r, rhat, p0, p1, v0, v1, s, t) and, under Jacobi,
// D^{-1} and the column-scaled values.
struct SolveWs {
    SolverScal* sc;
    double* part;
    BlockMap* bmap;
    SysMap* smap;
    int* ndone;
    void* vec[8];
    void* dinv;
    void* ahat;
};

// Partial component stride of the BiCGStab workspace for a map of G blocks:
// room for the products' sub-blocks, sol_subs(G) G <= max(2 G, kSolSlots) slots.
int bicg_stride(int G) { return std::max(2 * G, std::max(2 * kMaxGrid, hz::kSolSlots)); }

template <typename T>
size_t ws_layout(int n, int64_t nnz, bool jacobi, int nsys, int G, char* base, SolveWs* out) {
    const size_t vb = align_up(sizeof(cx<T>) * size_t(n > 0 ? n : 1));
    const int stride = bicg_stride(G);
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    SolveWs w{};
    w.sc = static_cast<SolverScal*>(take(sizeof(SolverScal) * size_t(nsys)));
    w.part = static_cast<double*>(take(sizeof(double) * size_t(hz::kParts) * size_t(stride)));
    w.bmap = static_cast<BlockMap*>(take(sizeof(BlockMap) * size_t(G)));
    w.smap = static_cast<SysMap*>(take(sizeof(SysMap) * size_t(nsys)));
    w.ndone = static_cast<int*>(take(sizeof(int)));
    for (auto& v : w.vec) v = take(vb);
    w.dinv = jacobi ? take(vb) : nullptr;
    w.ahat = jacobi ? take(sizeof(cx<T>) * size_t(nnz > 0 ? nnz : 1)) : nullptr;
    if (out) *out = w;
    return off;
}

// Worst case of the one-system map: G <= kMaxGrid.
template <typename T> size_t ws_bytes_single(int n, int64_t nnz, bool jacobi) {
    return ws_layout<T>(n, nnz, jacobi, 1, kMaxGrid, nullptr, nullptr);
}

template <typename T>
hz::BicgArgs<T> bicg_args(const WorkMap& m, const int* rp, const int* ci, const cx<T>* av, const cx<T>* b, cx<T>* x,
                          const SolveWs& w) {
    hz::BicgArgs<T> a{};
    a.G = m.G;
    a.stride = bicg_stride(m.G);
    a.bmap = w.bmap;
    a.smap = w.smap;
    a.ndone = w.ndone;
    a.row_ptr = rp;
    a.col_idx = ci;
    a.vals = av;
    a.b = b;
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

// Upload the map (host vectors stay alive until the caller's next sync).
int upload_map(hipStream_t s, const WorkMap& m, const SolveWs& w) {
    HZ_HIP(hipMemcpyAsync(w.bmap, m.blocks.data(), sizeof(BlockMap) * m.blocks.size(), hipMemcpyHostToDevice, s));
    HZ_HIP(hipMemcpyAsync(w.smap, m.systems.data(), sizeof(SysMap) * m.systems.size(), hipMemcpyHostToDevice, s));
    HZ_HIP(hipMemsetAsync(w.ndone, 0, sizeof(int), s));
    return HZ_OK;
}

// The iteration loop of BiCGStab on the (possibly column-scaled) matrix in
// `a` for every system of the map.  On entry r, rhat and the scalars are
// initialised (k_fin_init ran).  Launches at most maxiter iterations, then
// one more first kernel that concludes the last iteration; polls the
// done-counter between chunks of 8, 16, ..., 64 iterations.
// The gather-light products of a one-system solve on the block-tile row loop
// (L = 1) run as sub-blocks with an LDS result ring (k_bicg_A1t, k_bicg_B1t);
// the returned arguments carry their partial layout.
template <typename T> bool sub_products(const WorkMap& m, int L, bool fused) { return L == 1 && m.nsys == 1 && !fused; }
template <typename T> hz::BicgArgs<T> iteration_args(const WorkMap& m, hz::BicgArgs<T> a, int L, bool fused) {
    a.pf = sub_products<T>(m, L, fused) ? hz::sol_subs(m.G) : 1;
    return a;
}

// One gather-light iteration (P, A1, S, B1, C) on stream q.
template <typename T, int LL, int UU>
void enqueue_gather_light(hipStream_t q, const WorkMap& m, const hz::BicgArgs<T>& a, bool sub) {
    const dim3 G(m.G), B(kBlock);
    hipLaunchKernelGGL((hz::k_bicg_P<T>), G, B, 0, q, a);
    if (sub)
        hipLaunchKernelGGL((hz::k_bicg_A1t<T>), dim3(a.pf * m.G), dim3(hz::kSpBlock), 0, q, a);
    else
        hipLaunchKernelGGL((hz::k_bicg_A1<T, LL, UU>), G, B, 0, q, a);
    hipLaunchKernelGGL((hz::k_bicg_S<T>), G, B, 0, q, a);
    if (sub)
        hipLaunchKernelGGL((hz::k_bicg_B1t<T>), dim3(a.pf * m.G), dim3(hz::kSpBlock), 0, q, a);
    else
        hipLaunchKernelGGL((hz::k_bicg_B1<T, LL, UU>), G, B, 0, q, a);
}

template <typename T>
int iterate(hz_handle* h, hipStream_t s, const WorkMap& m, const hz::BicgArgs<T>& a0, int L, int maxiter, bool fused,
            bool poll_done = true, bool graphs = true) {
    const dim3 G(m.G), B(kBlock);
    const hz::BicgArgs<T> a = iteration_args(m, a0, L, fused);
    const bool sub = sub_products<T>(m, L, fused);
    int launched = 0, poll = poll_done ? 8 : 64;
    while (launched < maxiter) {
        const int k_n = (maxiter - launched) < poll ? (maxiter - launched) : poll;
        const bool tail = launched + k_n == maxiter;
        const int family = (fused ? 1 : 2) + (sizeof(T) == 4 ? 10 : 0);
        auto chunk = [&](auto&& record) {
            if (graphs) return launch_chunk(h, s, chunk_key(family, L, k_n, tail, a), record);
            record(s);  // direct launches: no graph is captured or instantiated (nothing allocated)
            return hipGetLastError() == hipSuccess ? int(HZ_OK) : int(HZ_ERR_HIP);
        };
        int rc = chunk([&](hipStream_t q) {
            with_lanes(L, [&]<int LL, int UU>() {
                for (int k = 0; k < k_n; ++k) {
                    if (fused) {
                        hipLaunchKernelGGL((hz::k_bicg_A<T, LL, UU>), G, B, 0, q, a);
                        hipLaunchKernelGGL((hz::k_bicg_B<T, LL, UU>), G, B, 0, q, a);
                    } else {
                        enqueue_gather_light<T, LL, UU>(q, m, a, sub);
                    }
                    hipLaunchKernelGGL((hz::k_bicg_C<T>), G, B, 0, q, a);
                }
                if (tail) hipLaunchKernelGGL((hz::k_bicg_P<T>), G, B, 0, q, a);
            });
        });
        if (rc) return rc;
        launched += k_n;
        if (!poll_done) continue;  // every chunk enqueued; kernels after the exit return at entry
        HZ_HIP(hipMemcpyAsync(h->hflag, a.ndone, sizeof(int), hipMemcpyDeviceToHost, s));
        HZ_HIP(hipStreamSynchronize(s));
        if (*h->hflag >= m.nsys) break;
        if (poll < 64) poll *= 2;
    }
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

// The single-system map of build_map(1, {0, n}, L) written by a kernel into
// the workspace (the asynchronous solve: no host buffer has to outlive the
// call, nothing is allocated and nothing waits), and the done-counter zeroed.
__global__ void k_map_one(BlockMap* bm, SysMap* sm, int* ndone, int n, int G, int groups, int K) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < G) {
        const int x = b / K;
        const int64_t x0 = int64_t(n) * x / groups, x1 = int64_t(n) * (x + 1) / groups;
        bm[b] = BlockMap{0, int(x0), int(x1), b % K, K, b};
    }
    if (b == 0) {
        sm[0] = SysMap{0, G, 0, n};
        *ndone = 0;
    }
}

// x = 0 by a kernel (the allocation-free solve records no memset, so that a
// caller may capture it in a graph).
__global__ void k_zero_c128(int n, double2* x) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = double2{0.0, 0.0};
}

int write_map_one(hipStream_t s, int n, const WorkMap& m, const SolveWs& w) {
    const int groups = (m.G % hz::kXcd == 0) ? hz::kXcd : 1, K = m.G / groups;
    hipLaunchKernelGGL(k_map_one, dim3((m.G + 255) / 256), dim3(256), 0, s, w.bmap, w.smap, w.ndone, n, m.G, groups,
                       K);
    return hipGetLastError() == hipSuccess ? HZ_OK : HZ_ERR_HIP;
}

// hz_solve_info of system 0 from its device scalars (asynchronous solve).
__global__ void k_info_out(const SolverScal* sc, hz_solve_info* info) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    hz_solve_info o;
    o.status = sc->bad_diag ? HZ_ERR_INVALID : sc->status;
    o.iterations = sc->bad_diag ? 0 : sc->iters;
    o.outer_steps = 0;
    o.renumbered = 0;
    o.relres_recursive = sc->relres;
    o.relres_true = sc->relres_true;
    o.breakdown = sc->why;
    o.reserved = 0;
    *info = o;
}

template <typename T>
void launch_sys_resid(int L, const WorkMap& m, const hz::BicgArgs<T>& a, const cx<T>* vals, const cx<T>* xin, cx<T>* y,
                      hipStream_t s) {
    with_lanes(L, [&]<int LL, int UU>() {
        hipLaunchKernelGGL((hz::k_sys_resid<T, LL, UU>), dim3(m.G), dim3(kBlock), 0, s, a, vals, xin, y);
    });
}

// FP64 solve of nsys systems after argument checks.  The matrix may be
// block diagonal (row_off = the systems' row offsets, host array); x is
// in/out; infos[j] receives system j's result.  Returns the largest status.
int solve_fp64(hz_handle* h, hipStream_t s, int nsys, const int* row_off, int nnz, const int* rp, const int* ci,
               const double2* A, const double2* bd, double2* xd, double rtol, int maxiter, int flags, char* ws,
               hz_solve_info* infos, hz_solve_info* info_dev = nullptr, bool direct = false) {
    const bool async = info_dev != nullptr;  // one system; nothing waits for the stream
    // direct (allocation-free solve): kernels only, no memset, no graph capture
    const int n = row_off[nsys] - row_off[0];
    const bool jacobi = (flags & HZ_PRECOND_JACOBI) != 0;
    const int L = nsys == 1 ? solve_lanes(h, rp, ci, n, nnz) : pick_lanes(h, rp, ci, n, nnz);
    const WorkMap m = build_map(nsys, row_off, L);
    SolveWs w;
    ws_layout<double>(n, nnz, jacobi, nsys, m.G, ws, &w);
    int rc = async ? write_map_one(s, n, m, w) : upload_map(s, m, w);
    if (rc) return rc;
    double2* r = static_cast<double2*>(w.vec[0]);
    double2* t = static_cast<double2*>(w.vec[7]);
    double2* dinv = static_cast<double2*>(w.dinv);
    hipLaunchKernelGGL(hz::k_sc_init, dim3((nsys + 255) / 256), dim3(256), 0, s, w.sc, nsys, rtol, maxiter);

    const double2* Aop = A;
    if (jacobi) {
        hipLaunchKernelGGL(hz::k_jacobi_diag<double>, grid1(n), dim3(kBlock), 0, s, n, rp, ci, A, dinv, w.sc);
        double2* ah = static_cast<double2*>(w.ahat);
        if (nnz > 0)
            hipLaunchKernelGGL(hz::k_colscale<double>, grid1(nnz), dim3(kBlock), 0, s, int64_t(nnz), ci, A,
                               static_cast<const double2*>(dinv), ah);
        Aop = ah;
    }
    const hz::BicgArgs<double> a = bicg_args<double>(m, rp, ci, Aop, bd, xd, w);
    // initial iterate (y = D x0 under Jacobi) and residual
    const double2* rsrc = bd;
    if (flags & HZ_X0_ZERO) {
        if (direct)
            hipLaunchKernelGGL(k_zero_c128, grid1(n), dim3(kBlock), 0, s, n, xd);
        else
            HZ_HIP(hipMemsetAsync(xd, 0, 16 * size_t(n), s));
    } else {
        if (jacobi) hipLaunchKernelGGL(hz::k_diag_apply<double>, grid1(n), dim3(kBlock), 0, s, n, dinv, xd, 1);
        launch_sys_resid<double>(L, m, a, Aop, xd, r, s);
        rsrc = r;
    }
    hipLaunchKernelGGL(hz::k_init<double>, dim3(m.G), dim3(kBlock), 0, s, a, rsrc);
    hipLaunchKernelGGL(hz::k_fin_init<double>, dim3(nsys), dim3(kBlock), 0, s, a);
    HZ_HIP(hipGetLastError());
    if (async) {
        rc = iterate<double>(h, s, m, a, L, maxiter, choose_fused(h, n), false, !direct);
        if (rc) return rc;
        hipLaunchKernelGGL(hz::k_zero_if<double>, dim3(m.G), dim3(kBlock), 0, s, a);
        if (jacobi) hipLaunchKernelGGL(hz::k_diag_apply<double>, grid1(n), dim3(kBlock), 0, s, n, dinv, xd, 0);
        const hz::BicgArgs<double> a0 = bicg_args<double>(m, rp, ci, A, bd, xd, w);
        launch_sys_resid<double>(L, m, a0, A, xd, t, s);
        hipLaunchKernelGGL(hz::k_fin_true<double>, dim3(1), dim3(kBlock), 0, s, a0);
        hipLaunchKernelGGL(k_info_out, dim3(1), dim3(64), 0, s, static_cast<const SolverScal*>(w.sc), info_dev);
        HZ_HIP(hipGetLastError());
        return HZ_OK;
    }
    SolverScal* hs = h->hsc;
    HZ_HIP(hipMemcpyAsync(hs, w.sc, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipMemcpyAsync(h->hflag, w.ndone, sizeof(int), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    if (hs->bad_diag) return HZ_ERR_INVALID;

    if (*h->hflag < nsys) {
        rc = iterate<double>(h, s, m, a, L, maxiter, choose_fused(h, n));
        if (rc) return rc;
    }
    hipLaunchKernelGGL(hz::k_zero_if<double>, dim3(m.G), dim3(kBlock), 0, s, a);
    if (jacobi) hipLaunchKernelGGL(hz::k_diag_apply<double>, grid1(n), dim3(kBlock), 0, s, n, dinv, xd, 0);
    // true residual with the caller's matrix
    const hz::BicgArgs<double> a0 = bicg_args<double>(m, rp, ci, A, bd, xd, w);
    launch_sys_resid<double>(L, m, a0, A, xd, t, s);
    hipLaunchKernelGGL(hz::k_fin_true<double>, dim3(nsys), dim3(kBlock), 0, s, a0);
    HZ_HIP(hipGetLastError());
    std::vector<SolverScal> out(nsys);
    HZ_HIP(hipMemcpyAsync(out.data(), w.sc, sizeof(SolverScal) * size_t(nsys), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    int worst = HZ_OK;
    for (int j = 0; j < nsys; ++j) {
        infos[j].status = out[j].status;
        infos[j].iterations = out[j].iters;
        infos[j].outer_steps = 0;
        infos[j].relres_recursive = out[j].relres;
        infos[j].relres_true = out[j].relres_true;
        infos[j].breakdown = out[j].why;
        worst = std::max(worst, out[j].status);
    }
    return worst;
}

// ------------------------------------------------------------------ level-set reordering

// Scratch of the ordering: BFS levels (later the permuted row lengths),
// non-empty-level flags, two device words (start node, last level), sort
// keys and values, and the rocPRIM sort/scan scratch.
struct LevelWs {
    int* level;  // n + 1
    int* active; // n + 1
    int* scal;   // [0] start node, [1] last level found
    unsigned* key;
    unsigned* key2;
    int* idx;
    int* bylevel;             // nodes sorted by (level, index)
    int* off;                 // n + 2: first position of each level in bylevel
    unsigned long long* ck;   // Cuthill-McKee keys of one level, and their sorted copy
    unsigned long long* ck2;
    int* cv;
    void* tmp;
    size_t tmp_bytes;
};

// rocPRIM scratch for the sorts and the scan of n items (the 32-bit level
// sort with end_bit bits, the 64-bit per-level sort, the row-pointer scan).
size_t prim_tmp_bytes(int n, unsigned end_bit) {
    size_t a = 0, b = 0, c = 0;
    const unsigned* ku = nullptr;
    unsigned* ko = nullptr;
    const unsigned long long* k64 = nullptr;
    unsigned long long* k64o = nullptr;
    const int* vi = nullptr;
    int* vo = nullptr;
    if (rocprim::radix_sort_pairs(nullptr, a, ku, ko, vi, vo, unsigned(n), 0u, end_bit) != hipSuccess) return 0;
    if (rocprim::radix_sort_pairs(nullptr, c, k64, k64o, vi, vo, unsigned(n), 0u, 64u) != hipSuccess) return 0;
    if (rocprim::inclusive_scan(nullptr, b, vi, vo, size_t(n) + 1, rocprim::plus<int>()) != hipSuccess) return 0;
    return std::max<size_t>(std::max(std::max(a, b), c), 1);
}

size_t level_layout(int n, char* base, LevelWs* out) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    const size_t nn = size_t(n > 0 ? n : 1);
    LevelWs w{};
    w.level = static_cast<int*>(take(sizeof(int) * (nn + 1)));
    w.active = static_cast<int*>(take(sizeof(int) * (nn + 1)));
    w.scal = static_cast<int*>(take(sizeof(int) * 4));
    w.key = static_cast<unsigned*>(take(sizeof(unsigned) * nn));
    w.key2 = static_cast<unsigned*>(take(sizeof(unsigned) * nn));
    w.idx = static_cast<int*>(take(sizeof(int) * nn));
    w.bylevel = static_cast<int*>(take(sizeof(int) * nn));
    w.off = static_cast<int*>(take(sizeof(int) * (nn + 2)));
    w.ck = static_cast<unsigned long long*>(take(sizeof(unsigned long long) * nn));
    w.ck2 = static_cast<unsigned long long*>(take(sizeof(unsigned long long) * nn));
    w.cv = static_cast<int*>(take(sizeof(int) * nn));
    w.tmp_bytes = prim_tmp_bytes(int(nn), 32u);
    w.tmp = take(w.tmp_bytes);
    if (out) *out = w;
    return off;
}

// Breadth-first levels from the node in w.scal[0]; *last = the deepest
// non-empty level.  Level steps are enqueued in chunks (16, 32, ..., 256)
// with one host read of the last level found between chunks; steps past the
// end return at entry.
int bfs(hz_handle* h, hipStream_t s, int n, const int* rp, const int* ci, const LevelWs& w, int* last) {
    hipLaunchKernelGGL(hz::k_bfs_seed, grid1(int64_t(n) + 1), dim3(kBlock), 0, s, n,
                       static_cast<const int*>(w.scal), w.level, w.active, w.scal + 1);
    const dim3 G(unsigned(std::min<int64_t>((int64_t(n) + kBlock - 1) / kBlock, 2 * kMaxGrid)));
    int L = 0, chunk = 16;
    for (;;) {
        for (int k = 0; k < chunk && L < n; ++k, ++L)
            hipLaunchKernelGGL(hz::k_bfs_level, G, dim3(kBlock), 0, s, n, rp, ci, w.level, w.active, w.scal + 1, L);
        HZ_HIP(hipGetLastError());
        HZ_HIP(hipMemcpyAsync(h->hflag, w.scal + 1, sizeof(int), hipMemcpyDeviceToHost, s));
        HZ_HIP(hipStreamSynchronize(s));
        if (*h->hflag < L || L >= n) break;  // level L is empty: the search is complete
        if (chunk < 256) chunk *= 2;
    }
    *last = *h->hflag;
    return HZ_OK;
}

// Level-set (Cuthill-McKee) ordering: a first search from node 0 finds a far
// node (the smallest index on its deepest level), a second search from there
// gives the levels.  A stable sort of (level, caller's index) groups the
// levels; then, level after level, each level is sorted stably by (smallest
// new position of a neighbour on the previous level, degree capped at 255).
// Unreached nodes come last in index order.  perm lists the caller's index
// of every new row, inv is its inverse (also the running positions while the
// levels are placed); level_out (nullable) receives the levels.
int level_order(hz_handle* h, hipStream_t s, int n, const int* rp, const int* ci, const LevelWs& w, int* perm,
                int* inv, int* level_out) {
    HZ_HIP(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(w.scal), 0, 1, s));
    int last = 0;
    int rc = bfs(h, s, n, rp, ci, w, &last);
    if (rc) return rc;
    HZ_HIP(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(w.scal), n, 1, s));
    hipLaunchKernelGGL(hz::k_bfs_far, grid1(n), dim3(kBlock), 0, s, n, static_cast<const int*>(w.level), last, w.scal);
    rc = bfs(h, s, n, rp, ci, w, &last);
    if (rc) return rc;
    if (level_out) HZ_HIP(hipMemcpyAsync(level_out, w.level, sizeof(int) * size_t(n), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(hz::k_order_keys, grid1(n), dim3(kBlock), 0, s, n, static_cast<const int*>(w.level), last, w.key,
                       w.idx);
    const unsigned top = unsigned(last) + 1;  // largest key
    unsigned end_bit = 1;
    while (end_bit < 32 && (top >> end_bit) != 0) ++end_bit;
    size_t tb = prim_tmp_bytes(n, end_bit);
    if (tb == 0 || tb > w.tmp_bytes) return HZ_ERR_WORKSPACE;
    tb = w.tmp_bytes;
    HZ_HIP(rocprim::radix_sort_pairs(w.tmp, tb, static_cast<const unsigned*>(w.key), w.key2,
                                     static_cast<const int*>(w.idx), w.bylevel, unsigned(n), 0u, end_bit, s));
    // level offsets to the host (levels 0..last, then the unreached bucket or n)
    hipLaunchKernelGGL(hz::k_level_starts, grid1(n), dim3(kBlock), 0, s, n, static_cast<const unsigned*>(w.key2),
                       w.off);
    HZ_HIP(hipGetLastError());
    std::vector<int> off(size_t(last) + 2);
    HZ_HIP(hipMemcpyAsync(off.data(), w.off, sizeof(int) * off.size(), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipMemcpyAsync(perm, w.bylevel, sizeof(int) * size_t(n), hipMemcpyDeviceToDevice, s));
    HZ_HIP(hipStreamSynchronize(s));
    // level 0 is the start node alone; every later level by its Cuthill-McKee keys
    hipLaunchKernelGGL(hz::k_cm_place, dim3(1), dim3(kBlock), 0, s, 1, static_cast<const int*>(perm), 0, inv);
    unsigned kbits = 8;
    while (kbits < 64 && (uint64_t(n) >> (kbits - 8)) != 0) ++kbits;
    size_t tb64 = 0;
    {
        const unsigned long long* k64 = nullptr;
        unsigned long long* k64o = nullptr;
        const int* vi = nullptr;
        int* vo = nullptr;
        HZ_HIP(rocprim::radix_sort_pairs(nullptr, tb64, k64, k64o, vi, vo, unsigned(n), 0u, kbits));
        if (tb64 > w.tmp_bytes) return HZ_ERR_WORKSPACE;
    }
    for (int L = 1; L <= last; ++L) {
        const int first = off[L], m = off[L + 1] - off[L];
        if (m <= 0) continue;
        hipLaunchKernelGGL(hz::k_cm_keys, grid1(m), dim3(kBlock), 0, s, m,
                           static_cast<const int*>(w.bylevel) + first, rp, ci, static_cast<const int*>(w.level), L,
                           static_cast<const int*>(inv), n, w.ck, w.cv);
        tb = w.tmp_bytes;
        HZ_HIP(rocprim::radix_sort_pairs(w.tmp, tb, static_cast<const unsigned long long*>(w.ck), w.ck2,
                                         static_cast<const int*>(w.cv), perm + first, unsigned(m), 0u, kbits, s));
        hipLaunchKernelGGL(hz::k_cm_place, grid1(m), dim3(kBlock), 0, s, m, static_cast<const int*>(perm) + first,
                           first, inv);
    }
    hipLaunchKernelGGL(hz::k_invert, grid1(n), dim3(kBlock), 0, s, n, static_cast<const int*>(perm), inv);
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

// P A P^T in CSR: row lengths in the new order, scan, copy with renumbered
// columns, per-row sort by column.
int permute_csr(hipStream_t s, int n, int nnz, const int* rp, const int* ci, const double2* v, const int* perm,
                const int* inv, const LevelWs& w, int* rp2, int* ci2, double2* v2) {
    hipLaunchKernelGGL(hz::k_perm_rowlen, grid1(n), dim3(kBlock), 0, s, n, rp, perm, w.level);
    size_t tb = w.tmp_bytes;
    HZ_HIP(rocprim::inclusive_scan(w.tmp, tb, static_cast<const int*>(w.level), rp2, size_t(n) + 1,
                                   rocprim::plus<int>(), s));
    if (nnz > 0) {
        hipLaunchKernelGGL(hz::k_perm_fill, grid1(int64_t(n) * 8), dim3(kBlock), 0, s, n, rp, ci, v, perm, inv,
                           static_cast<const int*>(rp2), ci2, v2);
        hipLaunchKernelGGL(hz::k_row_sort<double2>, grid1(n), dim3(kBlock), 0, s, n, static_cast<const int*>(rp2), ci2, v2);
    }
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

// A solve in the level-set numbering: the ordering scratch, the permutation
// and its inverse, P A P^T, and P b, P x.
struct ReorderWs {
    LevelWs lv;
    int* perm;
    int* inv;
    int* rp;
    int* ci;
    double2* vals;
    double2* b;
    double2* x;
};

size_t reorder_layout(int n, int64_t nnz, char* base, ReorderWs* out) {
    ReorderWs r{};
    size_t off = level_layout(n, base, &r.lv);
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    const size_t nn = size_t(n > 0 ? n : 1), nz = size_t(nnz > 0 ? nnz : 1);
    r.perm = static_cast<int*>(take(sizeof(int) * nn));
    r.inv = static_cast<int*>(take(sizeof(int) * nn));
    r.rp = static_cast<int*>(take(sizeof(int) * (nn + 1)));
    r.ci = static_cast<int*>(take(sizeof(int) * nz));
    r.vals = static_cast<double2*>(take(sizeof(double2) * nz));
    r.b = static_cast<double2*>(take(sizeof(double2) * nn));
    r.x = static_cast<double2*>(take(sizeof(double2) * nn));
    if (out) *out = r;
    return off;
}

// Renumber when HZ_REORDER is passed, never under HZ_NO_REORDER, otherwise
// when more than 5 % of the entries lie more than kFarRows off the diagonal
// (the same locality test that selects the gather-light iteration).
int want_reorder(hz_handle* h, hipStream_t s, int n, int nnz, const int* rp, const int* ci, int flags, bool* yes) {
    *yes = false;
    if (flags & HZ_NO_REORDER) return HZ_OK;
    if (flags & HZ_REORDER) {
        *yes = true;
        return HZ_OK;
    }
    int rc = enqueue_far_count(h, s, n, rp, ci);
    if (rc) return rc;
    HZ_HIP(hipStreamSynchronize(s));
    *yes = double(*h->hcount) > 0.05 * double(nnz);
    return HZ_OK;
}

// Workspace of a single-system solve: the ordering part (unless renumbering
// is ruled out) followed by the solver's own.
size_t single_ws_bytes(int n, int64_t nnz, int flags) {
    const size_t inner = ws_bytes_single<double>(n, nnz, (flags & HZ_PRECOND_JACOBI) != 0);
    return (flags & HZ_NO_REORDER) ? inner : reorder_layout(n, nnz, nullptr, nullptr) + inner;
}

// Runs inner(rp, ci, A, b, x, ws) on the system renumbered by level sets
// when want_reorder says so (P A P^T (P x) = P b, x scattered back), else on
// the caller's arrays.
template <typename Inner>
int with_renumbering(hz_handle* h, hipStream_t s, int n, int nnz, const int* rp, const int* ci, const double2* A,
                     const double2* b, double2* x, int flags, char* ws, hz_solve_info* info, Inner&& inner) {
    bool re = false;
    int rc = want_reorder(h, s, n, nnz, rp, ci, flags, &re);
    if (rc) return rc;
    if (!re) return inner(rp, ci, A, b, x, ws);
    ReorderWs r;
    const size_t off = reorder_layout(n, nnz, ws, &r);
    rc = level_order(h, s, n, rp, ci, r.lv, r.perm, r.inv, nullptr);
    if (rc) return rc;
    rc = permute_csr(s, n, nnz, rp, ci, A, r.perm, r.inv, r.lv, r.rp, r.ci, r.vals);
    if (rc) return rc;
    hipLaunchKernelGGL(hz::k_gather_perm<double>, grid1(n), dim3(kBlock), 0, s, n, r.perm, b, r.b);
    if (!(flags & HZ_X0_ZERO))
        hipLaunchKernelGGL(hz::k_gather_perm<double>, grid1(n), dim3(kBlock), 0, s, n, r.perm,
                           static_cast<const double2*>(x), r.x);
    HZ_HIP(hipGetLastError());
    rc = inner(r.rp, r.ci, r.vals, r.b, r.x, ws + off);
    if (rc < 0) return rc;
    info->renumbered = 1;
    hipLaunchKernelGGL(hz::k_scatter_perm<double>, grid1(n), dim3(kBlock), 0, s, n, r.perm,
                       static_cast<const double2*>(r.x), x);
    HZ_HIP(hipGetLastError());
    HZ_HIP(hipStreamSynchronize(s));
    return rc;
}

// Single-system FP64 solve (renumbered when the matrix wants it).
int solve_single(hz_handle* h, hipStream_t s, int n, int nnz, const int* rp, const int* ci, const double2* A,
                 const double2* b, double2* x, double rtol, int maxiter, int flags, char* ws, hz_solve_info* info) {
    const int row_off[2] = {0, n};
    return with_renumbering(h, s, n, nnz, rp, ci, A, b, x, flags, ws, info,
                            [&](const int* rp2, const int* ci2, const double2* A2, const double2* b2, double2* x2,
                                char* ws2) {
                                return solve_fp64(h, s, 1, row_off, nnz, rp2, ci2, A2, b2, x2, rtol, maxiter, flags,
                                                  ws2, info);
                            });
}

// ------------------------------------------------------------------ BiCGstab(l)

// Workspace: scalars, partials, the one-system map, the done counter, r~,
// r_0 .. r_l, u_0 .. u_l, a residual vector, Jacobi D^{-1} and A D^{-1},
// the Gram partials and the minimal-residual coefficients.
struct LWs {
    SolverScal* sc;
    double* part;
    BlockMap* bmap;
    SysMap* smap;
    int* ndone;
    double2* rt;
    double2* r[hz::kLMax + 1];
    double2* u[hz::kLMax + 1];
    double2* t;
    double2* dinv;
    double2* ahat;
    double* gpart;
    double2* gam;
};

size_t lws_layout(int n, int64_t nnz, int ell, bool jacobi, char* base, LWs* out) {
    const size_t vb = align_up(sizeof(double2) * size_t(n > 0 ? n : 1));
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    LWs w{};
    w.sc = static_cast<SolverScal*>(take(sizeof(SolverScal)));
    w.part = static_cast<double*>(take(sizeof(double) * size_t(hz::kParts) * size_t(bicg_stride(kMaxGrid))));
    w.bmap = static_cast<BlockMap*>(take(sizeof(BlockMap) * size_t(kMaxGrid)));
    w.smap = static_cast<SysMap*>(take(sizeof(SysMap)));
    w.ndone = static_cast<int*>(take(sizeof(int)));
    w.rt = static_cast<double2*>(take(vb));
    for (int p = 0; p <= ell; ++p) w.r[p] = static_cast<double2*>(take(vb));
    for (int p = 0; p <= ell; ++p) w.u[p] = static_cast<double2*>(take(vb));
    w.t = static_cast<double2*>(take(vb));
    w.dinv = jacobi ? static_cast<double2*>(take(vb)) : nullptr;
    w.ahat = jacobi ? static_cast<double2*>(take(sizeof(double2) * size_t(nnz > 0 ? nnz : 1))) : nullptr;
    w.gpart = static_cast<double*>(take(sizeof(double) * 2 * size_t(hz::kGramPairs) * size_t(hz::kGramMaxGrid)));
    w.gam = static_cast<double2*>(take(sizeof(double2) * (hz::kLMax + 1)));
    if (out) *out = w;
    return off;
}

size_t lsolve_ws_bytes(int n, int64_t nnz, int ell, int flags) {
    const size_t inner = lws_layout(n, nnz, ell, (flags & HZ_PRECOND_JACOBI) != 0, nullptr, nullptr);
    return (flags & HZ_NO_REORDER) ? inner : reorder_layout(n, nnz, nullptr, nullptr) + inner;
}

template <typename F> void with_ell(int ell, F&& f) {
    switch (ell) {
        case 1: f.template operator()<1>(); break;
        case 2: f.template operator()<2>(); break;
        case 3: f.template operator()<3>(); break;
        case 4: f.template operator()<4>(); break;
        case 5: f.template operator()<5>(); break;
        case 6: f.template operator()<6>(); break;
        case 7: f.template operator()<7>(); break;
        default: f.template operator()<8>(); break;
    }
}

// BiCGstab(l) of one system on (rp, ci, A); cycles in chunks of 1, 2, 4, 8
// with a poll of the done counter between chunks, each chunk replayed from a
// cached graph; one more first launch after maxcycles concludes the last.
int solve_l(hz_handle* h, hipStream_t s, int n, int nnz, const int* rp, const int* ci, const double2* A,
            const double2* bd, double2* xd, int ell, double rtol, int maxcycles, int flags, char* ws,
            hz_solve_info* info) {
    const bool jacobi = (flags & HZ_PRECOND_JACOBI) != 0;
    const int L = solve_lanes(h, rp, ci, n, nnz);
    const int row_off[2] = {0, n};
    const WorkMap m = build_map(1, row_off, L);
    LWs w;
    lws_layout(n, nnz, ell, jacobi, ws, &w);
    HZ_HIP(hipMemcpyAsync(w.bmap, m.blocks.data(), sizeof(BlockMap) * m.blocks.size(), hipMemcpyHostToDevice, s));
    HZ_HIP(hipMemcpyAsync(w.smap, m.systems.data(), sizeof(SysMap) * m.systems.size(), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(hz::k_sc_init, dim3(1), dim3(256), 0, s, w.sc, 1, rtol, maxcycles);
    const double2* Aop = A;
    if (jacobi) {
        hipLaunchKernelGGL(hz::k_jacobi_diag<double>, grid1(n), dim3(kBlock), 0, s, n, rp, ci, A, w.dinv, w.sc);
        if (nnz > 0)
            hipLaunchKernelGGL(hz::k_colscale<double>, grid1(nnz), dim3(kBlock), 0, s, int64_t(nnz), ci, A,
                               static_cast<const double2*>(w.dinv), w.ahat);
        Aop = w.ahat;
    }
    // the BiCGStab set-up and finishing kernels on the same map, scalars and partials
    hz::BicgArgs<double> ba{};
    ba.G = m.G;
    ba.stride = bicg_stride(m.G);  // room for the sub-block products' slots (shared regions C and I)
    ba.bmap = w.bmap;
    ba.smap = w.smap;
    ba.ndone = w.ndone;
    ba.row_ptr = rp;
    ba.col_idx = ci;
    ba.vals = Aop;
    ba.b = bd;
    ba.r = w.r[0];
    ba.rh = w.rt;
    ba.x = xd;
    ba.part = w.part;
    ba.sc = w.sc;
    HZ_HIP(hipMemsetAsync(w.ndone, 0, sizeof(int), s));
    HZ_HIP(hipMemsetAsync(w.u[0], 0, 16 * size_t(n), s));
    const double2* rsrc = bd;
    if (flags & HZ_X0_ZERO) {
        HZ_HIP(hipMemsetAsync(xd, 0, 16 * size_t(n), s));
    } else {
        if (jacobi) hipLaunchKernelGGL(hz::k_diag_apply<double>, grid1(n), dim3(kBlock), 0, s, n, w.dinv, xd, 1);
        launch_sys_resid<double>(L, m, ba, Aop, xd, w.t, s);
        rsrc = w.t;
    }
    hipLaunchKernelGGL(hz::k_init<double>, dim3(m.G), dim3(kBlock), 0, s, ba, rsrc);
    hipLaunchKernelGGL(hz::k_fin_init<double>, dim3(1), dim3(kBlock), 0, s, ba);
    HZ_HIP(hipGetLastError());
    SolverScal* hs = h->hsc;
    HZ_HIP(hipMemcpyAsync(hs, w.sc, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipMemcpyAsync(h->hflag, w.ndone, sizeof(int), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    if (hs->bad_diag) return HZ_ERR_INVALID;

    hz::LArgs la{};
    la.G = m.G;
    la.stride = ba.stride;
    const bool sub = L == 1;  // the tile row loop: AU and AR as sub-blocks with the LDS result ring
    la.pf = sub ? hz::sol_subs(m.G) : 1;
    la.bmap = w.bmap;
    la.smap = w.smap;
    la.ndone = w.ndone;
    la.row_ptr = rp;
    la.col_idx = ci;
    la.vals = Aop;
    la.rt = w.rt;
    for (int p = 0; p <= ell; ++p) {
        la.r[p] = w.r[p];
        la.u[p] = w.u[p];
    }
    la.x = xd;
    la.part = w.part;
    la.gpart = w.gpart;
    la.gam = w.gam;
    la.sc = w.sc;
    la.n = n;
    la.ell = ell;
    la.gG = int(std::min<int64_t>(hz::kGramMaxGrid, (int64_t(n) + hz::kGramBlock - 1) / hz::kGramBlock));
    const dim3 G(m.G), B(kBlock);
    auto cycle = [&](hipStream_t q) {
        with_lanes(L, [&]<int LL, int UU>() {
            for (int j = 0; j < ell; ++j) {
                hz::LArgs aj = la;
                aj.j = j;
                hipLaunchKernelGGL(hz::k_l_U, G, B, 0, q, aj);
                if (sub)
                    hipLaunchKernelGGL(hz::k_l_AUt, dim3(aj.pf * m.G), dim3(hz::kSpBlock), 0, q, aj);
                else
                    hipLaunchKernelGGL((hz::k_l_AU<LL, UU>), G, B, 0, q, aj);
                hipLaunchKernelGGL(hz::k_l_R, G, B, 0, q, aj);
                if (sub)
                    hipLaunchKernelGGL(hz::k_l_ARt, dim3(aj.pf * m.G), dim3(hz::kSpBlock), 0, q, aj);
                else
                    hipLaunchKernelGGL((hz::k_l_AR<LL, UU>), G, B, 0, q, aj);
            }
        });
        with_ell(ell, [&]<int EL>() {
            hipLaunchKernelGGL((hz::k_l_gram<EL>), dim3(la.gG), dim3(hz::kGramBlock), 0, q, la);
            hipLaunchKernelGGL((hz::k_l_mr<EL>), dim3(1), B, 0, q, la);
        });
        hipLaunchKernelGGL(hz::k_l_update, G, B, 0, q, la);
    };
    int launched = 0, poll = 1;
    int rc = HZ_OK;
    if (*h->hflag < 1) {
        while (launched < maxcycles) {
            const int k_n = (maxcycles - launched) < poll ? (maxcycles - launched) : poll;
            const bool tail = launched + k_n == maxcycles;
            hz::LArgs a0 = la;
            a0.j = 0;
            rc = launch_chunk(h, s, chunk_key(40 + ell, L, k_n, tail, la), [&](hipStream_t q) {
                for (int k = 0; k < k_n; ++k) cycle(q);
                if (tail) hipLaunchKernelGGL(hz::k_l_U, G, B, 0, q, a0);
            });
            if (rc) return rc;
            launched += k_n;
            HZ_HIP(hipMemcpyAsync(h->hflag, w.ndone, sizeof(int), hipMemcpyDeviceToHost, s));
            HZ_HIP(hipStreamSynchronize(s));
            if (*h->hflag >= 1) break;
            if (poll < 8) poll *= 2;
        }
    }
    hipLaunchKernelGGL(hz::k_zero_if<double>, G, B, 0, s, ba);
    if (jacobi) hipLaunchKernelGGL(hz::k_diag_apply<double>, grid1(n), dim3(kBlock), 0, s, n, w.dinv, xd, 0);
    hz::BicgArgs<double> b0 = ba;  // true residual with the caller's matrix
    b0.vals = A;
    launch_sys_resid<double>(L, m, b0, A, xd, w.t, s);
    hipLaunchKernelGGL(hz::k_fin_true<double>, dim3(1), B, 0, s, b0);
    HZ_HIP(hipGetLastError());
    SolverScal out;
    HZ_HIP(hipMemcpyAsync(&out, w.sc, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    info->status = out.status;
    info->iterations = out.iters;
    info->outer_steps = 0;
    info->relres_recursive = out.relres;
    info->relres_true = out.relres_true;
    info->breakdown = out.why;
    return out.status;
}

// ------------------------------------------------------------------ TFQMR

// Workspace: scalars, partials, the one-system map, the done counter, the
// TFQMR scalars, r_0, r~, w, u, u', A u, A u', v, d, a residual vector,
// Jacobi D^{-1} and A D^{-1}.
struct QWs {
    SolverScal* sc;
    double* part;
    BlockMap* bmap;
    SysMap* smap;
    int* ndone;
    hz::TScal* tq;
    double2 *r0, *rt, *w, *u, *u1, *au, *au1, *v, *d, *t;
    double2* dinv;
    double2* ahat;
};

size_t qws_layout(int n, int64_t nnz, bool jacobi, char* base, QWs* out) {
    const size_t vb = align_up(sizeof(double2) * size_t(n > 0 ? n : 1));
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    QWs w{};
    w.sc = static_cast<SolverScal*>(take(sizeof(SolverScal)));
    w.part = static_cast<double*>(take(sizeof(double) * size_t(hz::kParts) * size_t(kMaxGrid)));
    w.bmap = static_cast<BlockMap*>(take(sizeof(BlockMap) * size_t(kMaxGrid)));
    w.smap = static_cast<SysMap*>(take(sizeof(SysMap)));
    w.ndone = static_cast<int*>(take(sizeof(int)));
    w.tq = static_cast<hz::TScal*>(take(sizeof(hz::TScal)));
    for (double2** v : {&w.r0, &w.rt, &w.w, &w.u, &w.u1, &w.au, &w.au1, &w.v, &w.d, &w.t})
        *v = static_cast<double2*>(take(vb));
    w.dinv = jacobi ? static_cast<double2*>(take(vb)) : nullptr;
    w.ahat = jacobi ? static_cast<double2*>(take(sizeof(double2) * size_t(nnz > 0 ? nnz : 1))) : nullptr;
    if (out) *out = w;
    return off;
}

size_t qsolve_ws_bytes(int n, int64_t nnz, int flags) {
    const size_t inner = qws_layout(n, nnz, (flags & HZ_PRECOND_JACOBI) != 0, nullptr, nullptr);
    return (flags & HZ_NO_REORDER) ? inner : reorder_layout(n, nnz, nullptr, nullptr) + inner;
}

// TFQMR of one system on (rp, ci, A); iterations in chunks of 8, 16, ..., 64
// (three launches each) with a poll of the done counter between chunks,
// each chunk replayed from a cached graph.
int solve_q(hz_handle* h, hipStream_t s, int n, int nnz, const int* rp, const int* ci, const double2* A,
            const double2* bd, double2* xd, double rtol, int maxiter, int flags, char* ws, hz_solve_info* info) {
    const bool jacobi = (flags & HZ_PRECOND_JACOBI) != 0;
    const int L = solve_lanes(h, rp, ci, n, nnz);
    const int row_off[2] = {0, n};
    const WorkMap m = build_map(1, row_off, L);
    QWs w;
    qws_layout(n, nnz, jacobi, ws, &w);
    HZ_HIP(hipMemcpyAsync(w.bmap, m.blocks.data(), sizeof(BlockMap) * m.blocks.size(), hipMemcpyHostToDevice, s));
    HZ_HIP(hipMemcpyAsync(w.smap, m.systems.data(), sizeof(SysMap) * m.systems.size(), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(hz::k_sc_init, dim3(1), dim3(256), 0, s, w.sc, 1, rtol, maxiter);
    const double2* Aop = A;
    if (jacobi) {
        hipLaunchKernelGGL(hz::k_jacobi_diag<double>, grid1(n), dim3(kBlock), 0, s, n, rp, ci, A, w.dinv, w.sc);
        if (nnz > 0)
            hipLaunchKernelGGL(hz::k_colscale<double>, grid1(nnz), dim3(kBlock), 0, s, int64_t(nnz), ci, A,
                               static_cast<const double2*>(w.dinv), w.ahat);
        Aop = w.ahat;
    }
    hz::BicgArgs<double> ba{};  // the BiCGStab set-up and finishing kernels on the same map and scalars
    ba.G = m.G;
    ba.stride = m.stride;
    ba.bmap = w.bmap;
    ba.smap = w.smap;
    ba.ndone = w.ndone;
    ba.row_ptr = rp;
    ba.col_idx = ci;
    ba.vals = Aop;
    ba.b = bd;
    ba.r = w.r0;
    ba.rh = w.rt;
    ba.x = xd;
    ba.part = w.part;
    ba.sc = w.sc;
    HZ_HIP(hipMemsetAsync(w.ndone, 0, sizeof(int), s));
    const double2* rsrc = bd;
    if (flags & HZ_X0_ZERO) {
        HZ_HIP(hipMemsetAsync(xd, 0, 16 * size_t(n), s));
    } else {
        if (jacobi) hipLaunchKernelGGL(hz::k_diag_apply<double>, grid1(n), dim3(kBlock), 0, s, n, w.dinv, xd, 1);
        launch_sys_resid<double>(L, m, ba, Aop, xd, w.t, s);
        rsrc = w.t;
    }
    hipLaunchKernelGGL(hz::k_init<double>, dim3(m.G), dim3(kBlock), 0, s, ba, rsrc);
    hipLaunchKernelGGL(hz::k_fin_init<double>, dim3(1), dim3(kBlock), 0, s, ba);
    hz::QArgs qa{};
    qa.G = m.G;
    qa.stride = m.stride;
    qa.bmap = w.bmap;
    qa.smap = w.smap;
    qa.ndone = w.ndone;
    qa.row_ptr = rp;
    qa.col_idx = ci;
    qa.vals = Aop;
    qa.rt = w.rt;
    qa.w = w.w;
    qa.u = w.u;
    qa.u1 = w.u1;
    qa.au = w.au;
    qa.au1 = w.au1;
    qa.v = w.v;
    qa.d = w.d;
    qa.x = xd;
    qa.part = w.part;
    qa.sc = w.sc;
    qa.tq = w.tq;
    const dim3 G(m.G), B(kBlock);
    hipLaunchKernelGGL(hz::k_q_fin_init, dim3(1), B, 0, s, qa);
    with_lanes(L, [&]<int LL, int UU>() {
        hipLaunchKernelGGL((hz::k_q_init<LL, UU>), G, B, 0, s, qa, static_cast<const double2*>(w.r0));
    });
    HZ_HIP(hipGetLastError());
    SolverScal* hs = h->hsc;
    HZ_HIP(hipMemcpyAsync(hs, w.sc, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipMemcpyAsync(h->hflag, w.ndone, sizeof(int), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    if (hs->bad_diag) return HZ_ERR_INVALID;
    int launched = 0, poll = 8, rc = HZ_OK;
    const bool fused = choose_fused(h, n);  // K3 in one launch (two gathered vectors) or gather-light
    if (*h->hflag < 1) {
        while (launched < maxiter) {
            const int k_n = (maxiter - launched) < poll ? (maxiter - launched) : poll;
            rc = launch_chunk(h, s, chunk_key(fused ? 60 : 61, L, k_n, 0, qa), [&](hipStream_t q) {
                with_lanes(L, [&]<int LL, int UU>() {
                    for (int k = 0; k < k_n; ++k) {
                        hipLaunchKernelGGL(hz::k_q_even, G, B, 0, q, qa);
                        hipLaunchKernelGGL((hz::k_q_odd<LL, UU>), G, B, 0, q, qa);
                        if (fused) {
                            hipLaunchKernelGGL((hz::k_q_next<LL, UU>), G, B, 0, q, qa);
                        } else {
                            hipLaunchKernelGGL(hz::k_q_dir, G, B, 0, q, qa);
                            hipLaunchKernelGGL((hz::k_q_next_light<LL, UU>), G, B, 0, q, qa);
                        }
                    }
                });
            });
            if (rc) return rc;
            launched += k_n;
            HZ_HIP(hipMemcpyAsync(h->hflag, w.ndone, sizeof(int), hipMemcpyDeviceToHost, s));
            HZ_HIP(hipStreamSynchronize(s));
            if (*h->hflag >= 1) break;
            if (poll < 64) poll *= 2;
        }
        hipLaunchKernelGGL(hz::k_q_conclude, dim3(1), dim3(64), 0, s, qa);
    }
    hipLaunchKernelGGL(hz::k_zero_if<double>, G, B, 0, s, ba);
    if (jacobi) hipLaunchKernelGGL(hz::k_diag_apply<double>, grid1(n), dim3(kBlock), 0, s, n, w.dinv, xd, 0);
    hz::BicgArgs<double> b0 = ba;  // true residual with the caller's matrix
    b0.vals = A;
    launch_sys_resid<double>(L, m, b0, A, xd, w.t, s);
    hipLaunchKernelGGL(hz::k_fin_true<double>, dim3(1), B, 0, s, b0);
    HZ_HIP(hipGetLastError());
    SolverScal out;
    HZ_HIP(hipMemcpyAsync(&out, w.sc, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    info->status = out.status;
    info->iterations = out.iters;
    info->outer_steps = 0;
    info->relres_recursive = out.relres;
    info->relres_true = out.relres_true;
    info->breakdown = out.why;
    return out.status;
}


// ------------------------------------------------------------------ storage formats (ELL / HYB, SELL-C-sigma)

// Scratch of the format set-up calls: row lengths and their sorted copy, the
// SELL sort keys and row indices, chunk sizes, HYB remainders and offsets, a
// few result words and the rocPRIM scratch.
struct FmtWs {
    unsigned* len;
    unsigned* len2;
    unsigned long long* key;
    unsigned long long* key2;
    int* idx;
    long long* cw;
    int* rem;
    int* off;
    int* out;
    void* tmp;
    size_t tmp_bytes;
};

size_t fmt_tmp_bytes(int n) {
    size_t a = 0, b = 0, c = 0, d = 0;
    const unsigned* ku = nullptr;
    unsigned* ko = nullptr;
    const unsigned long long* k64 = nullptr;
    unsigned long long* k64o = nullptr;
    const int* vi = nullptr;
    int* vo = nullptr;
    const long long* li = nullptr;
    long long* lo = nullptr;
    if (rocprim::radix_sort_keys_desc(nullptr, a, ku, ko, unsigned(n), 0u, 32u) != hipSuccess) return 0;
    if (rocprim::radix_sort_pairs(nullptr, b, k64, k64o, vi, vo, unsigned(n), 0u, 64u) != hipSuccess) return 0;
    if (rocprim::exclusive_scan(nullptr, c, vi, vo, 0, size_t(n) + 1, rocprim::plus<int>()) != hipSuccess) return 0;
    if (rocprim::exclusive_scan(nullptr, d, li, lo, 0LL, size_t(n) + 1, rocprim::plus<long long>()) != hipSuccess)
        return 0;
    return std::max<size_t>(std::max(std::max(a, b), std::max(c, d)), 1);
}

size_t fmt_layout(int n, char* base, FmtWs* out) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    const size_t nn = size_t(n > 0 ? n : 1);
    FmtWs w{};
    w.len = static_cast<unsigned*>(take(sizeof(unsigned) * nn));
    w.len2 = static_cast<unsigned*>(take(sizeof(unsigned) * nn));
    w.key = static_cast<unsigned long long*>(take(sizeof(unsigned long long) * nn));
    w.key2 = static_cast<unsigned long long*>(take(sizeof(unsigned long long) * nn));
    w.idx = static_cast<int*>(take(sizeof(int) * nn));
    w.cw = static_cast<long long*>(take(sizeof(long long) * (nn + 1)));
    w.rem = static_cast<int*>(take(sizeof(int) * (nn + 1)));
    w.off = static_cast<int*>(take(sizeof(int) * (nn + 1)));
    w.out = static_cast<int*>(take(sizeof(int) * 4));
    w.tmp_bytes = fmt_tmp_bytes(n > 0 ? n : 1);
    w.tmp = take(w.tmp_bytes);
    if (out) *out = w;
    return w.tmp_bytes ? off : 0;
}

// Blocks of a one-thread-per-item format launch: a multiple of 8 when at least 8, for the XCD-contiguous mapping.
int fmt_grid(int64_t threads) {
    const int64_t b = (threads + hz::kFmtBlock - 1) / hz::kFmtBlock;
    return int(b >= 8 ? (b + 7) / 8 * 8 : b);
}

// Blocks of kFmtBlock threads covering n items (the set-up kernels index by kFmtBlock, not the solvers' kBlock).
dim3 fgrid(int64_t n) { return dim3(unsigned((n + hz::kFmtBlock - 1) / hz::kFmtBlock)); }

bool sell_shape_ok(int C, int t) { return C >= 1 && C <= 1024 && (t == 1 || t == 2 || t == 4 || t == 8); }


// ------------------------------------------------------------------ shared-pattern batches

// Lanes reserved per row for B systems: 16, 64 or 256.
int multi_lanes(int B) { return B <= 16 ? 16 : (B <= 64 ? 64 : hz::kMultiMax); }

template <typename F> void with_multi(int BL, F&& f) {
    switch (BL) {
        case 16: f.template operator()<16>(); break;
        case 64: f.template operator()<64>(); break;
        default: f.template operator()<hz::kMultiMax>(); break;
    }
}

constexpr int kMultiU = 4;  // entries in flight per lane in the batched row product (v = A p)
constexpr int kMultiUt = 3;  // the same for t = A s, whose epilogue holds more registers

// Values of a shared-pattern batch: explicit [nnz][B] values, or a
// frequency sweep K - k_j^2 M + i k_j Bm from three real [nnz] arrays and the
// host wavenumbers ks[B].
struct MultiVals {
    const double2* vals = nullptr;
    const double* K = nullptr;
    const double* M = nullptr;
    const double* Bm = nullptr;
    const double* ks = nullptr;
    bool kmb() const { return vals == nullptr; }
};

// Workspace of a shared-pattern batch: per-system scalars, partials
// [kParts][G][BL], the done counter, six [n][B] vectors (r, rhat, p, v, s,
// t) and, under Jacobi, D^{-1} [n][B] plus either the column-scaled values
// [nnz][B] (explicit values) or the scaled gather vectors q = D^{-1} p and
// u = D^{-1} s [n][B] and the rows' diagonal triples [n][4] (a sweep); a
// sweep also keeps its wavenumbers [B].
struct MultiWs {
    SolverScal* sc;
    double* part;
    int* ndone;
    double2* vec[6];
    double2* dinv;
    double2* ahat;
    double2* q;
    double2* u;
    double* kd;
    double* kw;
};

size_t multi_layout(int B, int n, int64_t nnz, bool jacobi, bool kmb, char* base, MultiWs* out) {
    const int BL = multi_lanes(B);
    const Geom geo = geom_for(n, kBlock / BL);
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    const size_t nb = size_t(n > 0 ? n : 1) * size_t(B), zb = size_t(nnz > 0 ? nnz : 1) * size_t(B);
    MultiWs w{};
    w.sc = static_cast<SolverScal*>(take(sizeof(SolverScal) * size_t(B)));
    w.part = static_cast<double*>(take(sizeof(double) * size_t(hz::kParts) * size_t(geo.G) * size_t(BL)));
    w.ndone = static_cast<int*>(take(sizeof(int)));
    for (auto& v : w.vec) v = static_cast<double2*>(take(sizeof(double2) * nb));
    w.dinv = jacobi ? static_cast<double2*>(take(sizeof(double2) * nb)) : nullptr;
    w.ahat = (jacobi && !kmb) ? static_cast<double2*>(take(sizeof(double2) * zb)) : nullptr;
    w.q = (jacobi && kmb) ? static_cast<double2*>(take(sizeof(double2) * nb)) : nullptr;
    w.u = (jacobi && kmb) ? static_cast<double2*>(take(sizeof(double2) * nb)) : nullptr;
    w.kd = (jacobi && kmb) ? static_cast<double*>(take(sizeof(double) * 4 * size_t(n > 0 ? n : 1))) : nullptr;
    w.kw = kmb ? static_cast<double*>(take(sizeof(double) * size_t(B))) : nullptr;
    if (out) *out = w;
    return off;
}

// The five-kernel iteration for every system of the batch, in chunks of 8,
// 16, ..., 64 iterations with a poll of the done counter between chunks; one
// more P-kernel after maxiter concludes the last iteration.
template <int VS>
int iterate_multi(hz_handle* h, hipStream_t s, const hz::MultiArgs& a, int BL, int maxiter) {
    const dim3 G(a.geo.G), Bk(kBlock);
    int launched = 0, poll = 8;
    while (launched < maxiter) {
        const int k_n = (maxiter - launched) < poll ? (maxiter - launched) : poll;
        const bool tail = launched + k_n == maxiter;
        int rc = launch_chunk(h, s, chunk_key(100 + VS, BL, k_n, tail, a), [&](hipStream_t q) {
            with_multi(BL, [&]<int BB>() {
                for (int k = 0; k < k_n; ++k) {
                    hipLaunchKernelGGL((hz::k_m_P<BB>), G, Bk, 0, q, a);
                    hipLaunchKernelGGL((hz::k_m_A1<BB, kMultiU, VS>), G, Bk, 0, q, a);
                    hipLaunchKernelGGL((hz::k_m_S<BB>), G, Bk, 0, q, a);
                    hipLaunchKernelGGL((hz::k_m_B1<BB, kMultiUt, VS>), G, Bk, 0, q, a);
                    hipLaunchKernelGGL((hz::k_m_C<BB>), G, Bk, 0, q, a);
                }
                if (tail) hipLaunchKernelGGL((hz::k_m_P<BB>), G, Bk, 0, q, a);
            });
        });
        if (rc) return rc;
        launched += k_n;
        HZ_HIP(hipMemcpyAsync(h->hflag, a.ndone, sizeof(int), hipMemcpyDeviceToHost, s));
        HZ_HIP(hipStreamSynchronize(s));
        if (*h->hflag >= a.B) break;
        if (poll < 64) poll *= 2;
    }
    return HZ_OK;
}

// y = b - A xin for every system of the batch (the caller's values).
template <int VS>
void launch_m_resid(int BL, const hz::MultiArgs& a, const double2* vals, const double2* xin, double2* y,
                    hipStream_t s) {
    with_multi(BL, [&]<int BB>() {
        hipLaunchKernelGGL((hz::k_m_resid<BB, kMultiU, VS>), dim3(a.geo.G), dim3(kBlock), 0, s, a, vals, xin, y);
    });
}

// B systems on one pattern (vectors [n][B]) after argument checks.  infos[j]
// receives system j's result; returns the largest status.
int solve_multi(hz_handle* h, hipStream_t s, int B, int n, int nnz, const int* rp, const int* ci,
                const MultiVals& mv, const double2* bd, double2* xd, double rtol, int maxiter, int flags, char* ws,
                hz_solve_info* infos) {
    const bool jacobi = (flags & HZ_PRECOND_JACOBI) != 0, kmb = mv.kmb();
    const int BL = multi_lanes(B);
    const Geom geo = geom_for(n, kBlock / BL);
    MultiWs w;
    multi_layout(B, n, nnz, jacobi, kmb, ws, &w);
    const int64_t nB = int64_t(n) * B;
    HZ_HIP(hipMemsetAsync(w.ndone, 0, sizeof(int), s));
    hipLaunchKernelGGL(hz::k_sc_init, dim3((B + 255) / 256), dim3(256), 0, s, w.sc, B, rtol, maxiter);
    hz::MultiArgs a{};
    a.n = n;
    a.B = B;
    a.geo = geo;
    a.row_ptr = rp;
    a.col_idx = ci;
    a.vals = mv.vals;
    a.K = mv.K;
    a.M = mv.M;
    a.Bm = mv.Bm;
    a.kw = w.kw;
    a.b = bd;
    a.r = w.vec[0];
    a.rh = w.vec[1];
    a.p = w.vec[2];
    a.v = w.vec[3];
    a.s = w.vec[4];
    a.t = w.vec[5];
    a.q = a.p;
    a.u = a.s;
    a.x = xd;
    a.part = w.part;
    a.sc = w.sc;
    a.ndone = w.ndone;
    if (kmb) HZ_HIP(hipMemcpyAsync(w.kw, mv.ks, sizeof(double) * size_t(B), hipMemcpyHostToDevice, s));
    if (jacobi) {
        if (kmb) {
            hipLaunchKernelGGL(hz::k_m_jacobi_kmb, grid1(nB), dim3(kBlock), 0, s, n, B, rp, ci, mv.K, mv.M, mv.Bm,
                               static_cast<const double*>(w.kw), w.dinv, w.sc);
            // P and S rebuild D^{-1} from the diagonal triples (24 bytes a row for all systems, not 16 B per system)
            hipLaunchKernelGGL(hz::k_m_diag_kmb, grid1(n), dim3(kBlock), 0, s, n, rp, ci, mv.K, mv.M, mv.Bm, w.kd);
            a.kd = w.kd;
            a.q = w.q;
            a.u = w.u;
        } else {
            hipLaunchKernelGGL(hz::k_m_jacobi, grid1(nB), dim3(kBlock), 0, s, n, B, rp, ci, mv.vals, w.dinv, w.sc);
            if (nnz > 0)
                hipLaunchKernelGGL(hz::k_m_colscale, grid1(int64_t(nnz) * B), dim3(kBlock), 0, s, int64_t(nnz), B,
                                   ci, mv.vals, static_cast<const double2*>(w.dinv), w.ahat);
            a.vals = w.ahat;
        }
    }
    const dim3 G(geo.G), Bk(kBlock);
    const double2* rsrc = bd;
    if (flags & HZ_X0_ZERO) {
        HZ_HIP(hipMemsetAsync(xd, 0, sizeof(double2) * size_t(nB), s));
    } else if (kmb) {
        // r = b - A x0 on the caller's x0, then y0 = D x0
        launch_m_resid<hz::VS_KMB>(BL, a, nullptr, static_cast<const double2*>(xd), a.r, s);
        if (jacobi)
            hipLaunchKernelGGL(hz::k_diag_apply<double>, grid1(nB), Bk, 0, s, int(nB),
                               static_cast<const double2*>(w.dinv), xd, 1);
        rsrc = a.r;
    } else {
        // y0 = D x0, then r = b - (A D^{-1}) y0
        if (jacobi)
            hipLaunchKernelGGL(hz::k_diag_apply<double>, grid1(nB), Bk, 0, s, int(nB),
                               static_cast<const double2*>(w.dinv), xd, 1);
        launch_m_resid<hz::VS_EXPLICIT>(BL, a, a.vals, static_cast<const double2*>(xd), a.r, s);
        rsrc = a.r;
    }
    with_multi(BL, [&]<int BB>() {
        hipLaunchKernelGGL((hz::k_m_init<BB>), G, Bk, 0, s, a, rsrc);
        hipLaunchKernelGGL((hz::k_m_fin_init<BB>), dim3(1), Bk, 0, s, a);
    });
    HZ_HIP(hipGetLastError());
    std::vector<SolverScal> hs(B);
    HZ_HIP(hipMemcpyAsync(hs.data(), w.sc, sizeof(SolverScal) * size_t(B), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipMemcpyAsync(h->hflag, w.ndone, sizeof(int), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < B; ++j)
        if (hs[j].bad_diag) return HZ_ERR_INVALID;
    if (*h->hflag < B) {
        int rc = kmb ? iterate_multi<hz::VS_KMB>(h, s, a, BL, maxiter)
                     : iterate_multi<hz::VS_EXPLICIT>(h, s, a, BL, maxiter);
        if (rc) return rc;
    }
    with_multi(BL, [&]<int BB>() {
        hipLaunchKernelGGL((hz::k_m_zero_if<BB>), G, Bk, 0, s, a);
    });
    if (jacobi)
        hipLaunchKernelGGL(hz::k_diag_apply<double>, grid1(nB), Bk, 0, s, int(nB),
                           static_cast<const double2*>(w.dinv), xd, 0);
    // true residual with the caller's values
    if (kmb)
        launch_m_resid<hz::VS_KMB>(BL, a, nullptr, static_cast<const double2*>(xd), a.t, s);
    else
        launch_m_resid<hz::VS_EXPLICIT>(BL, a, mv.vals, static_cast<const double2*>(xd), a.t, s);
    with_multi(BL, [&]<int BB>() { hipLaunchKernelGGL((hz::k_m_fin_true<BB>), dim3(1), Bk, 0, s, a); });
    HZ_HIP(hipGetLastError());
    HZ_HIP(hipMemcpyAsync(hs.data(), w.sc, sizeof(SolverScal) * size_t(B), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    int worst = HZ_OK;
    for (int j = 0; j < B; ++j) {
        infos[j].status = hs[j].status;
        infos[j].iterations = hs[j].iters;
        infos[j].outer_steps = 0;
        infos[j].renumbered = 0;
        infos[j].relres_recursive = hs[j].relres;
        infos[j].relres_true = hs[j].relres_true;
        infos[j].breakdown = hs[j].why;
        worst = std::max(worst, hs[j].status);
    }
    return worst;
}

// Batched adjoint workspace: the batched solver's workspace, conj(g) [n][B]
// and, unless A_j = A_j^T is asserted, the transposed pattern with the source
// entry of each transposed entry and the conjugate-transposed values [nnz][B].
struct AdjMultiWs {
    char* solve;
    double2* gconj;
    int* t_rp;
    int* t_ci;
    int* t_src;
    int* fill;
    double2* t_vals;
};

size_t adjoint_multi_layout(int B, int n, int64_t nnz, int flags, char* base, AdjMultiWs* out) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    const size_t nn = size_t(n > 0 ? n : 1), nz = size_t(nnz > 0 ? nnz : 1);
    AdjMultiWs a{};
    a.solve =
        static_cast<char*>(take(multi_layout(B, n, nnz, (flags & HZ_PRECOND_JACOBI) != 0, false, nullptr, nullptr)));
    a.gconj = static_cast<double2*>(take(sizeof(double2) * nn * size_t(B)));
    if (!(flags & HZ_SYMMETRIC)) {
        a.t_rp = static_cast<int*>(take(sizeof(int) * (nn + 1)));
        a.t_ci = static_cast<int*>(take(sizeof(int) * nz));
        a.t_src = static_cast<int*>(take(sizeof(int) * nz));
        a.fill = static_cast<int*>(take(sizeof(int) * nn));
        a.t_vals = static_cast<double2*>(take(sizeof(double2) * nz * size_t(B)));
    }
    if (out) *out = a;
    return off;
}

// Mixed refinement workspace: outer scalars, the complex64 solver's own
// workspace (vectors, partials, scalars, map, D^{-1}, demoted matrix), the
// FP64 residual and the complex64 right-hand side and correction.
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
    // the inner workspace always holds the demoted matrix (ahat) and, under Jacobi, D^{-1}
    char* inner = static_cast<char*>(take(ws_layout<float>(n, nnz, true, 1, kMaxGrid, nullptr, nullptr)));
    ws_layout<float>(n, nnz, true, 1, kMaxGrid, inner, &m.in);
    if (!jacobi) m.in.dinv = nullptr;
    m.r64 = static_cast<double2*>(take(sizeof(double2) * nn));
    m.b32 = static_cast<float2*>(take(sizeof(float2) * nn));
    m.d32 = static_cast<float2*>(take(sizeof(float2) * nn));
    if (out) *out = m;
    return off;
}

// ------------------------------------------------------------------ adjoint

// Adjoint workspace: the forward solver's workspace, conj(g), and (unless the
// caller asserts A = A^T) the conjugate transpose A^H in CSR.
struct AdjWs {
    char* solve;
    double2* gconj;
    int* t_rp;
    int* t_ci;
    double2* t_vals;
    int* fill;
};

size_t adjoint_layout(int n, int64_t nnz, int flags, char* base, AdjWs* out) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    const size_t nn = size_t(n > 0 ? n : 1), nz = size_t(nnz > 0 ? nnz : 1);
    AdjWs a{};
    a.solve = static_cast<char*>(take(single_ws_bytes(n, nnz, flags)));
    a.gconj = static_cast<double2*>(take(sizeof(double2) * nn));
    if (!(flags & HZ_SYMMETRIC)) {
        a.t_rp = static_cast<int*>(take(sizeof(int) * (nn + 1)));
        a.t_ci = static_cast<int*>(take(sizeof(int) * nz));
        a.t_vals = static_cast<double2*>(take(sizeof(double2) * nz));
        a.fill = static_cast<int*>(take(sizeof(int) * nn));
    }
    if (out) *out = a;
    return off;
}

void launch_grad_vals(int n, const int* rp, const int* ci, const double2* lam, const double2* x, double2* gv, int L,
                      hipStream_t s) {
    const Geom geo = geom_for(n, kBlock / L);
    with_lanes(L, [&]<int LL, int UU>() {
        constexpr int LG = LL == 1 ? 4 : LL;  // the tile form's lane count reads whole rows per lane group
        hipLaunchKernelGGL((hz::k_grad_vals<LG>), dim3(geo.G), dim3(kBlock), 0, s, n, geo, rp, ci, lam, x, gv);
    });
}


size_t mixed_ws_bytes(int n, int64_t nnz, int flags) {
    const size_t inner = mixed_layout(n, nnz, (flags & HZ_PRECOND_JACOBI) != 0, nullptr, nullptr);
    return (flags & HZ_NO_REORDER) ? inner : reorder_layout(n, nnz, nullptr, nullptr) + inner;
}

// Mixed-precision refinement of one system after argument checks; ws holds
// mixed_layout's workspace.
int solve_mixed(hz_handle* h, hipStream_t s, int n, int nnz, const int* rp, const int* ci, const double2* A,
                const double2* bd, double2* xd, double rtol, double inner_rtol, int maxiter, int max_outer, int flags,
                char* ws, hz_solve_info* info) {
    const bool jacobi = (flags & HZ_PRECOND_JACOBI) != 0;
    MixedWs mw;
    mixed_layout(n, nnz, jacobi, ws, &mw);
    const int L = pick_lanes(h, rp, ci, n, nnz);
    const Geom geo = geom_for(n, kBlock / L);
    const int row_off[2] = {0, n};
    const WorkMap m = build_map(1, row_off, L);
    int rc = upload_map(s, m, mw.in);
    if (rc) return rc;
    const dim3 one(1), B(kBlock);
    double* partI = mw.in.part + hz::kPartI * bicg_stride(m.G);  // the inner solve's region I

    hipLaunchKernelGGL(hz::k_sc_init, one, dim3(64), 0, s, mw.outer, 1, rtol, max_outer);
    hipLaunchKernelGGL(hz::k_sc_init, one, dim3(64), 0, s, mw.in.sc, 1, inner_rtol, maxiter);
    // complex64 copy of the (column-scaled) matrix; r64 holds the FP64 D^{-1} meanwhile
    const double2* dinv64 = nullptr;
    if (jacobi) {
        hipLaunchKernelGGL(hz::k_jacobi_diag<double>, grid1(n), B, 0, s, n, rp, ci, A, mw.r64, mw.outer);
        hipLaunchKernelGGL(hz::k_demote_vec, grid1(n), B, 0, s, n, static_cast<const double2*>(mw.r64),
                           static_cast<float2*>(mw.in.dinv));
        dinv64 = mw.r64;
    }
    if (nnz > 0)
        hipLaunchKernelGGL(hz::k_demote_vals, grid1(nnz), B, 0, s, int64_t(nnz), ci, A, dinv64,
                           static_cast<float2*>(mw.in.ahat));
    if (flags & HZ_X0_ZERO) HZ_HIP(hipMemsetAsync(xd, 0, 16 * size_t(n), s));
    hipLaunchKernelGGL(hz::k_dot_part<1>, dim3(geo.G), B, 0, s, n, geo, bd, nullptr, partI);
    hipLaunchKernelGGL(hz::k_fin_bnorm, one, B, 0, s, partI, geo.G, mw.outer);
    HZ_HIP(hipGetLastError());
    SolverScal* ho = h->hsc2;
    SolverScal* hi = h->hsc;
    HZ_HIP(hipMemcpyAsync(ho, mw.outer, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    if (ho->bad_diag) return HZ_ERR_INVALID;
    const bool fused = choose_fused(h, n);
    const hz::BicgArgs<float> ai =
        bicg_args<float>(m, rp, ci, static_cast<const float2*>(mw.in.ahat), mw.b32, mw.d32, mw.in);

    const float2* dinv32 = jacobi ? static_cast<const float2*>(mw.in.dinv) : nullptr;
    int inner_total = 0, outer = 0;
    for (;; ++outer) {
        // r = b - A x in FP64, and the outer decision
        launch_spmv<double, hz::EPI_RESID>(L, spmv_args<double>(n, geo, rp, ci, A, xd, mw.r64, bd, partI), s);
        hipLaunchKernelGGL(hz::k_fin_outer, one, B, 0, s, partI, geo.G, mw.outer, outer, max_outer);
        HZ_HIP(hipGetLastError());
        HZ_HIP(hipMemcpyAsync(ho, mw.outer, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
        HZ_HIP(hipStreamSynchronize(s));
        if (ho->done) break;
        // inner complex64 solve of A d = r / ||r|| from d = 0
        hipLaunchKernelGGL(hz::k_demote_scaled, grid1(n), B, 0, s, n, static_cast<const double2*>(mw.r64), mw.outer,
                           mw.b32);
        HZ_HIP(hipMemsetAsync(mw.d32, 0, 8 * size_t(n), s));
        HZ_HIP(hipMemsetAsync(mw.in.ndone, 0, sizeof(int), s));
        hipLaunchKernelGGL(hz::k_sc_init, one, dim3(64), 0, s, mw.in.sc, 1, inner_rtol, maxiter);
        hipLaunchKernelGGL(hz::k_init<float>, dim3(m.G), B, 0, s, ai, static_cast<const float2*>(mw.b32));
        hipLaunchKernelGGL(hz::k_fin_init<float>, one, B, 0, s, ai);
        HZ_HIP(hipGetLastError());
        rc = iterate<float>(h, s, m, ai, L, maxiter, fused);
        if (rc) return rc;
        HZ_HIP(hipMemcpyAsync(hi, mw.in.sc, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
        HZ_HIP(hipStreamSynchronize(s));
        inner_total += hi->iters;
        if (hi->status == HZ_NONFINITE) {
            info->status = HZ_NONFINITE;
            info->iterations = inner_total;
            info->outer_steps = outer + 1;
            return HZ_NONFINITE;
        }
        hipLaunchKernelGGL(hz::k_promote_add, grid1(n), B, 0, s, n, static_cast<const float2*>(mw.d32), dinv32,
                           static_cast<const SolverScal*>(mw.outer), xd);
    }
    if (ho->zero_x) HZ_HIP(hipMemsetAsync(xd, 0, 16 * size_t(n), s));
    HZ_HIP(hipGetLastError());
    HZ_HIP(hipStreamSynchronize(s));
    info->status = ho->status;
    info->iterations = inner_total;
    info->outer_steps = outer;
    info->relres_recursive = ho->relres;
    info->relres_true = ho->relres_true;
    return ho->status;
}

// Enqueue k iterations of the single-system BiCGStab (no poll).
template <typename T>
int launch_iterations(hz_handle* h, hipStream_t s, const WorkMap& m, const hz::BicgArgs<T>& a0, int L, int k,
                      bool fused) {
    const dim3 G(m.G), B(kBlock);
    const hz::BicgArgs<T> a = iteration_args(m, a0, L, fused);
    const bool sub = sub_products<T>(m, L, fused);
    const int family = (fused ? 3 : 4) + (sizeof(T) == 4 ? 10 : 0);
    return launch_chunk(h, s, chunk_key(family, L, k, 0, a), [&](hipStream_t q) {
        with_lanes(L, [&]<int LL, int UU>() {
            for (int i = 0; i < k; ++i) {
                if (fused) {
                    hipLaunchKernelGGL((hz::k_bicg_A<T, LL, UU>), G, B, 0, q, a);
                    hipLaunchKernelGGL((hz::k_bicg_B<T, LL, UU>), G, B, 0, q, a);
                } else {
                    enqueue_gather_light<T, LL, UU>(q, m, a, sub);
                }
                hipLaunchKernelGGL((hz::k_bicg_C<T>), G, B, 0, q, a);
            }
        });
    });
}

// Mixed precision with reliable updates (HZ_RELIABLE): one complex64
// BiCGStab on A D^{-1} y = b / ||b||; whenever its recursive residual has
// fallen by `delta` since the last update, or the inner iteration has ended,
// x += ||b|| D^{-1} y in FP64, r64 = b - A x in FP64, and the complex64
// residual is replaced by r64 / ||b||.  Convergence is decided on r64.  An
// inner iteration that ends without the true residual meeting rtol (an
// inner breakdown, or recursive convergence that the true residual does not
// confirm) restarts from the current r64.  info->outer_steps counts the
// reliable updates, info->iterations the complex64 iterations.
int solve_mixed_reliable(hz_handle* h, hipStream_t s, int n, int nnz, const int* rp, const int* ci, const double2* A,
                         const double2* bd, double2* xd, double rtol, double delta, int maxiter, int max_updates,
                         int flags, char* ws, hz_solve_info* info) {
    const bool jacobi = (flags & HZ_PRECOND_JACOBI) != 0;
    MixedWs mw;
    mixed_layout(n, nnz, jacobi, ws, &mw);
    const int L = pick_lanes(h, rp, ci, n, nnz);
    const Geom geo = geom_for(n, kBlock / L);
    const int row_off[2] = {0, n};
    const WorkMap m = build_map(1, row_off, L);
    int rc = upload_map(s, m, mw.in);
    if (rc) return rc;
    const dim3 one(1), B(kBlock);
    double* partI = mw.in.part + hz::kPartI * bicg_stride(m.G);  // the inner solve's region I
    hipLaunchKernelGGL(hz::k_sc_init, one, dim3(64), 0, s, mw.outer, 1, rtol, max_updates);
    const double2* dinv64 = nullptr;
    if (jacobi) {
        hipLaunchKernelGGL(hz::k_jacobi_diag<double>, grid1(n), B, 0, s, n, rp, ci, A, mw.r64, mw.outer);
        hipLaunchKernelGGL(hz::k_demote_vec, grid1(n), B, 0, s, n, static_cast<const double2*>(mw.r64),
                           static_cast<float2*>(mw.in.dinv));
        dinv64 = mw.r64;
    }
    if (nnz > 0)
        hipLaunchKernelGGL(hz::k_demote_vals, grid1(nnz), B, 0, s, int64_t(nnz), ci, A, dinv64,
                           static_cast<float2*>(mw.in.ahat));
    if (flags & HZ_X0_ZERO) HZ_HIP(hipMemsetAsync(xd, 0, 16 * size_t(n), s));
    hipLaunchKernelGGL(hz::k_dot_part<1>, dim3(geo.G), B, 0, s, n, geo, bd, nullptr, partI);
    hipLaunchKernelGGL(hz::k_fin_bnorm, one, B, 0, s, partI, geo.G, mw.outer);
    // the true residual of the initial iterate and the first decision
    launch_spmv<double, hz::EPI_RESID>(L, spmv_args<double>(n, geo, rp, ci, A, xd, mw.r64, bd, partI), s);
    hipLaunchKernelGGL(hz::k_fin_outer, one, B, 0, s, partI, geo.G, mw.outer, 0, max_updates);
    HZ_HIP(hipGetLastError());
    SolverScal* ho = h->hsc2;
    SolverScal* hi = h->hsc;
    HZ_HIP(hipMemcpyAsync(ho, mw.outer, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    if (ho->bad_diag) return HZ_ERR_INVALID;
    const bool fused = choose_fused(h, n);
    const hz::BicgArgs<float> ai =
        bicg_args<float>(m, rp, ci, static_cast<const float2*>(mw.in.ahat), mw.b32, mw.d32, mw.in);
    const float2* dinv32 = jacobi ? static_cast<const float2*>(mw.in.dinv) : nullptr;

    // (re)start the complex64 iteration from the current r64: y = 0, r = rhat = r64 / ||b||
    auto start_inner = [&]() -> int {
        hipLaunchKernelGGL(hz::k_ru_demote, grid1(n), B, 0, s, n, static_cast<const double2*>(mw.r64),
                           static_cast<const SolverScal*>(mw.outer), ai.r);
        HZ_HIP(hipMemsetAsync(mw.d32, 0, 8 * size_t(n), s));
        HZ_HIP(hipMemsetAsync(mw.in.ndone, 0, sizeof(int), s));
        hipLaunchKernelGGL(hz::k_sc_init, one, dim3(64), 0, s, mw.in.sc, 1, rtol, maxiter);
        hipLaunchKernelGGL(hz::k_init<float>, dim3(m.G), B, 0, s, ai, static_cast<const float2*>(ai.r));
        hipLaunchKernelGGL(hz::k_fin_init<float>, one, B, 0, s, ai);
        HZ_HIP(hipGetLastError());
        return HZ_OK;
    };
    int updates = 0, inner_done_total = 0, launched = 0, poll = 8;
    if (!ho->done) {
        // the inner right-hand side b / ||b|| (its norm, about 1, scales the inner test)
        hipLaunchKernelGGL(hz::k_ru_demote, grid1(n), B, 0, s, n, bd, static_cast<const SolverScal*>(mw.outer),
                           mw.b32);
        rc = start_inner();
        if (rc) return rc;
    }
    double ref = ho->relres;
    while (!ho->done) {
        const int k = std::min(poll, std::max(1, maxiter - launched));
        rc = launch_iterations<float>(h, s, m, ai, L, k, fused);
        if (rc) return rc;
        launched += k;
        HZ_HIP(hipMemcpyAsync(hi, mw.in.sc, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
        HZ_HIP(hipStreamSynchronize(s));
        if (hi->pending && !hi->done) {  // conclude a half-step exit
            with_lanes(L, [&]<int LL, int UU>() {
                hipLaunchKernelGGL((hz::k_bicg_P<float>), dim3(m.G), B, 0, s, ai);
            });
            HZ_HIP(hipMemcpyAsync(hi, mw.in.sc, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
            HZ_HIP(hipStreamSynchronize(s));
        }
        if (poll < 64) poll *= 2;
        const bool inner_end = hi->done != 0;
        if (!(inner_end || hi->relres <= delta * ref || launched >= maxiter)) continue;
        // reliable update: promote y, the FP64 true residual, the decision
        hipLaunchKernelGGL(hz::k_ru_promote, grid1(n), B, 0, s, n, mw.d32, dinv32,
                           static_cast<const SolverScal*>(mw.outer), xd);
        ++updates;
        launch_spmv<double, hz::EPI_RESID>(L, spmv_args<double>(n, geo, rp, ci, A, xd, mw.r64, bd, partI), s);
        hipLaunchKernelGGL(hz::k_fin_outer, one, B, 0, s, partI, geo.G, mw.outer, updates, max_updates);
        HZ_HIP(hipGetLastError());
        HZ_HIP(hipMemcpyAsync(ho, mw.outer, sizeof(SolverScal), hipMemcpyDeviceToHost, s));
        HZ_HIP(hipStreamSynchronize(s));
        if (hi->status == HZ_NONFINITE && inner_end) {
            info->status = HZ_NONFINITE;
            info->iterations = inner_done_total + hi->iters;
            info->outer_steps = updates;
            return HZ_NONFINITE;
        }
        if (ho->done) {
            inner_done_total += inner_end ? hi->iters : hi->iter - 1;
            break;
        }
        if (launched >= maxiter) {
            inner_done_total += inner_end ? hi->iters : hi->iter - 1;
            ho->status = HZ_NOT_CONVERGED;
            break;
        }
        ref = ho->relres;
        if (inner_end) {  // the inner iteration ended without the true residual meeting rtol: restart it
            inner_done_total += hi->iters;
            rc = start_inner();
            if (rc) return rc;
        } else {
            hipLaunchKernelGGL(hz::k_ru_replace, dim3(m.G), B, 0, s, ai, static_cast<const double2*>(mw.r64),
                               static_cast<const SolverScal*>(mw.outer));
            HZ_HIP(hipGetLastError());
        }
    }
    if (ho->zero_x) HZ_HIP(hipMemsetAsync(xd, 0, 16 * size_t(n), s));
    HZ_HIP(hipGetLastError());
    HZ_HIP(hipStreamSynchronize(s));
    info->status = ho->status;
    info->iterations = inner_done_total;
    info->outer_steps = updates;
    info->relres_recursive = ho->relres;
    info->relres_true = ho->relres_true;
    return ho->status;
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
        case HZ_ERR_TOO_LARGE: return "system too large for the static scratch of the allocation-free solve";
        default: return "unknown helmz status";
    }
}

// Slots of the one-launch reductions: 2 kB1MaxGrid words, then the broken
// word; all armed (and synchronised) before the handle is returned.  The
// last block waits at most 2 s of the device's wall clock for the others
// (HZ_B1_WAIT_TICKS overrides the limit in ticks; 0 makes every wait give up
// at once, the failure path, for tests).
static int b1_arm(hz_handle* h) {
    const size_t words = 2 * size_t(hz::kB1MaxGrid);
    HZ_HIP(hipMalloc(reinterpret_cast<void**>(&h->b1.slot), words * sizeof(unsigned long long) + 256));
    h->b1.broken = reinterpret_cast<unsigned*>(h->b1.slot + words);
    int khz = 0;
    HZ_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device));
    h->b1.limit = (khz > 0 ? static_cast<unsigned long long>(khz) : 100000ull) * 2000ull;
    if (const char* e = std::getenv("HZ_B1_WAIT_TICKS")) h->b1.limit = std::strtoull(e, nullptr, 10);
    hipLaunchKernelGGL(hz::k_b1_arm, dim3((words + hz::kB1Block - 1) / hz::kB1Block), dim3(hz::kB1Block), 0, nullptr,
                       h->b1);
    HZ_HIP(hipGetLastError());
    HZ_HIP(hipStreamSynchronize(nullptr));
    return HZ_OK;
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
        hipHostMalloc(reinterpret_cast<void**>(&h->hsc2), sizeof(SolverScal), hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess ||
        hipGetSymbolAddress(&h->scratch_dev, HIP_SYMBOL(scratch)) != hipSuccess || h->scratch_dev == nullptr ||
        b1_arm(h) != HZ_OK) {
        hz_handle_destroy(h);
        return HZ_ERR_HIP;
    }
    *out = h;
    return HZ_OK;
}

int hz_handle_destroy(hz_handle* h) {
    if (h == nullptr) return HZ_OK;
    if (h->part) (void)hipFree(h->part);
    if (h->b1.slot) (void)hipFree(h->b1.slot);
    if (h->dflag) (void)hipFree(h->dflag);
    if (h->dcount) (void)hipFree(h->dcount);
    if (h->hcount) (void)hipHostFree(h->hcount);
    if (h->hflag) (void)hipHostFree(h->hflag);
    if (h->hsc) (void)hipHostFree(h->hsc);
    if (h->hsc2) (void)hipHostFree(h->hsc2);
    for (GraphEntry& g : h->graphs) graph_release(g);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    delete h;
    return HZ_OK;
}

int hz_autotune_set(hz_handle* h, int n, int nnz, const int* rp, const int* ci, int lanes, int form,
                    int form_lanes) {
    if (h == nullptr || n < 0 || nnz < 0) return HZ_ERR_INVALID;
    if (n > 0 && (rp == nullptr || (nnz > 0 && ci == nullptr))) return HZ_ERR_INVALID;
    auto lane_ok = [](int v) { return v == 2 || v == 4 || v == 8 || v == 16 || v == 32 || v == 64; };
    if (!(lanes == 1 || lane_ok(lanes))) return HZ_ERR_INVALID;
    if (form == SP_PIPE) {
        if (!lane_ok(form_lanes)) return HZ_ERR_INVALID;
    } else if (form == SP_TILE) {
        if (form_lanes != hz::kTileLanes) return HZ_ERR_INVALID;
    } else {
        return HZ_ERR_INVALID;
    }
    for (auto it = h->tune.begin(); it != h->tune.end();)
        it = (it->rp == rp && it->ci == ci && it->n == n && it->nnz == nnz) ? h->tune.erase(it) : it + 1;
    h->tune.push_back(TuneEntry{rp, ci, n, nnz, lanes, SpPlan{form, form_lanes}});
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

int hz_autotune_spmv(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci,
                     const hz_c128* vals, const hz_c128* x, hz_c128* y, int* lanes, int* form, int* form_lanes) {
    int rc = spmv_common_checks(h, n, nnz, rp, ci, vals, x, y, sizeof(hz_c128));
    if (rc) return rc;
    if (lanes == nullptr) return HZ_ERR_INVALID;
    *lanes = rule_lanes(n, nnz);
    if (form != nullptr) *form = SP_PIPE;
    if (form_lanes != nullptr) *form_lanes = *lanes;
    if (n == 0) return HZ_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) {
        if (ev[0]) (void)hipEventDestroy(ev[0]);
        return HZ_ERR_HIP;
    }
    const double2* A = reinterpret_cast<const double2*>(vals);
    const double2* xd = reinterpret_cast<const double2*>(x);
    double2* yd = reinterpret_cast<double2*>(y);
    // 2 warm-up and 5 timed launches of one candidate; the faster of two rounds counts
    auto time_it = [&](auto&& launch, float& best) {
        for (int k = 0; k < 2; ++k) launch();
        if (hipEventRecord(ev[0], s) != hipSuccess) rc = HZ_ERR_HIP;
        for (int k = 0; k < 5; ++k) launch();
        float ms = 0.f;
        if (rc == HZ_OK && (hipEventRecord(ev[1], s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                            hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess))
            rc = HZ_ERR_HIP;
        if (rc == HZ_OK && ms < best) best = ms;
    };
    // the solver kernels' lane count, timed on their row product (1 = block tiles)
    constexpr int kNCand = 7;
    constexpr int kCand[kNCand] = {1, 2, 4, 8, 16, 32, 64};
    float best_ms[kNCand];
    for (float& b : best_ms) b = 1e30f;
    rc = HZ_OK;
    for (int round = 0; round < 2 && rc == HZ_OK; ++round)
        for (int c = 0; c < kNCand && rc == HZ_OK; ++c) {
            const int L = kCand[c];
            const auto a = spmv_args<double>(n, geom_for(n, kBlock / L), rp, ci, A, xd, yd, nullptr, nullptr);
            time_it([&] { launch_spmv<double, hz::EPI_NONE>(L, a, s); }, best_ms[c]);
        }
    // the standalone product's plan: pipelined rows at each lane count, and block tiles
    constexpr int kPlans = 7;
    const SpPlan plans[kPlans] = {{SP_PIPE, 2},  {SP_PIPE, 4},  {SP_PIPE, 8}, {SP_PIPE, 16},
                                  {SP_PIPE, 32}, {SP_PIPE, 64}, {SP_TILE, hz::kTileLanes}};
    float plan_ms[kPlans];
    for (float& b : plan_ms) b = 1e30f;
    if (nnz > 0)
        for (int round = 0; round < 2 && rc == HZ_OK; ++round)
            for (int c = 0; c < kPlans && rc == HZ_OK; ++c)
                time_it([&] { launch_sp<double>(plans[c], n, nnz, rp, ci, A, xd, yd, s); }, plan_ms[c]);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (rc) return rc;
    // The rule's choice stands unless a candidate is more than 3 % faster, so
    // that near-ties (timing noise) do not flip the choice from run to run.
    constexpr float kMargin = 0.97f;
    const int rule = rule_lanes(n, nnz);
    int bc = 0;
    for (int c = 1; c < kNCand; ++c)
        if (best_ms[c] < best_ms[bc]) bc = c;
    for (int c = 0; c < kNCand; ++c)
        if (kCand[c] == rule && best_ms[bc] >= kMargin * best_ms[c]) bc = c;
    SpPlan sp{SP_PIPE, rule};
    if (nnz > 0) {
        const SpPlan def = default_sp(n, nnz);
        int bp = 0;
        for (int c = 1; c < kPlans; ++c)
            if (plan_ms[c] < plan_ms[bp]) bp = c;
        for (int c = 0; c < kPlans; ++c)  // the untuned default unless another is more than 3 % faster
            if (plans[c].form == def.form && (def.form == SP_TILE || plans[c].L == def.L) &&
                plan_ms[bp] >= kMargin * plan_ms[c])
                bp = c;
        sp = plans[bp];
    }
    for (auto it = h->tune.begin(); it != h->tune.end();)
        it = (it->rp == rp && it->ci == ci && it->n == n && it->nnz == nnz) ? h->tune.erase(it) : it + 1;
    h->tune.push_back(TuneEntry{rp, ci, n, nnz, kCand[bc], sp});
    *lanes = kCand[bc];
    if (form != nullptr) *form = sp.form;
    if (form_lanes != nullptr) *form_lanes = sp.L;
    return HZ_OK;
}

int csr_zspmv(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci, const hz_c128* vals,
              const hz_c128* x, hz_c128* y) {
    int rc = spmv_common_checks(h, n, nnz, rp, ci, vals, x, y, sizeof(hz_c128));
    if (rc || n == 0) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    standalone_spmv<double>(h, n, nnz, rp, ci, reinterpret_cast<const double2*>(vals),
                            reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), s);
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

int csr_cspmv(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci, const hz_c64* vals,
              const hz_c64* x, hz_c64* y) {
    int rc = spmv_common_checks(h, n, nnz, rp, ci, vals, x, y, sizeof(hz_c64));
    if (rc || n == 0) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    standalone_spmv<float>(h, n, nnz, rp, ci, reinterpret_cast<const float2*>(vals),
                           reinterpret_cast<const float2*>(x), reinterpret_cast<float2*>(y), s);
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

int zdotc(hz_handle* h, hz_stream stream, int n, const hz_c128* x, const hz_c128* y, hz_c128* out) {
    if (h == nullptr || n < 0 || out == nullptr) return HZ_ERR_INVALID;
    if (n > 0 && (x == nullptr || y == nullptr)) return HZ_ERR_INVALID;
    if (misaligned(x, 16) || misaligned(y, 16) || misaligned(out, 16)) return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hz::B1Shape sh = hz::b1_shape(n);
    hipLaunchKernelGGL(hz::k_zdot_s<0>, dim3(sh.G), dim3(hz::kB1Block), 0, s, int64_t(n), sh.per,
                       reinterpret_cast<const double2*>(x), reinterpret_cast<const double2*>(y), h->b1,
                       static_cast<void*>(out));
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

int dznrm2(hz_handle* h, hz_stream stream, int n, const hz_c128* x, double* out) {
    if (h == nullptr || n < 0 || out == nullptr) return HZ_ERR_INVALID;
    if (n > 0 && x == nullptr) return HZ_ERR_INVALID;
    if (misaligned(x, 16) || misaligned(out, 8)) return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hz::B1Shape sh = hz::b1_shape(n);
    hipLaunchKernelGGL(hz::k_zdot_s<1>, dim3(sh.G), dim3(hz::kB1Block), 0, s, int64_t(n), sh.per,
                       reinterpret_cast<const double2*>(x), static_cast<const double2*>(nullptr), h->b1,
                       static_cast<void*>(out));
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
    const hz::B1Shape sh = hz::b1_shape(n);
    hipLaunchKernelGGL(hz::k_zaxpy_s, dim3(sh.G), dim3(hz::kB1Block), 0, s, int64_t(n), sh.per, a,
                       reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y));
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

int hz_stream_read(hz_handle* h, hz_stream stream, const void* buf, size_t bytes, double* out) {
    if (h == nullptr || out == nullptr || bytes % 16 != 0 || (bytes > 0 && buf == nullptr)) return HZ_ERR_INVALID;
    if (misaligned(buf, 16) || misaligned(out, 8)) return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hz::StreamShape sh = hz::stream_shape(int64_t(bytes / 16));
    static_assert(hz::kStreamMaxGrid <= kParts * kMaxGrid, "partials of the stream read fit the handle's buffer");
    hipLaunchKernelGGL(hz::k_stream_read, dim3(sh.G), dim3(hz::kStreamBlock), 0, s, static_cast<const double2*>(buf),
                       int64_t(bytes / 16), sh.per, h->part);
    hipLaunchKernelGGL(hz::k_stream_fin, dim3(1), dim3(hz::kStreamBlock), 0, s, static_cast<const double*>(h->part),
                       sh.G, out);
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

int hz_stream_copy(hz_handle* h, hz_stream stream, const void* src, void* dst, size_t bytes) {
    if (h == nullptr || bytes % 16 != 0) return HZ_ERR_INVALID;
    if (bytes == 0) return HZ_OK;
    if (src == nullptr || dst == nullptr || misaligned(src, 16) || misaligned(dst, 16)) return HZ_ERR_INVALID;
    if (overlap(src, bytes, dst, bytes)) return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hz::StreamShape sh = hz::stream_shape(int64_t(bytes / 16));
    hipLaunchKernelGGL(hz::k_stream_copy, dim3(sh.G), dim3(hz::kStreamBlock), 0, s, static_cast<const double2*>(src),
                       int64_t(bytes / 16), sh.per, static_cast<double2*>(dst));
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

size_t zbicgstab_workspace_bytes(int n, int nnz, int flags) {
    if (n < 0 || nnz < 0) return 0;
    return single_ws_bytes(n, nnz, flags);
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
    if ((flags & HZ_REORDER) && (flags & HZ_NO_REORDER)) return HZ_ERR_INVALID;
    const size_t need = single_ws_bytes(n, nnz, flags);
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (flags & HZ_VALIDATE) {
        rc = validate_csr(h, s, n, nnz, rp, ci);
        if (rc) return rc;
    }
    return solve_single(h, s, n, nnz, rp, ci, reinterpret_cast<const double2*>(vals),
                        reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(x), rtol, maxiter, flags,
                        static_cast<char*>(ws), info);
}

int zbicgstab_solve_async(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci,
                          const hz_c128* vals, const hz_c128* b, hz_c128* x, double rtol, int maxiter, int flags,
                          void* ws, size_t ws_bytes, hz_solve_info* info_dev) {
    if (h == nullptr || info_dev == nullptr || misaligned(info_dev, 8)) return HZ_ERR_INVALID;
    int rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (!(rtol >= 0.0) || maxiter < 0 || n == 0) return HZ_ERR_INVALID;
    if (b == nullptr || x == nullptr || misaligned(b, 16) || misaligned(x, 16) || misaligned(vals, 16))
        return HZ_ERR_INVALID;
    if (overlap(b, 16 * size_t(n), x, 16 * size_t(n))) return HZ_ERR_INVALID;
    if (flags & (HZ_REORDER | HZ_VALIDATE | HZ_RELIABLE)) return HZ_ERR_INVALID;
    const int f = flags | HZ_NO_REORDER;
    const size_t need = single_ws_bytes(n, nnz, f);
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    const int row_off[2] = {0, n};
    hz_solve_info unused;
    return solve_fp64(h, static_cast<hipStream_t>(stream), 1, row_off, nnz, rp, ci,
                      reinterpret_cast<const double2*>(vals), reinterpret_cast<const double2*>(b),
                      reinterpret_cast<double2*>(x), rtol, maxiter, f, static_cast<char*>(ws), &unused, info_dev);
}

size_t zbicgstab_noalloc_max_bytes(void) { return kScratchBytes; }

int zbicgstab_solve_noalloc(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci,
                            const hz_c128* vals, const hz_c128* b, hz_c128* x, double rtol, int maxiter, int flags,
                            hz_solve_info* info_dev) {
    if (h == nullptr || info_dev == nullptr || misaligned(info_dev, 8)) return HZ_ERR_INVALID;
    int rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (!(rtol >= 0.0) || maxiter < 0 || n == 0) return HZ_ERR_INVALID;
    if (b == nullptr || x == nullptr || misaligned(b, 16) || misaligned(x, 16) || misaligned(vals, 16))
        return HZ_ERR_INVALID;
    if (overlap(b, 16 * size_t(n), x, 16 * size_t(n))) return HZ_ERR_INVALID;
    if (flags & (HZ_REORDER | HZ_VALIDATE | HZ_RELIABLE)) return HZ_ERR_INVALID;
    const int f = flags | HZ_NO_REORDER;
    if (single_ws_bytes(n, nnz, f) > kScratchBytes) return HZ_ERR_TOO_LARGE;
    if (h->scratch_dev == nullptr) return HZ_ERR_HIP;
    const int row_off[2] = {0, n};
    hz_solve_info unused;
    return solve_fp64(h, static_cast<hipStream_t>(stream), 1, row_off, nnz, rp, ci,
                      reinterpret_cast<const double2*>(vals), reinterpret_cast<const double2*>(b),
                      reinterpret_cast<double2*>(x), rtol, maxiter, f, static_cast<char*>(h->scratch_dev), &unused,
                      info_dev, true);
}

size_t zbicgstabl_workspace_bytes(int n, int nnz, int ell, int flags) {
    if (n < 0 || nnz < 0 || ell < 1 || ell > hz::kLMax) return 0;
    return lsolve_ws_bytes(n, nnz, ell, flags);
}

int zbicgstabl_solve(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci,
                     const hz_c128* vals, const hz_c128* b, hz_c128* x, int ell, double rtol, int maxcycles,
                     int flags, void* ws, size_t ws_bytes, hz_solve_info* info) {
    if (info) std::memset(info, 0, sizeof(*info));
    if (h == nullptr || info == nullptr) return HZ_ERR_INVALID;
    int rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (!(rtol >= 0.0) || maxcycles < 0 || ell < 1 || ell > hz::kLMax) return HZ_ERR_INVALID;
    if (n == 0) return HZ_OK;
    if (b == nullptr || x == nullptr || misaligned(b, 16) || misaligned(x, 16) || misaligned(vals, 16))
        return HZ_ERR_INVALID;
    if (overlap(b, 16 * size_t(n), x, 16 * size_t(n))) return HZ_ERR_INVALID;
    if ((flags & HZ_REORDER) && (flags & HZ_NO_REORDER)) return HZ_ERR_INVALID;
    if (flags & HZ_RELIABLE) return HZ_ERR_INVALID;  // a flag of the mixed solve only
    const size_t need = lsolve_ws_bytes(n, nnz, ell, flags);
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (flags & HZ_VALIDATE) {
        rc = validate_csr(h, s, n, nnz, rp, ci);
        if (rc) return rc;
    }
    return with_renumbering(h, s, n, nnz, rp, ci, reinterpret_cast<const double2*>(vals),
                            reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(x), flags,
                            static_cast<char*>(ws), info,
                            [&](const int* rp2, const int* ci2, const double2* A2, const double2* b2, double2* x2,
                                char* ws2) {
                                return solve_l(h, s, n, nnz, rp2, ci2, A2, b2, x2, ell, rtol, maxcycles, flags, ws2,
                                               info);
                            });
}

size_t ztfqmr_workspace_bytes(int n, int nnz, int flags) {
    if (n < 0 || nnz < 0) return 0;
    return qsolve_ws_bytes(n, nnz, flags);
}

int ztfqmr_solve(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci, const hz_c128* vals,
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
    if ((flags & HZ_REORDER) && (flags & HZ_NO_REORDER)) return HZ_ERR_INVALID;
    if (flags & HZ_RELIABLE) return HZ_ERR_INVALID;
    const size_t need = qsolve_ws_bytes(n, nnz, flags);
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (flags & HZ_VALIDATE) {
        rc = validate_csr(h, s, n, nnz, rp, ci);
        if (rc) return rc;
    }
    return with_renumbering(h, s, n, nnz, rp, ci, reinterpret_cast<const double2*>(vals),
                            reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(x), flags,
                            static_cast<char*>(ws), info,
                            [&](const int* rp2, const int* ci2, const double2* A2, const double2* b2, double2* x2,
                                char* ws2) {
                                return solve_q(h, s, n, nnz, rp2, ci2, A2, b2, x2, rtol, maxiter, flags, ws2, info);
                            });
}

static int check_row_off(int nsys, const int* row_off, int* n_total) {
    if (nsys < 1 || row_off == nullptr || row_off[0] != 0) return HZ_ERR_INVALID;
    for (int j = 0; j < nsys; ++j)
        if (row_off[j + 1] < row_off[j]) return HZ_ERR_INVALID;
    *n_total = row_off[nsys];
    return HZ_OK;
}

size_t zbicgstab_varbatch_workspace_bytes(int nsys, const int* row_off, int nnz, int flags) {
    int n = 0;
    if (nnz < 0 || check_row_off(nsys, row_off, &n) != HZ_OK) return 0;
    // the lane count (hence the block count) is chosen per call: size for the largest map
    size_t most = 0;
    for (int L = 2; L <= 64; L *= 2) {
        const WorkMap m = build_map(nsys, row_off, L);
        most = std::max(most, ws_layout<double>(n, nnz, (flags & HZ_PRECOND_JACOBI) != 0, nsys, m.G, nullptr, nullptr));
    }
    return most;
}

int zbicgstab_solve_varbatch(hz_handle* h, hz_stream stream, int nsys, const int* row_off, int nnz, const int* rp,
                             const int* ci, const hz_c128* vals, const hz_c128* b, hz_c128* x, double rtol,
                             int maxiter, int flags, void* ws, size_t ws_bytes, hz_solve_info* infos) {
    if (h == nullptr || infos == nullptr || nsys < 1) return HZ_ERR_INVALID;
    std::memset(infos, 0, sizeof(hz_solve_info) * size_t(nsys));
    int n = 0;
    int rc = check_row_off(nsys, row_off, &n);
    if (rc) return rc;
    rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (!(rtol >= 0.0) || maxiter < 0) return HZ_ERR_INVALID;
    if (n == 0) return HZ_OK;
    if (b == nullptr || x == nullptr || misaligned(b, 16) || misaligned(x, 16) || misaligned(vals, 16))
        return HZ_ERR_INVALID;
    if (overlap(b, 16 * size_t(n), x, 16 * size_t(n))) return HZ_ERR_INVALID;
    const size_t need = zbicgstab_varbatch_workspace_bytes(nsys, row_off, nnz, flags);
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (flags & HZ_VALIDATE) {
        rc = validate_csr(h, s, n, nnz, rp, ci);
        if (rc) return rc;
    }
    return solve_fp64(h, s, nsys, row_off, nnz, rp, ci, reinterpret_cast<const double2*>(vals),
                      reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(x), rtol, maxiter, flags,
                      static_cast<char*>(ws), infos);
}

// A batch of more than kSweepGroup systems runs as groups of up to
// kSweepGroup systems of neighbouring diagonal keys (k_m_diag_key), one
// group after another: the group's b, x and value columns, the keys, and
// the group's solve (BL = 16 lanes per row).
struct BatchGroupWs {
    double2* bg;
    double2* xg;
    double2* vg;
    double* key;
    char* solve;
};

static size_t batch_group_layout(int n, int nnz, int flags, char* base, BatchGroupWs* out) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    BatchGroupWs w{};
    w.bg = reinterpret_cast<double2*>(take(sizeof(double2) * size_t(n > 0 ? n : 1) * hz::kSweepGroup));
    w.xg = reinterpret_cast<double2*>(take(sizeof(double2) * size_t(n > 0 ? n : 1) * hz::kSweepGroup));
    w.vg = reinterpret_cast<double2*>(take(sizeof(double2) * size_t(nnz > 0 ? nnz : 1) * hz::kSweepGroup));
    w.key = reinterpret_cast<double*>(take(sizeof(double) * hz::kMultiMax));
    w.solve = take(multi_layout(hz::kSweepGroup, n, nnz, (flags & HZ_PRECOND_JACOBI) != 0, false, nullptr, nullptr));
    if (out) *out = w;
    return off;
}

size_t zbicgstab_batched_workspace_bytes(int nsys, int n, int nnz, int flags) {
    if (nsys < 1 || nsys > hz::kMultiMax || n < 0 || nnz < 0) return 0;
    if (nsys > hz::kSweepGroup) return batch_group_layout(n, nnz, flags, nullptr, nullptr);
    return multi_layout(nsys, n, nnz, (flags & HZ_PRECOND_JACOBI) != 0, false, nullptr, nullptr);
}

int zbicgstab_solve_batched(hz_handle* h, hz_stream stream, int nsys, int n, int nnz, const int* rp, const int* ci,
                            const hz_c128* vals, const hz_c128* b, hz_c128* x, double rtol, int maxiter, int flags,
                            void* ws, size_t ws_bytes, hz_solve_info* infos) {
    if (h == nullptr || infos == nullptr || nsys < 1 || nsys > hz::kMultiMax) return HZ_ERR_INVALID;
    std::memset(infos, 0, sizeof(hz_solve_info) * size_t(nsys));
    int rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (!(rtol >= 0.0) || maxiter < 0) return HZ_ERR_INVALID;
    if (int64_t(n) * nsys >= (int64_t(1) << 31)) return HZ_ERR_INVALID;
    if (n == 0) return HZ_OK;
    if (b == nullptr || x == nullptr || misaligned(b, 16) || misaligned(x, 16) || misaligned(vals, 16))
        return HZ_ERR_INVALID;
    const size_t vb = 16 * size_t(n) * size_t(nsys);
    if (overlap(b, vb, x, vb)) return HZ_ERR_INVALID;
    const size_t need = zbicgstab_batched_workspace_bytes(nsys, n, nnz, flags);
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (flags & HZ_VALIDATE) {
        rc = validate_csr(h, s, n, nnz, rp, ci);
        if (rc) return rc;
    }
    MultiVals mv;
    mv.vals = reinterpret_cast<const double2*>(vals);
    if (nsys <= hz::kSweepGroup)
        return solve_multi(h, s, nsys, n, nnz, rp, ci, mv, reinterpret_cast<const double2*>(b),
                           reinterpret_cast<double2*>(x), rtol, maxiter, flags, static_cast<char*>(ws), infos);
    // Groups of up to kSweepGroup systems in order of their diagonal keys (ties by index): in a frequency sweep
    // that is the order of the wavenumbers, and neighbours need similar iteration counts, so few lanes idle
    // while a group finishes; a group of 16 systems' values (16 nnz * 16 bytes) is read per product instead
    // of all systems' values for as long as the slowest system runs.  Each system still runs its own BiCGStab.
    BatchGroupWs w;
    batch_group_layout(n, nnz, flags, static_cast<char*>(ws), &w);
    hipLaunchKernelGGL(hz::k_m_diag_key, dim3(nsys), dim3(kBlock), 0, s, n, nsys, rp, ci,
                       reinterpret_cast<const double2*>(vals), w.key);
    HZ_HIP(hipGetLastError());
    std::vector<double> key(nsys);
    HZ_HIP(hipMemcpyAsync(key.data(), w.key, sizeof(double) * size_t(nsys), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    for (double& k : key)
        if (!(k == k)) k = HUGE_VAL;  // a NaN key sorts last
    std::vector<int> order(nsys);
    for (int j = 0; j < nsys; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&key](int u, int v) { return key[u] < key[v]; });
    const int ngroups = (nsys + hz::kSweepGroup - 1) / hz::kSweepGroup;
    int worst = HZ_OK;
    for (int g = 0; g < ngroups; ++g) {
        const int j0 = int(int64_t(nsys) * g / ngroups), j1 = int(int64_t(nsys) * (g + 1) / ngroups);
        const int Bg = j1 - j0;
        hz::GroupCols idx{};
        for (int k = 0; k < Bg; ++k) idx.j[k] = order[j0 + k];
        const dim3 grid = grid1(int64_t(n) * Bg);
        hipLaunchKernelGGL(hz::k_m_cols, grid, dim3(kBlock), 0, s, n, nsys, Bg, idx,
                           reinterpret_cast<const double2*>(b), w.bg, 0);
        if (!(flags & HZ_X0_ZERO))
            hipLaunchKernelGGL(hz::k_m_cols, grid, dim3(kBlock), 0, s, n, nsys, Bg, idx,
                               static_cast<const double2*>(reinterpret_cast<double2*>(x)), w.xg, 0);
        if (nnz > 0)  // the group's value columns: entries play the part of rows
            hipLaunchKernelGGL(hz::k_m_cols, grid1(int64_t(nnz) * Bg), dim3(kBlock), 0, s, nnz, nsys, Bg, idx,
                               reinterpret_cast<const double2*>(vals), w.vg, 0);
        HZ_HIP(hipGetLastError());
        MultiVals mg;
        mg.vals = w.vg;
        hz_solve_info gi[hz::kSweepGroup];
        rc = solve_multi(h, s, Bg, n, nnz, rp, ci, mg, w.bg, w.xg, rtol, maxiter, flags & ~HZ_VALIDATE, w.solve, gi);
        if (rc < 0) return rc;
        hipLaunchKernelGGL(hz::k_m_cols, grid, dim3(kBlock), 0, s, n, nsys, Bg, idx, static_cast<const double2*>(w.xg),
                           reinterpret_cast<double2*>(x), 1);
        HZ_HIP(hipGetLastError());
        for (int k = 0; k < Bg; ++k) infos[order[j0 + k]] = gi[k];
        worst = std::max(worst, rc);
    }
    HZ_HIP(hipStreamSynchronize(s));
    return worst;
}

// A sweep of more than kSweepGroup systems runs as groups of up to
// kSweepGroup systems of neighbouring wavenumbers, one group after another:
// each group's solve (BL = 16 lanes per row) and its b and x columns.
size_t sweep_group_bytes(int n, int nnz, int flags) {
    const size_t cols = align_up(sizeof(double2) * size_t(n > 0 ? n : 1) * hz::kSweepGroup);
    return multi_layout(hz::kSweepGroup, n, nnz, (flags & HZ_PRECOND_JACOBI) != 0, true, nullptr, nullptr) +
           2 * cols;
}

size_t zbicgstab_sweep_workspace_bytes(int nsys, int n, int nnz, int flags) {
    if (nsys < 1 || nsys > hz::kMultiMax || n < 0 || nnz < 0) return 0;
    const size_t one = multi_layout(nsys, n, nnz, (flags & HZ_PRECOND_JACOBI) != 0, true, nullptr, nullptr);
    return nsys > hz::kSweepGroup ? std::max(one, sweep_group_bytes(n, nnz, flags)) : one;
}

int zbicgstab_solve_sweep(hz_handle* h, hz_stream stream, int nsys, int n, int nnz, const int* rp, const int* ci,
                          const double* K, const double* M, const double* Bmat, const double* ks, const hz_c128* b,
                          hz_c128* x, double rtol, int maxiter, int flags, void* ws, size_t ws_bytes,
                          hz_solve_info* infos) {
    if (h == nullptr || infos == nullptr || nsys < 1 || nsys > hz::kMultiMax) return HZ_ERR_INVALID;
    std::memset(infos, 0, sizeof(hz_solve_info) * size_t(nsys));
    int rc = check_csr_args(n, nnz, rp, ci, K);
    if (rc) return rc;
    if (!(rtol >= 0.0) || maxiter < 0 || ks == nullptr) return HZ_ERR_INVALID;
    for (int j = 0; j < nsys; ++j)
        if (!std::isfinite(ks[j])) return HZ_ERR_INVALID;
    if (int64_t(n) * nsys >= (int64_t(1) << 31)) return HZ_ERR_INVALID;
    if (n == 0) return HZ_OK;
    if (nnz > 0 && (M == nullptr || Bmat == nullptr || misaligned(K, 8) || misaligned(M, 8) || misaligned(Bmat, 8)))
        return HZ_ERR_INVALID;
    if (b == nullptr || x == nullptr || misaligned(b, 16) || misaligned(x, 16)) return HZ_ERR_INVALID;
    const size_t vb = 16 * size_t(n) * size_t(nsys);
    if (overlap(b, vb, x, vb)) return HZ_ERR_INVALID;
    const size_t need = zbicgstab_sweep_workspace_bytes(nsys, n, nnz, flags);
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (flags & HZ_VALIDATE) {
        rc = validate_csr(h, s, n, nnz, rp, ci);
        if (rc) return rc;
    }
    MultiVals mv;
    mv.K = K;
    mv.M = M;
    mv.Bm = Bmat;
    mv.ks = ks;
    if (nsys <= hz::kSweepGroup)
        return solve_multi(h, s, nsys, n, nnz, rp, ci, mv, reinterpret_cast<const double2*>(b),
                           reinterpret_cast<double2*>(x), rtol, maxiter, flags, static_cast<char*>(ws), infos);
    // Groups of up to kSweepGroup systems in order of wavenumber (ties by index), solved one after another:
    // the systems of a group need similar iteration counts, so few lanes idle while a group finishes, and a
    // group's gathered columns (16 systems x 16 bytes per row) stay in the XCD's L2.  Each system still runs
    // its own BiCGStab; only the launch grouping and the partial-sum trees differ from one wide batch.
    std::vector<int> order(nsys);
    for (int j = 0; j < nsys; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [ks](int u, int v) { return ks[u] < ks[v]; });
    char* base = static_cast<char*>(ws);
    const size_t cols = align_up(sizeof(double2) * size_t(n) * hz::kSweepGroup);
    double2* bg = reinterpret_cast<double2*>(base);
    double2* xg = reinterpret_cast<double2*>(base + cols);
    char* gws = base + 2 * cols;
    const int ngroups = (nsys + hz::kSweepGroup - 1) / hz::kSweepGroup;
    int worst = HZ_OK;
    for (int g = 0; g < ngroups; ++g) {
        // near-equal groups (sizes differ by at most one)
        const int j0 = int(int64_t(nsys) * g / ngroups), j1 = int(int64_t(nsys) * (g + 1) / ngroups);
        const int Bg = j1 - j0;
        hz::GroupCols idx{};
        double kg[hz::kSweepGroup];
        for (int k = 0; k < Bg; ++k) {
            idx.j[k] = order[j0 + k];
            kg[k] = ks[order[j0 + k]];
        }
        const dim3 grid = grid1(int64_t(n) * Bg);
        hipLaunchKernelGGL(hz::k_m_cols, grid, dim3(kBlock), 0, s, n, nsys, Bg, idx,
                           reinterpret_cast<const double2*>(b), bg, 0);
        if (!(flags & HZ_X0_ZERO))
            hipLaunchKernelGGL(hz::k_m_cols, grid, dim3(kBlock), 0, s, n, nsys, Bg, idx,
                               static_cast<const double2*>(reinterpret_cast<double2*>(x)), xg, 0);
        HZ_HIP(hipGetLastError());
        MultiVals mg = mv;
        mg.ks = kg;
        hz_solve_info gi[hz::kSweepGroup];
        rc = solve_multi(h, s, Bg, n, nnz, rp, ci, mg, bg, xg, rtol, maxiter, flags, gws, gi);
        if (rc < 0) return rc;
        hipLaunchKernelGGL(hz::k_m_cols, grid, dim3(kBlock), 0, s, n, nsys, Bg, idx, static_cast<const double2*>(xg),
                           reinterpret_cast<double2*>(x), 1);
        HZ_HIP(hipGetLastError());
        for (int k = 0; k < Bg; ++k) infos[order[j0 + k]] = gi[k];
        worst = std::max(worst, rc);
    }
    HZ_HIP(hipStreamSynchronize(s));
    return worst;
}

size_t zbicgstab_mixed_workspace_bytes(int n, int nnz, int flags) {
    if (n < 0 || nnz < 0) return 0;
    return mixed_ws_bytes(n, nnz, flags);
}

int zbicgstab_solve_mixed(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci,
                          const hz_c128* vals, const hz_c128* b, hz_c128* x, double rtol, double inner_rtol,
                          int maxiter, int max_outer, int flags, void* ws, size_t ws_bytes, hz_solve_info* info) {
    if (info) std::memset(info, 0, sizeof(*info));
    if (h == nullptr || info == nullptr) return HZ_ERR_INVALID;
    int rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (!(rtol >= 0.0) || !(inner_rtol > 0.0) || maxiter < 0 || max_outer < 0) return HZ_ERR_INVALID;
    if ((flags & HZ_RELIABLE) && !(inner_rtol < 1.0)) return HZ_ERR_INVALID;
    if (n == 0) return HZ_OK;
    if (b == nullptr || x == nullptr || misaligned(b, 16) || misaligned(x, 16) || misaligned(vals, 16))
        return HZ_ERR_INVALID;
    if (overlap(b, 16 * size_t(n), x, 16 * size_t(n))) return HZ_ERR_INVALID;
    if ((flags & HZ_REORDER) && (flags & HZ_NO_REORDER)) return HZ_ERR_INVALID;
    const size_t need = mixed_ws_bytes(n, nnz, flags);
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (flags & HZ_VALIDATE) {
        rc = validate_csr(h, s, n, nnz, rp, ci);
        if (rc) return rc;
    }
    const double2* A = reinterpret_cast<const double2*>(vals);
    const double2* bd = reinterpret_cast<const double2*>(b);
    double2* xd = reinterpret_cast<double2*>(x);
    char* w = static_cast<char*>(ws);
    bool re = false;
    rc = want_reorder(h, s, n, nnz, rp, ci, flags, &re);
    if (rc) return rc;
    auto run = [&](const int* rp_, const int* ci_, const double2* A_, const double2* b_, double2* x_, char* w_) {
        return (flags & HZ_RELIABLE)
                   ? solve_mixed_reliable(h, s, n, nnz, rp_, ci_, A_, b_, x_, rtol, inner_rtol, maxiter, max_outer,
                                          flags, w_, info)
                   : solve_mixed(h, s, n, nnz, rp_, ci_, A_, b_, x_, rtol, inner_rtol, maxiter, max_outer, flags, w_,
                                 info);
    };
    if (!re) return run(rp, ci, A, bd, xd, w);
    // P A P^T (P x) = P b in the level-set numbering, then x scattered back
    ReorderWs r;
    const size_t off = reorder_layout(n, nnz, w, &r);
    rc = level_order(h, s, n, rp, ci, r.lv, r.perm, r.inv, nullptr);
    if (rc) return rc;
    rc = permute_csr(s, n, nnz, rp, ci, A, r.perm, r.inv, r.lv, r.rp, r.ci, r.vals);
    if (rc) return rc;
    hipLaunchKernelGGL(hz::k_gather_perm<double>, grid1(n), dim3(kBlock), 0, s, n, r.perm, bd, r.b);
    if (!(flags & HZ_X0_ZERO))
        hipLaunchKernelGGL(hz::k_gather_perm<double>, grid1(n), dim3(kBlock), 0, s, n, r.perm,
                           static_cast<const double2*>(xd), r.x);
    HZ_HIP(hipGetLastError());
    rc = run(r.rp, r.ci, r.vals, r.b, r.x, w + off);
    if (rc < 0) return rc;
    info->renumbered = 1;
    hipLaunchKernelGGL(hz::k_scatter_perm<double>, grid1(n), dim3(kBlock), 0, s, n, r.perm,
                       static_cast<const double2*>(r.x), xd);
    HZ_HIP(hipGetLastError());
    HZ_HIP(hipStreamSynchronize(s));
    return rc;
}



int csr_zspmv_rect(hz_handle* h, hz_stream stream, int m, int ncols, int nnz, const int* rp, const int* ci,
                   const hz_c128* vals, const hz_c128* x, hz_c128* y) {
    if (h == nullptr || m < 0 || ncols < 0) return HZ_ERR_INVALID;
    int rc = check_csr_args(m, nnz, rp, ci, vals);
    if (rc || m == 0) return rc;
    if (y == nullptr || (ncols > 0 && x == nullptr)) return HZ_ERR_INVALID;
    if (ncols == 0 && nnz > 0) return HZ_ERR_INVALID;  // entries need columns
    if (misaligned(x, 16) || misaligned(y, 16) || misaligned(vals, 16)) return HZ_ERR_INVALID;
    if (ncols > 0 && overlap(x, 16 * size_t(ncols), y, 16 * size_t(m))) return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ncols > 0) {
        standalone_spmv<double>(h, m, nnz, rp, ci, reinterpret_cast<const double2*>(vals),
                                reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), s);
    } else {  // no columns, so no entries: y = 0 by the vector rows
        const int L = pick_lanes(h, rp, ci, m, nnz);
        auto a = spmv_args<double>(m, geom_for(m, kBlock / L), rp, ci, reinterpret_cast<const double2*>(vals),
                                   reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), nullptr,
                                   nullptr);
        launch_spmv<double, hz::EPI_NONE>(L, a, s);
    }
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

int csr_zgrad_vals(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci, const hz_c128* lambda,
                   const hz_c128* x, hz_c128* grad_vals) {
    if (h == nullptr) return HZ_ERR_INVALID;
    int rc = check_csr_args(n, nnz, rp, ci, grad_vals);
    if (rc || n == 0 || nnz == 0) return rc;
    if (lambda == nullptr || x == nullptr || misaligned(lambda, 16) || misaligned(x, 16) || misaligned(grad_vals, 16))
        return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    launch_grad_vals(n, rp, ci, reinterpret_cast<const double2*>(lambda), reinterpret_cast<const double2*>(x),
                     reinterpret_cast<double2*>(grad_vals), pick_lanes(h, rp, ci, n, nnz), s);
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

size_t zbicgstab_adjoint_workspace_bytes(int n, int nnz, int flags) {
    if (n < 0 || nnz < 0) return 0;
    return adjoint_layout(n, nnz, flags, nullptr, nullptr);
}

int zbicgstab_adjoint(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci, const hz_c128* vals,
                      const hz_c128* x, const hz_c128* grad_x, hz_c128* grad_b, hz_c128* grad_vals, double rtol,
                      int maxiter, int flags, void* ws, size_t ws_bytes, hz_solve_info* info) {
    if (info) std::memset(info, 0, sizeof(*info));
    if (h == nullptr || info == nullptr) return HZ_ERR_INVALID;
    int rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (!(rtol >= 0.0) || maxiter < 0) return HZ_ERR_INVALID;
    if (n == 0) return HZ_OK;
    if (grad_x == nullptr || grad_b == nullptr || misaligned(grad_x, 16) || misaligned(grad_b, 16) ||
        misaligned(vals, 16))
        return HZ_ERR_INVALID;
    if (grad_vals != nullptr && (x == nullptr || misaligned(x, 16) || misaligned(grad_vals, 16))) return HZ_ERR_INVALID;
    if (overlap(grad_x, 16 * size_t(n), grad_b, 16 * size_t(n))) return HZ_ERR_INVALID;
    if ((flags & HZ_REORDER) && (flags & HZ_NO_REORDER)) return HZ_ERR_INVALID;
    AdjWs a;
    const size_t need = adjoint_layout(n, nnz, flags, static_cast<char*>(ws), &a);
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (flags & HZ_VALIDATE) {
        rc = validate_csr(h, s, n, nnz, rp, ci);
        if (rc) return rc;
    }
    const double2* A = reinterpret_cast<const double2*>(vals);
    const double2* g = reinterpret_cast<const double2*>(grad_x);
    double2* lam = reinterpret_cast<double2*>(grad_b);
    const int sflags = (flags & (HZ_PRECOND_JACOBI | HZ_REORDER | HZ_NO_REORDER)) | HZ_X0_ZERO;
    if (flags & HZ_SYMMETRIC) {
        // A^H lambda = g  <=>  A conj(lambda) = conj(g)  when A = A^T
        hipLaunchKernelGGL(hz::k_conj, grid1(n), dim3(kBlock), 0, s, n, g, a.gconj);
        HZ_HIP(hipGetLastError());
        rc = solve_single(h, s, n, nnz, rp, ci, A, a.gconj, lam, rtol, maxiter, sflags, a.solve, info);
        if (rc < 0) return rc;
        hipLaunchKernelGGL(hz::k_conj, grid1(n), dim3(kBlock), 0, s, n, static_cast<const double2*>(lam), lam);
    } else {
        // A^H in CSR: column counts, scan, scatter, per-row sort
        HZ_HIP(hipMemsetAsync(a.t_rp, 0, sizeof(int) * (size_t(n) + 1), s));
        if (nnz > 0) hipLaunchKernelGGL(hz::k_tr_count, grid1(nnz), dim3(kBlock), 0, s, int64_t(nnz), ci, a.t_rp);
        hipLaunchKernelGGL(hz::k_scan_1block, dim3(1), dim3(1024), 0, s, n + 1, a.t_rp);
        HZ_HIP(hipMemcpyAsync(a.fill, a.t_rp, sizeof(int) * size_t(n), hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(hz::k_tr_scatter, grid1(n), dim3(kBlock), 0, s, n, rp, ci, A, a.fill, a.t_ci, a.t_vals);
        hipLaunchKernelGGL(hz::k_row_sort<double2>, grid1(n), dim3(kBlock), 0, s, n, static_cast<const int*>(a.t_rp), a.t_ci,
                           a.t_vals);
        HZ_HIP(hipGetLastError());
        rc = solve_single(h, s, n, nnz, a.t_rp, a.t_ci, a.t_vals, g, lam, rtol, maxiter, sflags, a.solve, info);
        if (rc < 0) return rc;
    }
    if (grad_vals != nullptr && nnz > 0)
        launch_grad_vals(n, rp, ci, lam, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(grad_vals),
                         pick_lanes(h, rp, ci, n, nnz), s);
    HZ_HIP(hipGetLastError());
    HZ_HIP(hipStreamSynchronize(s));
    return info->status;
}

size_t zbicgstab_adjoint_batched_workspace_bytes(int nsys, int n, int nnz, int flags) {
    if (nsys < 1 || nsys > hz::kMultiMax || n < 0 || nnz < 0) return 0;
    return adjoint_multi_layout(nsys, n, nnz, flags, nullptr, nullptr);
}

int zbicgstab_adjoint_batched(hz_handle* h, hz_stream stream, int nsys, int n, int nnz, const int* rp, const int* ci,
                              const hz_c128* vals, const hz_c128* x, const hz_c128* grad_x, hz_c128* grad_b,
                              hz_c128* grad_vals, double rtol, int maxiter, int flags, void* ws, size_t ws_bytes,
                              hz_solve_info* infos) {
    if (h == nullptr || infos == nullptr || nsys < 1 || nsys > hz::kMultiMax) return HZ_ERR_INVALID;
    std::memset(infos, 0, sizeof(hz_solve_info) * size_t(nsys));
    int rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (!(rtol >= 0.0) || maxiter < 0) return HZ_ERR_INVALID;
    if (int64_t(n) * nsys >= (int64_t(1) << 31)) return HZ_ERR_INVALID;
    if (n == 0) return HZ_OK;
    const size_t vb = 16 * size_t(n) * size_t(nsys);
    if (grad_x == nullptr || grad_b == nullptr || misaligned(grad_x, 16) || misaligned(grad_b, 16) ||
        misaligned(vals, 16))
        return HZ_ERR_INVALID;
    if (grad_vals != nullptr && (x == nullptr || misaligned(x, 16) || misaligned(grad_vals, 16))) return HZ_ERR_INVALID;
    if (overlap(grad_x, vb, grad_b, vb)) return HZ_ERR_INVALID;
    AdjMultiWs a;
    const size_t need = adjoint_multi_layout(nsys, n, nnz, flags, static_cast<char*>(ws), &a);
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (flags & HZ_VALIDATE) {
        rc = validate_csr(h, s, n, nnz, rp, ci);
        if (rc) return rc;
    }
    const double2* A = reinterpret_cast<const double2*>(vals);
    const double2* g = reinterpret_cast<const double2*>(grad_x);
    double2* lam = reinterpret_cast<double2*>(grad_b);
    const int64_t nB = int64_t(n) * nsys;
    const int sflags = (flags & HZ_PRECOND_JACOBI) | HZ_X0_ZERO;
    if (flags & HZ_SYMMETRIC) {
        // A_j^H lambda_j = g_j  <=>  A_j conj(lambda_j) = conj(g_j)  when A_j = A_j^T
        hipLaunchKernelGGL(hz::k_conj, grid1(nB), dim3(kBlock), 0, s, int(nB), g, a.gconj);
        HZ_HIP(hipGetLastError());
        MultiVals mv;
        mv.vals = A;
        rc = solve_multi(h, s, nsys, n, nnz, rp, ci, mv, a.gconj, lam, rtol, maxiter, sflags, a.solve, infos);
        if (rc < 0) return rc;
        hipLaunchKernelGGL(hz::k_conj, grid1(nB), dim3(kBlock), 0, s, int(nB), static_cast<const double2*>(lam), lam);
    } else {
        // transposed pattern with source entries (count, scan, scatter, per-row sort), then conj values per system
        HZ_HIP(hipMemsetAsync(a.t_rp, 0, sizeof(int) * (size_t(n) + 1), s));
        if (nnz > 0) hipLaunchKernelGGL(hz::k_tr_count, grid1(nnz), dim3(kBlock), 0, s, int64_t(nnz), ci, a.t_rp);
        hipLaunchKernelGGL(hz::k_scan_1block, dim3(1), dim3(1024), 0, s, n + 1, a.t_rp);
        HZ_HIP(hipMemcpyAsync(a.fill, a.t_rp, sizeof(int) * size_t(n), hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(hz::k_tr_scatter_idx, grid1(n), dim3(kBlock), 0, s, n, rp, ci, a.fill, a.t_ci, a.t_src);
        hipLaunchKernelGGL(hz::k_row_sort<int>, grid1(n), dim3(kBlock), 0, s, n, static_cast<const int*>(a.t_rp),
                           a.t_ci, a.t_src);
        if (nnz > 0)
            hipLaunchKernelGGL(hz::k_m_conj_vals, grid1(int64_t(nnz) * nsys), dim3(kBlock), 0, s, int64_t(nnz), nsys,
                               static_cast<const int*>(a.t_src), A, a.t_vals);
        HZ_HIP(hipGetLastError());
        MultiVals mv;
        mv.vals = a.t_vals;
        rc = solve_multi(h, s, nsys, n, nnz, a.t_rp, a.t_ci, mv, g, lam, rtol, maxiter, sflags, a.solve, infos);
        if (rc < 0) return rc;
    }
    if (grad_vals != nullptr && nnz > 0) {
        const int BL = multi_lanes(nsys);
        hz::MultiArgs m{};
        m.n = n;
        m.B = nsys;
        m.geo = geom_for(n, kBlock / BL);
        m.row_ptr = rp;
        m.col_idx = ci;
        with_multi(BL, [&]<int BB>() {
            hipLaunchKernelGGL((hz::k_m_grad_vals<BB>), dim3(m.geo.G), dim3(kBlock), 0, s, m,
                               static_cast<const double2*>(lam), reinterpret_cast<const double2*>(x),
                               reinterpret_cast<double2*>(grad_vals));
        });
    }
    HZ_HIP(hipGetLastError());
    HZ_HIP(hipStreamSynchronize(s));
    return rc;
}

// ------------------------------------------------------------------ planned product in the caller's numbering

// A plan: the level-set permutation, its inverse, P A P^T and room for P x,
// then the ordering scratch (used while the plan is built).
struct SpPlanWs {
    int* perm;
    int* inv;
    int* rp;
    int* ci;
    double2* vals;
    double2* xp;
    LevelWs lv;
};

static size_t spplan_layout(int n, int64_t nnz, char* base, SpPlanWs* out) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    const size_t nn = size_t(n > 0 ? n : 1), nz = size_t(nnz > 0 ? nnz : 1);
    SpPlanWs w{};
    w.perm = static_cast<int*>(take(sizeof(int) * nn));
    w.inv = static_cast<int*>(take(sizeof(int) * nn));
    w.rp = static_cast<int*>(take(sizeof(int) * (nn + 1)));
    w.ci = static_cast<int*>(take(sizeof(int) * nz));
    w.vals = static_cast<double2*>(take(sizeof(double2) * nz));
    w.xp = static_cast<double2*>(take(sizeof(double2) * nn));
    off += level_layout(n, base ? base + off : nullptr, &w.lv);
    if (out) *out = w;
    return off;
}

size_t csr_reorder_workspace_bytes(int n, int nnz) {
    if (n < 0 || nnz < 0) return 0;
    return level_layout(n, nullptr, nullptr);
}

size_t csr_zspmv_plan_bytes(int n, int nnz) {
    if (n < 0 || nnz < 0) return 0;
    return spplan_layout(n, nnz, nullptr, nullptr);
}

int csr_zspmv_plan(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci, const hz_c128* vals,
                   void* plan, size_t plan_bytes) {
    if (h == nullptr) return HZ_ERR_INVALID;
    int rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (n == 0) return HZ_OK;
    if (misaligned(vals, 16)) return HZ_ERR_INVALID;
    SpPlanWs w;
    const size_t need = spplan_layout(n, nnz, static_cast<char*>(plan), &w);
    if (plan == nullptr || plan_bytes < need || misaligned(plan, kAlign)) return HZ_ERR_WORKSPACE;
    if (overlap(plan, need, rp, 4 * (size_t(n) + 1)) || overlap(plan, need, ci, 4 * size_t(nnz)) ||
        overlap(plan, need, vals, 16 * size_t(nnz)))
        return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = level_order(h, s, n, rp, ci, w.lv, w.perm, w.inv, nullptr);
    if (rc) return rc;
    rc = permute_csr(s, n, nnz, rp, ci, reinterpret_cast<const double2*>(vals), w.perm, w.inv, w.lv, w.rp, w.ci,
                     w.vals);
    if (rc) return rc;
    HZ_HIP(hipStreamSynchronize(s));
    return HZ_OK;
}

int csr_zspmv_planned(hz_handle* h, hz_stream stream, int n, int nnz, const void* plan, size_t plan_bytes,
                      const hz_c128* x, hz_c128* y) {
    if (h == nullptr || n < 0 || nnz < 0) return HZ_ERR_INVALID;
    if (n == 0) return HZ_OK;
    if (x == nullptr || y == nullptr || misaligned(x, 16) || misaligned(y, 16)) return HZ_ERR_INVALID;
    if (overlap(x, 16 * size_t(n), y, 16 * size_t(n))) return HZ_ERR_INVALID;
    SpPlanWs w;
    const size_t need = spplan_layout(n, nnz, static_cast<char*>(const_cast<void*>(plan)), &w);
    if (plan == nullptr || plan_bytes < need || misaligned(plan, kAlign)) return HZ_ERR_WORKSPACE;
    if (overlap(plan, need, x, 16 * size_t(n)) || overlap(plan, need, y, 16 * size_t(n))) return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (nnz == 0) {
        hipLaunchKernelGGL(k_zero_c128, grid1(n), dim3(kBlock), 0, s, n, reinterpret_cast<double2*>(y));
        HZ_HIP(hipGetLastError());
        return HZ_OK;
    }
    // x into the plan's numbering, then the block-tile product writing row k to y[perm[k]]
    hipLaunchKernelGGL(hz::k_gather_perm<double>, grid1(n), dim3(kBlock), 0, s, n, static_cast<const int*>(w.perm),
                       reinterpret_cast<const double2*>(x), w.xp);
    hz::SpArgs<double> a{n, nnz, geom_sp(n, hz::kTileRows), w.rp, w.ci, w.vals, w.xp, reinterpret_cast<double2*>(y),
                         w.perm};
    if (a.geo.G >= hz::kSpMaxGrid) {
        a.geo.G = hz::kSpTileGrid;
        hipLaunchKernelGGL((hz::k_spmv_tile<double>), dim3(a.geo.G), dim3(hz::kSpBlock), 0, s, a);
    } else {
        hipLaunchKernelGGL((hz::k_spmv_tile1<double>), dim3(a.geo.G), dim3(hz::kSpBlock), 0, s, a);
    }
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

int csr_level_order(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci, int* perm, int* inv,
                    int* level, void* ws, size_t ws_bytes) {
    if (h == nullptr) return HZ_ERR_INVALID;
    int rc = check_csr_args(n, nnz, rp, ci, reinterpret_cast<const void*>(ci));
    if (rc) return rc;
    if (n == 0) return HZ_OK;
    if (perm == nullptr || inv == nullptr || misaligned(perm, 4) || misaligned(inv, 4) || misaligned(level, 4))
        return HZ_ERR_INVALID;
    if (overlap(perm, 4 * size_t(n), inv, 4 * size_t(n))) return HZ_ERR_INVALID;
    LevelWs w;
    const size_t need = level_layout(n, static_cast<char*>(ws), &w);
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = level_order(h, s, n, rp, ci, w, perm, inv, level);
    if (rc) return rc;
    HZ_HIP(hipStreamSynchronize(s));
    return HZ_OK;
}

int csr_zpermute(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci, const hz_c128* vals,
                 const int* perm, const int* inv, int* rp_out, int* ci_out, hz_c128* vals_out, void* ws,
                 size_t ws_bytes) {
    if (h == nullptr) return HZ_ERR_INVALID;
    int rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (n == 0) return HZ_OK;
    if (perm == nullptr || inv == nullptr || rp_out == nullptr || misaligned(perm, 4) || misaligned(inv, 4) ||
        misaligned(rp_out, 4))
        return HZ_ERR_INVALID;
    if (nnz > 0 && (ci_out == nullptr || vals_out == nullptr || misaligned(ci_out, 4) || misaligned(vals, 16) ||
                    misaligned(vals_out, 16)))
        return HZ_ERR_INVALID;
    const size_t rb = 4 * (size_t(n) + 1), cb = 4 * size_t(nnz), vb = 16 * size_t(nnz);
    if (overlap(rp_out, rb, rp, rb) || overlap(rp_out, rb, ci, cb) || overlap(rp_out, rb, vals, vb) ||
        (nnz > 0 && (overlap(ci_out, cb, rp, rb) || overlap(ci_out, cb, ci, cb) || overlap(ci_out, cb, vals, vb) ||
                     overlap(vals_out, vb, rp, rb) || overlap(vals_out, vb, ci, cb) ||
                     overlap(vals_out, vb, vals, vb))))
        return HZ_ERR_INVALID;
    LevelWs w;
    const size_t need = level_layout(n, static_cast<char*>(ws), &w);
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // perm must be a permutation with inverse inv (every index in range)
    HZ_HIP(hipMemsetAsync(h->dflag, 0, sizeof(int), s));
    hipLaunchKernelGGL(hz::k_check_perm, grid1(n), dim3(kBlock), 0, s, n, perm, inv, h->dflag);
    HZ_HIP(hipGetLastError());
    HZ_HIP(hipMemcpyAsync(h->hflag, h->dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    if (*h->hflag) return HZ_ERR_INVALID;
    rc = permute_csr(s, n, nnz, rp, ci, reinterpret_cast<const double2*>(vals), perm, inv, w, rp_out, ci_out,
                     reinterpret_cast<double2*>(vals_out));
    if (rc) return rc;
    HZ_HIP(hipStreamSynchronize(s));
    return HZ_OK;
}


// ------------------------------------------------------------------ storage formats: C-ABI

size_t csr_format_workspace_bytes(int n) {
    if (n < 0) return 0;
    return fmt_layout(n, nullptr, nullptr);
}

int csr_row_stats(hz_handle* h, hz_stream stream, int n, const int* rp, void* ws, size_t ws_bytes, int* max_len,
                  int* hyb_width) {
    if (h == nullptr || n < 0 || max_len == nullptr || hyb_width == nullptr) return HZ_ERR_INVALID;
    *max_len = *hyb_width = 0;
    if (n == 0) return HZ_OK;
    if (rp == nullptr || misaligned(rp, 4)) return HZ_ERR_INVALID;
    FmtWs w;
    const size_t need = fmt_layout(n, static_cast<char*>(ws), &w);
    if (need == 0) return HZ_ERR_HIP;
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(hz::k_fmt_len, fgrid(n), dim3(hz::kFmtBlock), 0, s, n, rp, w.len);
    size_t tb = w.tmp_bytes;
    HZ_HIP(rocprim::radix_sort_keys_desc(w.tmp, tb, static_cast<const unsigned*>(w.len), w.len2, unsigned(n), 0u,
                                         32u, s));
    hipLaunchKernelGGL(hz::k_fmt_stats, dim3(1), dim3(64), 0, s, n, static_cast<const unsigned*>(w.len2), w.out);
    HZ_HIP(hipGetLastError());
    int hv[2];
    HZ_HIP(hipMemcpyAsync(hv, w.out, sizeof(hv), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    *max_len = hv[0];
    *hyb_width = hv[1];
    return HZ_OK;
}

int csr_to_hyb(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci, const hz_c128* vals,
               int K, int* ell_col, hz_c128* ell_val, int coo_cap, int* coo_row, int* coo_col, hz_c128* coo_val,
               void* ws, size_t ws_bytes, int* coo_nnz) {
    if (h == nullptr || coo_nnz == nullptr || K < 0 || coo_cap < 0) return HZ_ERR_INVALID;
    *coo_nnz = 0;
    int rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (n == 0) return HZ_OK;
    if (K > 0 && (ell_col == nullptr || ell_val == nullptr)) return HZ_ERR_INVALID;
    if (misaligned(vals, 16) || misaligned(ell_col, 4) || misaligned(ell_val, 16) || misaligned(coo_row, 4) ||
        misaligned(coo_col, 4) || misaligned(coo_val, 16))
        return HZ_ERR_INVALID;
    FmtWs w;
    const size_t need = fmt_layout(n, static_cast<char*>(ws), &w);
    if (need == 0) return HZ_ERR_HIP;
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = validate_csr(h, s, n, nnz, rp, ci);
    if (rc) return rc;
    hipLaunchKernelGGL(hz::k_hyb_rem, fgrid(int64_t(n) + 1), dim3(hz::kFmtBlock), 0, s, n, rp, K, w.rem);
    size_t tb = w.tmp_bytes;
    HZ_HIP(rocprim::exclusive_scan(w.tmp, tb, static_cast<const int*>(w.rem), w.off, 0, size_t(n) + 1,
                                   rocprim::plus<int>(), s));
    int total = 0;
    HZ_HIP(hipMemcpyAsync(&total, w.off + n, sizeof(int), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    *coo_nnz = total;
    if (total > coo_cap) return HZ_ERR_WORKSPACE;
    if (total > 0 && (coo_row == nullptr || coo_col == nullptr || coo_val == nullptr)) return HZ_ERR_INVALID;
    hipLaunchKernelGGL(hz::k_hyb_fill, fgrid(n), dim3(hz::kFmtBlock), 0, s, n, rp, ci,
                       reinterpret_cast<const double2*>(vals), K, static_cast<const int*>(w.off), ell_col,
                       reinterpret_cast<double2*>(ell_val), coo_row, coo_col, reinterpret_cast<double2*>(coo_val));
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

int hyb_zspmv(hz_handle* h, hz_stream stream, int n, int K, const int* ell_col, const hz_c128* ell_val, int coo_nnz,
              const int* coo_row, const int* coo_col, const hz_c128* coo_val, const hz_c128* x, hz_c128* y) {
    if (h == nullptr || n < 0 || K < 0 || coo_nnz < 0) return HZ_ERR_INVALID;
    if (n == 0) return HZ_OK;
    if (x == nullptr || y == nullptr || misaligned(x, 16) || misaligned(y, 16)) return HZ_ERR_INVALID;
    if (K > 0 && (ell_col == nullptr || ell_val == nullptr)) return HZ_ERR_INVALID;
    if (coo_nnz > 0 && (coo_row == nullptr || coo_col == nullptr || coo_val == nullptr)) return HZ_ERR_INVALID;
    if (misaligned(ell_col, 4) || misaligned(ell_val, 16) || misaligned(coo_row, 4) || misaligned(coo_col, 4) ||
        misaligned(coo_val, 16))
        return HZ_ERR_INVALID;
    if (overlap(x, 16 * size_t(n), y, 16 * size_t(n))) return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int G = fmt_grid(n);
    const auto* ev = reinterpret_cast<const double2*>(ell_val);
    const auto* xv = reinterpret_cast<const double2*>(x);
    auto* yv = reinterpret_cast<double2*>(y);
    static const bool looped = std::getenv("HZ_ELL_LOOP") != nullptr;  // the generic loop for every width
    if (K >= 1 && K <= 8 && !looped)
        hipLaunchKernelGGL((hz::k_ell_spmv_full<8>), dim3(G), dim3(hz::kFmtBlock), 0, s, n, K, G, ell_col, ev, xv, yv);
    else if (K >= 1 && K <= 16 && !looped)
        hipLaunchKernelGGL((hz::k_ell_spmv_full<16>), dim3(G), dim3(hz::kFmtBlock), 0, s, n, K, G, ell_col, ev, xv,
                           yv);
    else
        hipLaunchKernelGGL((hz::k_ell_spmv<4>), dim3(G), dim3(hz::kFmtBlock), 0, s, n, K, G, ell_col, ev, xv, yv);
    if (coo_nnz > 0)
        hipLaunchKernelGGL(hz::k_coo_add, fgrid(coo_nnz), dim3(hz::kFmtBlock), 0, s, coo_nnz, coo_row, coo_col,
                           reinterpret_cast<const double2*>(coo_val), reinterpret_cast<const double2*>(x),
                           reinterpret_cast<double2*>(y));
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

int csr_sell_analyze(hz_handle* h, hz_stream stream, int n, const int* rp, int C, int sigma, int t, int* perm,
                     int64_t* chunk_ptr, void* ws, size_t ws_bytes, int64_t* slots) {
    if (h == nullptr || n < 0 || slots == nullptr || !sell_shape_ok(C, t)) return HZ_ERR_INVALID;
    if (sigma < 1 || (sigma > 1 && sigma % C != 0)) return HZ_ERR_INVALID;
    *slots = 0;
    if (chunk_ptr == nullptr || misaligned(chunk_ptr, 8)) return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n == 0) {
        HZ_HIP(hipMemsetAsync(chunk_ptr, 0, sizeof(int64_t), s));
        return HZ_OK;
    }
    if (rp == nullptr || perm == nullptr || misaligned(rp, 4) || misaligned(perm, 4)) return HZ_ERR_INVALID;
    FmtWs w;
    const size_t need = fmt_layout(n, static_cast<char*>(ws), &w);
    if (need == 0) return HZ_ERR_HIP;
    if (ws == nullptr || ws_bytes < need || misaligned(ws, kAlign)) return HZ_ERR_WORKSPACE;
    const int nch = (n + C - 1) / C;
    if (sigma == 1) {
        hipLaunchKernelGGL(hz::k_iota, fgrid(n), dim3(hz::kFmtBlock), 0, s, n, perm);
    } else {
        hipLaunchKernelGGL(hz::k_sell_keys, fgrid(n), dim3(hz::kFmtBlock), 0, s, n, rp, sigma, w.key, w.idx);
        size_t tb = w.tmp_bytes;
        HZ_HIP(rocprim::radix_sort_pairs(w.tmp, tb, static_cast<const unsigned long long*>(w.key), w.key2,
                                         static_cast<const int*>(w.idx), perm, unsigned(n), 0u, 64u, s));
    }
    long long* cp = reinterpret_cast<long long*>(chunk_ptr);
    hipLaunchKernelGGL(hz::k_sell_widths, fgrid(int64_t(nch) + 1), dim3(hz::kFmtBlock), 0, s, n, nch, C, t, rp,
                       static_cast<const int*>(perm), w.cw);
    size_t tb = w.tmp_bytes;
    HZ_HIP(rocprim::exclusive_scan(w.tmp, tb, static_cast<const long long*>(w.cw), cp, 0LL, size_t(nch) + 1,
                                   rocprim::plus<long long>(), s));
    HZ_HIP(hipGetLastError());
    long long total = 0;
    HZ_HIP(hipMemcpyAsync(&total, cp + nch, sizeof(long long), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    *slots = total;
    return HZ_OK;
}

int csr_to_sell(hz_handle* h, hz_stream stream, int n, int nnz, const int* rp, const int* ci, const hz_c128* vals,
                int C, int t, const int* perm, const int64_t* chunk_ptr, int64_t slots, int* sell_col,
                hz_c128* sell_val) {
    if (h == nullptr || !sell_shape_ok(C, t) || slots < 0) return HZ_ERR_INVALID;
    int rc = check_csr_args(n, nnz, rp, ci, vals);
    if (rc) return rc;
    if (n == 0) return HZ_OK;
    if (perm == nullptr || chunk_ptr == nullptr || misaligned(perm, 4) || misaligned(chunk_ptr, 8) ||
        misaligned(vals, 16))
        return HZ_ERR_INVALID;
    if (slots > 0 && (sell_col == nullptr || sell_val == nullptr || misaligned(sell_col, 4) ||
                      misaligned(sell_val, 16)))
        return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = validate_csr(h, s, n, nnz, rp, ci);
    if (rc) return rc;
    const int nch = (n + C - 1) / C;
    HZ_HIP(hipMemsetAsync(h->dflag, 0, sizeof(int), s));
    hipLaunchKernelGGL(hz::k_sell_fill, fgrid(int64_t(nch) * C), dim3(hz::kFmtBlock), 0, s, n, nch, C, t, rp, ci,
                       reinterpret_cast<const double2*>(vals), perm, reinterpret_cast<const long long*>(chunk_ptr),
                       (long long)slots, sell_col, reinterpret_cast<double2*>(sell_val), h->dflag);
    HZ_HIP(hipGetLastError());
    HZ_HIP(hipMemcpyAsync(h->hflag, h->dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    HZ_HIP(hipStreamSynchronize(s));
    return *h->hflag ? HZ_ERR_INVALID : HZ_OK;
}

int sell_zspmv(hz_handle* h, hz_stream stream, int n, int C, int t, const int* perm, const int64_t* chunk_ptr,
               const int* sell_col, const hz_c128* sell_val, const hz_c128* x, hz_c128* y) {
    if (h == nullptr || n < 0 || !sell_shape_ok(C, t)) return HZ_ERR_INVALID;
    if (n == 0) return HZ_OK;
    if (perm == nullptr || chunk_ptr == nullptr || x == nullptr || y == nullptr) return HZ_ERR_INVALID;
    if (misaligned(perm, 4) || misaligned(chunk_ptr, 8) || misaligned(sell_col, 4) || misaligned(sell_val, 16) ||
        misaligned(x, 16) || misaligned(y, 16))
        return HZ_ERR_INVALID;
    if (overlap(x, 16 * size_t(n), y, 16 * size_t(n))) return HZ_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nch = (n + C - 1) / C;
    const int G = fmt_grid(int64_t(nch) * C * t);
    const auto* cp = reinterpret_cast<const long long*>(chunk_ptr);
    const auto* sv = reinterpret_cast<const double2*>(sell_val);
    const auto* xv = reinterpret_cast<const double2*>(x);
    auto* yv = reinterpret_cast<double2*>(y);
    switch (t) {
        case 1:
            hipLaunchKernelGGL((hz::k_sell_spmv<1, 4>), dim3(G), dim3(hz::kFmtBlock), 0, s, n, nch, C, G, perm, cp,
                               sell_col, sv, xv, yv);
            break;
        case 2:
            hipLaunchKernelGGL((hz::k_sell_spmv<2, 4>), dim3(G), dim3(hz::kFmtBlock), 0, s, n, nch, C, G, perm, cp,
                               sell_col, sv, xv, yv);
            break;
        case 4:
            hipLaunchKernelGGL((hz::k_sell_spmv<4, 4>), dim3(G), dim3(hz::kFmtBlock), 0, s, n, nch, C, G, perm, cp,
                               sell_col, sv, xv, yv);
            break;
        default:
            hipLaunchKernelGGL((hz::k_sell_spmv<8, 4>), dim3(G), dim3(hz::kFmtBlock), 0, s, n, nch, C, G, perm, cp,
                               sell_col, sv, xv, yv);
            break;
    }
    HZ_HIP(hipGetLastError());
    return HZ_OK;
}

}  // extern "C"
