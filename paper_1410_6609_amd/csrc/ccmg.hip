// Host side of the cell-centered multigrid Poisson solver: hierarchy set-up,
// workspace carving, cycle driver and the C ABI declared in include/ccmg.h.
//
// Design (MI355X): all level arrays live in one caller-owned workspace; every
// smoother pass reads one buffer and writes the other (ping-pong), so a pass
// can fuse several red-black half-sweeps with the residual, the restriction or
// the prolongation without racing against neighbouring tiles.  The V-cycle of
// Sec. 3 / Sec. 5.3 becomes, per level: one or two fused pre-smoothing passes
// (the last one also restricts the residual), the coarsest-grid CG, and one or
// two fused post-smoothing passes (the first one adds the magnified coarse
// correction on the fly, the finest-level last one also reduces the residual
// norm).  Cycles are enqueued in batches; a device-side flag set by the norm
// reduction makes the remaining kernels of a batch return at once, so the
// host reads the control block once per batch instead of once per cycle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ccmg.h"
#include "ccmg_kernels.hpp"

using namespace ccmg;

namespace {

// tile shape of the smoother pass: 64 cells along x (32 lanes x 2), M rows per
// thread, two row strips per wave, WY waves
#ifndef CCMG_ROWS
#define CCMG_ROWS 2
#endif
#ifndef CCMG_WAVES
#define CCMG_WAVES 8
#endif
// FP32 passes hold half the registers and LDS per strip: 16-wave blocks
// (64-row tiles, less halo) fit; FP64 passes keep 8 waves
#ifndef CCMG_WAVES_F32
#define CCMG_WAVES_F32 16
#endif
// Scale of the block capacity that the z-chunk choice assumes, and the chunk
// length from which the FP64 passes march whole unrolled blocks: both only
// move work between blocks and code paths (a second build varies them to test
// that the iterates do not depend on the decomposition)
#ifndef CCMG_CHUNK_CAPACITY_SCALE
#define CCMG_CHUNK_CAPACITY_SCALE 1
#endif
#ifndef CCMG_PAD_MIN_PLANES
#define CCMG_PAD_MIN_PLANES 64
#endif
constexpr int kM = CCMG_ROWS;
constexpr int kWY = CCMG_WAVES;
// waves (strip pairs) per block of the smoother passes, per storage type
template <typename T>
constexpr int kWYof = sizeof(T) == 4 ? CCMG_WAVES_F32 : CCMG_WAVES;

struct LevelBuf {
    int nx = 0, ny = 0, nz = 0;
    size_t n = 0;
    double* phi = nullptr;   // FP64 home buffer (level 0: the caller's phi)
    double* tmp = nullptr;   // FP64 ping-pong partner
    double* b = nullptr;     // FP64 b-tilde
    float* phi32 = nullptr;  // FP32 hierarchy (FP32-IR)
    float* tmp32 = nullptr;
    float* b32 = nullptr;
};

struct Grid {
    int tiles_x, tiles_y, zchunks, zc;
    int blocks() const { return tiles_x * tiles_y * zchunks; }
};

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// Tile-and-chunk decomposition of one pass with S stages over an nx*ny*nz
// level.  A block owning zc planes marches zc + 2S steps (the z halo costs
// 2S), and blocks run in rounds of `capacity` (CUs x resident blocks per CU).
// The chunking minimises rounds x (zc + 2S): long chunks on large levels,
// short ones (more blocks, fewer sequential steps) on small, latency-bound
// levels.
Grid pass_grid(int nx, int ny, int nz, int tx, int ty, int S, int capacity)
{
    Grid g;
    g.tiles_x = cdiv(nx, tx);
    g.tiles_y = cdiv(ny, ty);
    const int xy = g.tiles_x * g.tiles_y;
    // one chunk per tile that already fills most of the machine in one round:
    // the level is large and bandwidth-bound, and shorter chunks would only
    // add z-halo planes (the step count below would prefer, e.g., 8 chunks in
    // 7 rounds to 220 blocks in one for 512^3, and run 11 % slower)
    if (5 * xy >= 4 * capacity && xy <= capacity) {
        g.zc = nz + (nz & 1);
        g.zchunks = 1;
        return g;
    }
    long best = -1;
    int best_zc = nz + (nz & 1);
    for (int chunks = 1; chunks <= (nz + 1) / 2; ++chunks) {
        int zc = cdiv(nz, chunks);
        zc += zc & 1;
        const int nch = cdiv(nz, zc);
        if (nch != chunks) continue;   // same zc as a smaller chunk count
        const long blocks = (long)xy * nch;
        const long rounds = (blocks + capacity - 1) / capacity;
        const long cost = rounds * (zc + 2 * S);
        if (best < 0 || cost < best) { best = cost; best_zc = zc; }
    }
    g.zc = best_zc;
    g.zchunks = cdiv(nz, best_zc);
    return g;
}

// Upper bound of the blocks of any pass over a level: the largest halo
// (S = 5 stages: two fused sweeps and a residual stage, H = 6) gives the
// smallest tiles, and chunks hold at least two planes.
constexpr int kMaxHalo = 6;
int max_pass_blocks(int nx, int ny, int nz)
{
    const int wy = CCMG_WAVES < CCMG_WAVES_F32 ? CCMG_WAVES : CCMG_WAVES_F32;
    return cdiv(nx, 64 - 2 * kMaxHalo) * cdiv(ny, 2 * wy * CCMG_ROWS - 2 * kMaxHalo) * cdiv(nz, 2);
}

}  // namespace

struct ccmg_solver {
    int nx, ny, nz;
    double h;
    ccmg_face bc[6];
    int sh[6];
    bool periodic = false;       // some axis is periodic
    ccmg_options opt;
    hipStream_t stream = nullptr;
    int L = 0;
    LevelBuf lv[CCMG_MAX_LEVELS];
    int cg_maxit = 0;
    int lb = -1;   // first level of the single-workgroup bottom, or -1
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    size_t need_bytes = 0;
    Ctl* ctl = nullptr;
    double* partials = nullptr;
    int max_partials = 0;
    // Poisson-Boltzmann: kappa^2, the chord constant of the nonlinear iteration
    // (1 for the linear operator), and the nonlinear residual and correction
    double kappa2 = 0.0;
    double pb_c = 1.0;
    double* pb_r = nullptr;
    double* pb_d = nullptr;
    double* face_vals[6] = {};   // per-cell boundary values (workspace)
    bool face_on[6] = {};        // face uses face_vals instead of bc[].value
    // variable permittivity: stored face coefficients per level (workspace)
    double* vkx[CCMG_MAX_LEVELS] = {};
    double* vky[CCMG_MAX_LEVELS] = {};
    double* vkz[CCMG_MAX_LEVELS] = {};
    bool vc_on = false;
    // kernel timing (ccmg_profile_*)
    bool prof = false;
    struct ProfRec { int cycle, which; hipEvent_t a, b; };
    std::vector<ProfRec> prof_recs;
    std::vector<hipEvent_t> prof_pool;
    double prof_ms[8] = {0};
    int prof_n[8] = {0};
    // host mirrors
    std::vector<char> ctl_host;
    std::vector<double> hist;
    int last_cycles = 0;
    std::string err;
};

namespace {

std::string g_create_err;

int fail(ccmg_solver* s, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) s->err = buf; else g_create_err = buf;
    return code;
}

#define HIPCHK(s, call)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return fail((s), CCMG_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define LAUNCHCHK(s)                                                                       \
    do {                                                                                   \
        hipError_t e_ = hipGetLastError();                                                 \
        if (e_ != hipSuccess) return fail((s), CCMG_E_HIP, "kernel launch: %s", hipGetErrorString(e_)); \
    } while (0)

bool is_device_ptr(const void* p)
{
    if (p == nullptr) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// pass dispatch: only the (stages, load, residual) combinations the driver
// uses are instantiated
// ---------------------------------------------------------------------------
int g_num_cus = 256;   // set from the device at workspace attachment
constexpr size_t kBottomMaxLds = 160 * 1024;
constexpr int kPadMinPlanes = CCMG_PAD_MIN_PLANES;   // z-chunks from which FP64 passes march whole unrolled blocks
constexpr int kFoldMaxBlocks = 4096;   // grid of the fold (grid-stride over x-rows)

template <typename T, int SPHI, int LOAD, int RES>
bool launch_one(const PassParams<T>& P0, hipStream_t st)
{
    constexpr int WYT = kWYof<T>;
    using Sh = PassShape<T, SPHI, RES, kM, WYT, LOAD>;
    auto kern = k_pass<T, SPHI, LOAD, RES, kM, WYT>;
    static int per_cu = 0;
    if (per_cu == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(kern), 64 * WYT, 0) !=
                hipSuccess || nb < 1) {
            (void)hipGetLastError();
            nb = 1;
        }
        per_cu = nb;
    }
    static_assert(Sh::H <= kMaxHalo, "halo larger than the partials bound assumes");
    PassParams<T> P = P0;
    const Grid g = pass_grid(P.nx, P.ny, P.nz, Sh::TX, Sh::TY, Sh::S, g_num_cus * per_cu * CCMG_CHUNK_CAPACITY_SCALE);
    P.tiles_x = g.tiles_x;
    P.tiles_y = g.tiles_y;
    P.zchunks = g.zchunks;
    P.zc = g.zc;
    // the norm reduction stores one partial per block, then one workgroup adds them
    constexpr bool kNormRes = RES == RES_NORM || RES == RES_NORM_R32 || RES == RES_STORE;
    if (kNormRes && g.blocks() > P.max_partials) return false;
    // long FP64 marches run whole unrolled blocks of steps (k_pass PAD)
    constexpr bool kPadKernel = sizeof(T) == 8 && SPHI > 0;
    if (kPadKernel && g.zc >= kPadMinPlanes)
        hipLaunchKernelGGL((k_pass<T, SPHI, LOAD, RES, kM, WYT, kPadKernel>), dim3(g.blocks()), dim3(64 * WYT), 0, st, P);
    else
        hipLaunchKernelGGL(kern, dim3(g.blocks()), dim3(64 * WYT), 0, st, P);
    if constexpr (kNormRes)
        hipLaunchKernelGGL(k_finish_norm<64 * WYT>, dim3(1), dim3(64 * WYT), 0, st, (const double*)P.partials,
                           g.blocks(), P.ctl, P.fin, P.cycle, 1);
    return true;
}

template <typename T, int SPHI>
bool dispatch_sphi(int load, int res, const PassParams<T>& P, hipStream_t st)
{
    // the V-cycle uses: pre-smoothing from phi or zero (last pass restricts),
    // post-smoothing from phi with or without the prolongation (the finest
    // level's last pass reduces the norm; FP32 levels never do)
    constexpr bool kNorm = sizeof(T) == 8;
    switch (load) {
    case LOAD_PHI:
        if (res == RES_NONE) return launch_one<T, SPHI, LOAD_PHI, RES_NONE>(P, st);
        if (res == RES_RESTRICT) return launch_one<T, SPHI, LOAD_PHI, RES_RESTRICT>(P, st);
        if constexpr (kNorm)
            if (res == RES_NORM) return launch_one<T, SPHI, LOAD_PHI, RES_NORM>(P, st);
        return false;
    case LOAD_ZERO:
        if (res == RES_NONE) return launch_one<T, SPHI, LOAD_ZERO, RES_NONE>(P, st);
        if (res == RES_RESTRICT) return launch_one<T, SPHI, LOAD_ZERO, RES_RESTRICT>(P, st);
        return false;
    case LOAD_PROLONG:
        if (res == RES_NONE) return launch_one<T, SPHI, LOAD_PROLONG, RES_NONE>(P, st);
        if constexpr (kNorm)
            if (res == RES_NORM) return launch_one<T, SPHI, LOAD_PROLONG, RES_NORM>(P, st);
        return false;
    default: return false;
    }
}

template <typename T>
bool dispatch(int sphi, int load, int res, const PassParams<T>& P, hipStream_t st);

template <>
bool dispatch<double>(int sphi, int load, int res, const PassParams<double>& P, hipStream_t st)
{
    if (sphi == 0) {
        if (load == LOAD_PHI && res == RES_NORM) { return launch_one<double, 0, LOAD_PHI, RES_NORM>(P, st); }
        if (load == LOAD_PHI && res == RES_STORE) { return launch_one<double, 0, LOAD_PHI, RES_STORE>(P, st); }
        if (load == LOAD_PHI && res == RES_NORM_R32) { return launch_one<double, 0, LOAD_PHI, RES_NORM_R32>(P, st); }
        if (load == LOAD_CORR && res == RES_NORM_R32) { return launch_one<double, 0, LOAD_CORR, RES_NORM_R32>(P, st); }
        return false;
    }
    if (sphi == 2) return dispatch_sphi<double, 2>(load, res, P, st);
    if (sphi == 4) return dispatch_sphi<double, 4>(load, res, P, st);
    return false;
}

template <>
bool dispatch<float>(int sphi, int load, int res, const PassParams<float>& P, hipStream_t st)
{
    if (sphi == 2) return dispatch_sphi<float, 2>(load, res, P, st);
    if (sphi == 4) return dispatch_sphi<float, 4>(load, res, P, st);
    return false;
}

template <typename T>
void launch_cg(const T* b, T* x, int nx, int ny, int nz, const int* sh, double shift, double rtol, int maxit,
               Ctl* ctl, hipStream_t st)
{
    const int n = nx * ny * nz;
    if (n <= kCgWaveMax) {
        const size_t lds = (size_t)(nx + 2) * (ny + 2) * (nz + 2) * sizeof(double);
        hipLaunchKernelGGL((k_coarse_cg_wave<T>), dim3(1), dim3(64), lds, st, b, x, nx, ny, nz, sh[0], sh[1], sh[2],
                           sh[3], sh[4], sh[5], shift, rtol, maxit, ctl);
        return;
    }
    const int npt = cdiv(n, kCgThreads);
#define CG_CASE(N)                                                                                          \
    hipLaunchKernelGGL((k_coarse_cg<T, N>), dim3(1), dim3(kCgThreads), 0, st, b, x, nx, ny, nz, sh[0], sh[1], \
                       sh[2], sh[3], sh[4], sh[5], shift, rtol, maxit, ctl)
    if (npt <= 1) CG_CASE(1);
    else if (npt <= 2) CG_CASE(2);
    else if (npt <= 4) CG_CASE(4);
    else if (npt <= 8) CG_CASE(8);
    else CG_CASE(16);
#undef CG_CASE
}

int grid1d(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 8192); }

// ---------------------------------------------------------------------------
// one level's kernel list: pre-smoothing passes (last one restricts), then
// post-smoothing passes (first one prolongates), with ping-pong buffers
// ---------------------------------------------------------------------------
struct PassSpec {
    int sphi;   // half-sweeps in this pass
    int load;
    int res;
};

std::vector<PassSpec> level_passes(int nu1, int nu2, int fuse, bool first_zero, int post_last_res)
{
    std::vector<PassSpec> v;
    int left = nu1;
    bool first = true;
    while (left > 0) {
        const int k = std::min(fuse, left);
        left -= k;
        v.push_back({2 * k, first ? (first_zero ? LOAD_ZERO : LOAD_PHI) : LOAD_PHI, left == 0 ? RES_RESTRICT : RES_NONE});
        first = false;
    }
    left = nu2;
    first = true;
    while (left > 0) {
        const int k = std::min(fuse, left);
        left -= k;
        v.push_back({2 * k, first ? LOAD_PROLONG : LOAD_PHI, left == 0 ? post_last_res : RES_NONE});
        first = false;
    }
    return v;
}

// Destination buffer of every pass of a level so that the level ends in its
// home buffer.  Returns true if a final copy tmp -> home is needed.
bool assign_dst(int nk, bool first_src_is_home, std::vector<int>& dst_is_home)
{
    dst_is_home.assign(nk, 0);
    if (!first_src_is_home || nk % 2 == 0) {
        for (int i = nk - 1, h = 1; i >= 0; --i, h ^= 1) dst_is_home[i] = h;
        return false;
    }
    for (int i = 0, h = 0; i < nk; ++i, h ^= 1) dst_is_home[i] = h;
    return true;
}

template <typename T>
struct LevelPtrs {
    T* home[CCMG_MAX_LEVELS];
    T* tmp[CCMG_MAX_LEVELS];
    T* b[CCMG_MAX_LEVELS];
};

// Diagonal shift of level l in the integer-stencil form (Poisson-Boltzmann):
// the level operator is s_l (S_l + shift) with s_l = 1/(2^l h^2), and the
// reaction term of level l is 2^l c kappa^2 (c: chord constant), so
// shift = 2^l c kappa^2 / s_l = 4^l h^2 c kappa^2: kappa^2 times the square of
// the level's spacing, the operator rediscretised there.
double level_shift(const ccmg_solver* s, int l)
{
    return s->kappa2 > 0.0 ? std::ldexp(s->kappa2 * s->pb_c * s->h * s->h, 2 * l) : 0.0;
}

template <typename T>
PassParams<T> base_params(const ccmg_solver* s, int l)
{
    PassParams<T> P;
    std::memset(&P, 0, sizeof P);
    P.nx = s->lv[l].nx;
    P.ny = s->lv[l].ny;
    P.nz = s->lv[l].nz;
    for (int f = 0; f < 6; ++f) P.sh[f] = s->sh[f];
    P.ctl = s->ctl;
    P.partials = s->partials;
    P.max_partials = s->max_partials;
    P.omega = (T)s->opt.omega;
    P.shift = (T)level_shift(s, l);
    return P;
}

// Event bracketing of finest-level passes (only for FP64 cycles that report a
// norm, i.e. cycles of a solve).  Returns the record index or -1.
int prof_begin(ccmg_solver* s, int l, int cycle, int which)
{
    if (!s->prof || l != 0 || cycle <= 0 || which >= 8) return -1;
    hipEvent_t ev[2];
    for (int i = 0; i < 2; ++i) {
        if (s->prof_pool.empty()) {
            if (hipEventCreate(&ev[i]) != hipSuccess) return -1;
        } else {
            ev[i] = s->prof_pool.back();
            s->prof_pool.pop_back();
        }
    }
    if (hipEventRecord(ev[0], s->stream) != hipSuccess) return -1;
    s->prof_recs.push_back({cycle, which, ev[0], ev[1]});
    return (int)s->prof_recs.size() - 1;
}

void prof_end(ccmg_solver* s, int idx)
{
    if (idx < 0) return;
    (void)hipEventRecord(s->prof_recs[idx].b, s->stream);
}

// After a synchronised solve: accumulate the passes of cycles 1..cycles.
void prof_collect(ccmg_solver* s, int cycles)
{
    for (auto& r : s->prof_recs) {
        float ms = 0.f;
        if (r.cycle <= cycles && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            s->prof_ms[r.which] += ms;
            s->prof_n[r.which] += 1;
        }
        s->prof_pool.push_back(r.a);
        s->prof_pool.push_back(r.b);
    }
    s->prof_recs.clear();
}

// Enqueue one V-cycle over levels l0..L-1 of the hierarchy `H` (type T).
// Level l0 starts from its home buffer (or from zero if l0_zero) and ends in
// it.  If fin_cycle > 0, the last pass of level l0 reduces the residual norm
// and finalises cycle `fin_cycle`.
template <typename T>
int enqueue_vcycle(ccmg_solver* s, const LevelPtrs<T>& H, bool l0_zero, int fin_cycle)
{
    const int L = s->L;
    const int fuse = s->opt.fuse_sweeps;
    hipStream_t st = s->stream;
    // descend
    struct Pending { std::vector<PassSpec> ps; std::vector<int> dh; bool copy; size_t next; };
    Pending pend[CCMG_MAX_LEVELS];
    // levels [lbot, L) are handled by the single-workgroup bottom kernel (if any)
    const int lbot = s->lb > 0 ? s->lb : L - 1;
    for (int l = 0; l < lbot; ++l) {
        const bool zero = (l > 0) || l0_zero;
        const int post_res = (l == 0 && fin_cycle > 0) ? RES_NORM : RES_NONE;
        pend[l].ps = level_passes(s->opt.nu1, s->opt.nu2, fuse, zero, post_res);
        pend[l].copy = assign_dst((int)pend[l].ps.size(), !zero, pend[l].dh);
        pend[l].next = 0;
        // pre-smoothing passes
        T* cur = zero ? nullptr : H.home[l];
        for (size_t i = 0; i < pend[l].ps.size(); ++i) {
            const PassSpec& p = pend[l].ps[i];
            if (p.load == LOAD_PROLONG) break;
            PassParams<T> P = base_params<T>(s, l);
            P.phi_in = cur;
            P.b = H.b[l];
            P.phi_out = pend[l].dh[i] ? H.home[l] : H.tmp[l];
            P.bc_out = H.b[l + 1];
            const int pi = prof_begin(s, l, fin_cycle, (int)i);
            if (!dispatch<T>(p.sphi, p.load, p.res, P, st))
                return fail(s, CCMG_E_ARG, "unsupported smoother pass (%d,%d,%d)", p.sphi, p.load, p.res);
            prof_end(s, pi);
            cur = P.phi_out;
            pend[l].next = i + 1;
        }
    }
    if (lbot < L - 1) {
        BottomParams<T> B;
        std::memset(&B, 0, sizeof B);
        B.b_in = H.b[lbot];
        B.phi_out = H.home[lbot];
        B.nlev = L - lbot;
        for (int i = 0; i < B.nlev; ++i) {
            B.nx[i] = s->lv[lbot + i].nx;
            B.ny[i] = s->lv[lbot + i].ny;
            B.nz[i] = s->lv[lbot + i].nz;
        }
        for (int f = 0; f < 6; ++f) B.sh[f] = s->sh[f];
        for (int i = 0; i < B.nlev; ++i) B.shift[i] = level_shift(s, lbot + i);
        B.omega = (T)s->opt.omega;
        B.nu1 = s->opt.nu1;
        B.nu2 = s->opt.nu2;
        B.cg_rtol = sizeof(T) == 4 ? s->opt.ir_cg_rtol : s->opt.cg_rtol;   // the FP32 cycles' own tolerance
        B.cg_maxit = s->cg_maxit;
        B.ctl = s->ctl;
        int nphi = 0, nb = 0;
        bottom_layout(B, nphi, nb);
        const int lc = B.nlev - 1;
        const size_t npl = (size_t)(B.nx[lc] + 2) * (B.ny[lc] + 2) * (B.nz[lc] + 2);
        const size_t lds = (((size_t)(nphi + nb) * sizeof(T) + 7) & ~(size_t)7) + npl * sizeof(double);
        if (lds > kBottomMaxLds) return fail(s, CCMG_E_ARG, "internal: bottom levels need %zu bytes of LDS", lds);
        hipLaunchKernelGGL((k_bottom<T>), dim3(1), dim3(kBottomThreads), lds, st, B);
    } else {
        // coarsest level alone
        const int l = L - 1;
        const LevelBuf& B = s->lv[l];
        launch_cg<T>(H.b[l], H.home[l], B.nx, B.ny, B.nz, s->sh, level_shift(s, l),
                     sizeof(T) == 4 ? s->opt.ir_cg_rtol : s->opt.cg_rtol,
                     s->cg_maxit, s->ctl, st);
    }
    // ascend
    for (int l = lbot - 1; l >= 0; --l) {
        Pending& pd = pend[l];
        T* cur = (pd.next > 0) ? (pd.dh[pd.next - 1] ? H.home[l] : H.tmp[l]) : H.home[l];
        for (size_t i = pd.next; i < pd.ps.size(); ++i) {
            const PassSpec& p = pd.ps[i];
            PassParams<T> P = base_params<T>(s, l);
            P.phi_in = cur;
            P.b = H.b[l];
            P.ec = H.home[l + 1];
            P.phi_out = pd.dh[i] ? H.home[l] : H.tmp[l];
            if (p.res == RES_NORM) {
                P.fin = FIN_CYCLE;
                P.cycle = fin_cycle;
            }
            const int pi = prof_begin(s, l, fin_cycle, (int)i);
            if (!dispatch<T>(p.sphi, p.load, p.res, P, st))
                return fail(s, CCMG_E_ARG, "unsupported smoother pass (%d,%d,%d)", p.sphi, p.load, p.res);
            prof_end(s, pi);
            cur = P.phi_out;
        }
        if (pd.copy) {
            const size_t n = s->lv[l].n;
            // level 0: the norm pass of this cycle may just have set `done`, so this copy always runs
            hipLaunchKernelGGL((k_copy<T>), dim3(grid1d(n)), dim3(256), 0, st, (const T*)H.tmp[l], H.home[l], n,
                               l == 0 ? (const Ctl*)nullptr : (const Ctl*)s->ctl);
        }
    }
    LAUNCHCHK(s);
    return CCMG_OK;
}

LevelPtrs<double> fp64_ptrs(ccmg_solver* s, double* phi0)
{
    LevelPtrs<double> H;
    for (int l = 0; l < s->L; ++l) {
        H.home[l] = l == 0 ? phi0 : s->lv[l].phi;
        H.tmp[l] = s->lv[l].tmp;
        H.b[l] = s->lv[l].b;
    }
    return H;
}

LevelPtrs<float> fp32_ptrs(ccmg_solver* s)
{
    LevelPtrs<float> H;
    for (int l = 0; l < s->L; ++l) {
        H.home[l] = s->lv[l].phi32;
        H.tmp[l] = s->lv[l].tmp32;
        H.b[l] = s->lv[l].b32;
    }
    return H;
}

int enqueue_ctl_init(ccmg_solver* s, double rtol)
{
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s->stream, s->ctl, rtol);
    LAUNCHCHK(s);
    return CCMG_OK;
}

// ---- variable permittivity -----------------------------------------------
VcLevel vc_level(const ccmg_solver* s, int l)
{
    VcLevel V{};
    V.kx = s->vkx[l];
    V.ky = s->vky[l];
    V.kz = s->vkz[l];
    V.nx = s->lv[l].nx;
    V.ny = s->lv[l].ny;
    V.nz = s->lv[l].nz;
    for (int fc = 0; fc < 6; ++fc) V.dir[fc] = s->bc[fc].kind == CCMG_DIRICHLET;
    for (int a = 0; a < 3; ++a) V.per[a] = s->bc[2 * a].kind == CCMG_PERIODIC;
    return V;
}

int vc_grid(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 4096); }

int enqueue_vc_fold(ccmg_solver* s, const double* f, bool homogeneous)
{
    VcFold P{};
    P.f = f;
    P.bt = s->lv[0].b;
    P.h = s->h;
    P.homogeneous = homogeneous;
    for (int fc = 0; fc < 6; ++fc) {
        P.value[fc] = s->bc[fc].value;
        P.face[fc] = s->face_on[fc] ? s->face_vals[fc] : nullptr;
    }
    hipLaunchKernelGGL(k_vc_fold, dim3(vc_grid(s->lv[0].n)), dim3(256), 0, s->stream, P, vc_level(s, 0));
    LAUNCHCHK(s);
    return CCMG_OK;
}

// Fused stored-stencil residual pass over level l (no periodic axis):
// RESTRICT writes the coarse b-tilde and zeroes the coarse phi, otherwise the
// blocks store their norm partials.  Returns the block count, 0 if the grid
// needs more partials than the workspace holds (nothing launched).
template <bool RESTRICT>
int launch_vc_res(ccmg_solver* s, int l, const double* phi, double* bc_out, double* phic, int fin)
{
    static int per_cu = 0;
    if (per_cu == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(k_vc_res<RESTRICT>),
                                                         64 * kVcPassWaves, 0) != hipSuccess || nb < 1) {
            (void)hipGetLastError();
            nb = 1;
        }
        per_cu = nb;
    }
    const LevelBuf& B = s->lv[l];
    const Grid g = pass_grid(B.nx, B.ny, B.nz, kVcPassTX, kVcPassTY, 2, g_num_cus * per_cu * CCMG_CHUNK_CAPACITY_SCALE);
    if (!RESTRICT && g.blocks() > s->max_partials) return 0;
    VcResParams P;
    std::memset(&P, 0, sizeof P);
    P.L = vc_level(s, l);
    P.phi = phi;
    P.b = B.b;
    P.bc_out = bc_out;
    P.phic = phic;
    P.partials = s->partials;
    P.ctl = s->ctl;
    P.fin = fin;
    P.zc = g.zc;
    P.tiles_x = g.tiles_x;
    P.tiles_y = g.tiles_y;
    P.zchunks = g.zchunks;
    hipLaunchKernelGGL(k_vc_res<RESTRICT>, dim3(g.blocks()), dim3(64 * kVcPassWaves), 0, s->stream, P);
    return g.blocks();
}

int enqueue_vc_norm(ccmg_solver* s, const double* phi, int fin, double* r_out, double rscale, int cycle)
{
    if (!s->periodic && r_out == nullptr) {
        const int nb = launch_vc_res<false>(s, 0, phi, nullptr, nullptr, fin);
        if (nb > 0) {
            hipLaunchKernelGGL(k_finish_norm<64 * kVcPassWaves>, dim3(1), dim3(64 * kVcPassWaves), 0, s->stream,
                               (const double*)s->partials, nb, s->ctl, fin, cycle, fin == FIN_CYCLE ? 1 : 0);
            LAUNCHCHK(s);
            return CCMG_OK;
        }
    }
    if (phi == nullptr) return fail(s, CCMG_E_ARG, "internal: a zero-guess norm needs the fused residual pass");
    const int g = std::max(1, std::min(vc_grid(s->lv[0].n), s->max_partials));
    hipLaunchKernelGGL(k_vc_norm, dim3(g), dim3(kVcNormThreads), 0, s->stream, vc_level(s, 0), phi,
                       (const double*)s->lv[0].b, r_out, rscale, s->partials, s->ctl, fin, cycle);
    hipLaunchKernelGGL(k_finish_norm<kVcNormThreads>, dim3(1), dim3(kVcNormThreads), 0, s->stream,
                       (const double*)s->partials, g, s->ctl, fin, cycle, fin == FIN_CYCLE ? 1 : 0);
    LAUNCHCHK(s);
    return CCMG_OK;
}

void enqueue_vc_sweeps(ccmg_solver* s, int l, double* phi, int sweeps)
{
    const VcLevel V = vc_level(s, l);
    const size_t half = ((size_t)(V.nx + 1) / 2) * V.ny * V.nz;
    for (int k = 0; k < sweeps; ++k)
        for (int colour = 0; colour < 2; ++colour)
            hipLaunchKernelGGL(k_vc_sweep, dim3(vc_grid(half)), dim3(256), 0, s->stream, V, phi,
                               (const double*)s->lv[l].b, colour, (const Ctl*)s->ctl);
}

// one V(nu1,nu2)-cycle on the variable-permittivity hierarchy; fin_cycle > 0
// finalises the finest residual norm as that cycle
// `sweeps` red-black sweeps on level l, after the prolongation of the coarse
// correction ec (home += omega * e(parent)) when ec is given.  Without a
// periodic axis each sweep is one fused pass (k_vc_pass; the first one also
// applies the prolongation) from one buffer into the other, ending in `home`
// (a copy when the count is odd); a periodic axis takes the separate
// prolongation and the colour kernels.
void enqueue_vc_smooth(ccmg_solver* s, int l, double* home, int sweeps, const double* ec, bool zero_in = false)
{
    const LevelBuf& B = s->lv[l];
    if (s->periodic || sweeps <= 0) {
        if (ec != nullptr)
            hipLaunchKernelGGL(k_vc_prolong, dim3(vc_grid(B.n)), dim3(256), 0, s->stream, home, ec, B.nx, B.ny, B.nz,
                               s->opt.omega, (const Ctl*)s->ctl);
        enqueue_vc_sweeps(s, l, home, sweeps);
        return;
    }
    static int per_cu = 0;
    if (per_cu == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(k_vc_pass<true>),
                                                         64 * kVcPassWaves, 0) != hipSuccess || nb < 1) {
            (void)hipGetLastError();
            nb = 1;
        }
        per_cu = nb;
    }
    const Grid g = pass_grid(B.nx, B.ny, B.nz, kVcPassTX, kVcPassTY, 2, g_num_cus * per_cu * CCMG_CHUNK_CAPACITY_SCALE);
    VcPassParams P;
    std::memset(&P, 0, sizeof P);
    P.L = vc_level(s, l);
    P.b = B.b;
    P.ec = ec;
    P.omega = s->opt.omega;
    P.ctl = s->ctl;
    P.zc = g.zc;
    P.tiles_x = g.tiles_x;
    P.tiles_y = g.tiles_y;
    P.zchunks = g.zchunks;
    double* buf[2] = {home, B.tmp};
    int cur = 0;
    for (int k = 0; k < sweeps; ++k) {
        P.phi_in = (k == 0 && zero_in) ? nullptr : buf[cur];   // zero_in: home holds no guess yet (zero)
        P.phi_out = buf[cur ^ 1];
        if (k == 0 && ec != nullptr)
            hipLaunchKernelGGL(k_vc_pass<true>, dim3(g.blocks()), dim3(64 * kVcPassWaves), 0, s->stream, P);
        else
            hipLaunchKernelGGL(k_vc_pass<false>, dim3(g.blocks()), dim3(64 * kVcPassWaves), 0, s->stream, P);
        cur ^= 1;
    }
    if (cur != 0)
        hipLaunchKernelGGL((k_copy<double>), dim3(grid1d(B.n)), dim3(256), 0, s->stream, (const double*)B.tmp, home,
                           B.n, (const Ctl*)s->ctl);
}

// l0_zero: the finest guess is zero and not loaded (no periodic axis)
int enqueue_vc_cycle(ccmg_solver* s, double* phi0, int fin_cycle, bool l0_zero = false)
{
    const int L = s->L;
    auto home = [&](int l) { return l == 0 ? phi0 : s->lv[l].phi; };
    for (int l = 0; l + 1 < L; ++l) {
        enqueue_vc_smooth(s, l, home(l), s->opt.nu1, nullptr, l == 0 && l0_zero);
        if (!s->periodic) {
            launch_vc_res<true>(s, l, home(l), s->lv[l + 1].b, home(l + 1), 0);
        } else {
            const size_t nc = s->lv[l + 1].n;
            hipLaunchKernelGGL(k_vc_restrict, dim3(vc_grid(nc)), dim3(256), 0, s->stream, vc_level(s, l),
                               (const double*)home(l), (const double*)s->lv[l].b, s->lv[l + 1].b, home(l + 1),
                               (const Ctl*)s->ctl);
        }
    }
    {
        const VcLevel V = vc_level(s, L - 1);
        if (s->lv[L - 1].n <= (size_t)kVcCgThreads) {
            hipLaunchKernelGGL(k_vc_cg_cell, dim3(1), dim3(kVcCgThreads), 0, s->stream, V,
                               (const double*)s->lv[L - 1].b, home(L - 1), s->opt.cg_rtol, s->cg_maxit,
                               (const Ctl*)s->ctl);
        } else {
            const size_t lds = 4 * sizeof(double) * s->lv[L - 1].n;
            hipLaunchKernelGGL(k_vc_cg, dim3(1), dim3(kVcCgThreads), lds, s->stream, V,
                               (const double*)s->lv[L - 1].b, home(L - 1), s->opt.cg_rtol, s->cg_maxit,
                               (const Ctl*)s->ctl);
        }
    }
    for (int l = L - 2; l >= 0; --l) enqueue_vc_smooth(s, l, home(l), s->opt.nu2, home(l + 1));
    LAUNCHCHK(s);
    if (fin_cycle > 0) return enqueue_vc_norm(s, phi0, FIN_CYCLE, nullptr, 0.0, fin_cycle);
    return CCMG_OK;
}

// b-tilde_0 = h^2 (f + boundary terms); homogeneous=true drops the boundary
// values.  With init_norm (constant coefficients only) the same kernel also
// reduces ||b-tilde|| and finalises it as the initial residual of the zero
// guess (FIN_INIT), in place of a norm pass over b-tilde.
int enqueue_fold(ccmg_solver* s, const double* f, bool homogeneous, bool init_norm = false)
{
    if (s->vc_on) return enqueue_vc_fold(s, f, homogeneous);
    const LevelBuf& B = s->lv[0];
    FoldParams P{};
    P.f = f;
    P.bt = B.b;
    P.nx = B.nx;
    P.ny = B.ny;
    P.nz = B.nz;
    P.h = s->h;
    P.h2 = s->h * s->h;
    for (int fc = 0; fc < 6; ++fc) {
        const double g = homogeneous ? 0.0 : s->bc[fc].value;
        P.t[fc] = s->bc[fc].kind == CCMG_DIRICHLET ? 2.0 * g / (s->h * s->h) : g / s->h;
        P.face[fc] = (!homogeneous && s->face_on[fc]) ? s->face_vals[fc] : nullptr;
        P.dirichlet[fc] = s->bc[fc].kind == CCMG_DIRICHLET;
    }
    const int rows = B.ny * B.nz;
    if (init_norm) {
        const int nb = std::max(1, std::min({rows, s->max_partials, kFoldMaxBlocks}));
        hipLaunchKernelGGL(k_fold<true>, dim3(nb), dim3(kFoldThreads), 0, s->stream, P, s->partials);
        hipLaunchKernelGGL(k_finish_norm<512>, dim3(1), dim3(512), 0, s->stream, (const double*)s->partials, nb, s->ctl,
                           (int)FIN_INIT, 0, 0);
    } else {
        hipLaunchKernelGGL(k_fold<false>, dim3(std::min(rows, kFoldMaxBlocks)), dim3(kFoldThreads), 0, s->stream, P,
                           (double*)nullptr);
    }
    LAUNCHCHK(s);
    return CCMG_OK;
}

// residual-norm pass on the finest level (FP64) finalised as `fin`
int enqueue_norm(ccmg_solver* s, const double* phi, int fin, int res, double* r_out, float* r32_out, int cycle)
{
    if (s->vc_on) {
        if (res != RES_NORM) return fail(s, CCMG_E_ARG, "internal: norm kind with variable permittivity");
        return enqueue_vc_norm(s, phi, fin, r_out, 0.0, cycle);
    }
    PassParams<double> P = base_params<double>(s, 0);
    P.phi_in = phi;
    P.b = s->lv[0].b;
    P.fin = fin;
    P.cycle = cycle;
    P.r_out = r_out;
    P.r32_out = r32_out;
    if (!dispatch<double>(0, LOAD_PHI, res, P, s->stream)) return fail(s, CCMG_E_ARG, "norm pass");
    LAUNCHCHK(s);
    return CCMG_OK;
}

struct CtlHead {
    double rtol, bnorm, rnorm, rel, sig_cur, sig_next;
    int done, status, cycles, bzero;
    unsigned reserved;
    int cg_iters;
    int pad[2];
    double pb_max;
};
static_assert(sizeof(CtlHead) == offsetof(Ctl, hist), "control block header layout");

int read_ctl(ccmg_solver* s, CtlHead& h, int hist_upto)
{
    HIPCHK(s, hipMemcpyAsync(&h, s->ctl, sizeof h, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if (hist_upto >= 0) {
        const int n = std::min(hist_upto + 1, kMaxHist);
        s->hist.resize(n);
        HIPCHK(s, hipMemcpy(s->hist.data(), s->ctl->hist, n * sizeof(double), hipMemcpyDeviceToHost));
    }
    return CCMG_OK;
}

// Whole control block (header and history) to the host in one copy.
int read_all(ccmg_solver* s, CtlHead& h)
{
    s->ctl_host.resize(sizeof(Ctl));
    HIPCHK(s, hipMemcpyAsync(s->ctl_host.data(), s->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    std::memcpy(&h, s->ctl_host.data(), sizeof h);
    const Ctl* c = reinterpret_cast<const Ctl*>(s->ctl_host.data());
    const int n = std::max(0, std::min(h.cycles + 1, kMaxHist));
    s->hist.assign(c->hist, c->hist + n);
    return CCMG_OK;
}

// Run the cycle loop after the initial residual pass.  `enqueue_step(k)`
// enqueues cycle / refinement step k (k >= 1) ending with FIN_CYCLE(k).  The
// first batch is enqueued right behind the initial pass without waiting (its
// kernels return at once if the initial guess already satisfies the
// tolerance); the host synchronises once per batch, and sizes the next batch
// from the observed contraction.
template <typename F>
int run_loop(ccmg_solver* s, int max_cycles, F enqueue_step, CtlHead& h)
{
    int k = 0;
    int batch = s->last_cycles > 0 ? s->last_cycles : 8;
    int rc;
    for (;;) {
        batch = std::max(0, std::min(batch, max_cycles - k));
        for (int i = 0; i < batch; ++i) {
            rc = enqueue_step(k + 1 + i);
            if (rc) return rc;
        }
        k += batch;
        rc = read_all(s, h);
        if (rc) return rc;
        if (h.done || k >= max_cycles) break;
        if (!(h.rtol > 0.0)) {
            // no tolerance can stop the loop early (rtol = 0: fixed cycle count)
            batch = max_cycles - k;
            continue;
        }
        // estimate the remaining cycles from the last contraction, clamped
        // before the conversion (the logarithm ratio can be huge or infinite)
        const int c = h.cycles;
        const double rate = (c >= 1 && s->hist[c - 1] > 0.0) ? s->hist[c] / s->hist[c - 1] : 0.5;
        double need = 2.0;
        if (rate > 0.0 && rate < 1.0 && h.rel > 0.0) need = std::ceil(std::log(h.rtol / h.rel) / std::log(rate));
        if (!(need >= 1.0)) need = 1.0;
        batch = need >= 64.0 ? 64 : (int)need;
    }
    return CCMG_OK;
}

int finish_stats(ccmg_solver* s, const CtlHead& h, int inner_per_step, ccmg_stats* st,
                 std::chrono::steady_clock::time_point t0)
{
    prof_collect(s, h.cycles);
    s->last_cycles = h.cycles > 0 ? h.cycles : s->last_cycles;
    if (st) {
        st->cycles = h.cycles;
        st->inner_cycles = h.cycles * inner_per_step;
        st->rel_res0 = s->hist.empty() ? 0.0 : s->hist[0];
        st->rel_res = h.rel;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (h.status == -5) return fail(s, CCMG_E_NONFINITE, "residual is not finite after %d cycles", h.cycles);
    if (!h.done) return fail(s, CCMG_E_NOCONV, "relative residual %.3e >= rtol after %d cycles", h.rel, h.cycles);
    return CCMG_OK;
}

// Whole solve on b-tilde_0 already in the workspace.  phi: initial guess in,
// solution out; with zero_guess the guess is phi = 0 and phi is output only.
// init_done: the fold already finalised the initial norm (zero guess,
// constant coefficients).
int solve_folded(ccmg_solver* s, double* phi, double rtol, int max_cycles, ccmg_stats* st,
                 std::chrono::steady_clock::time_point t0, bool zero_guess = false, bool init_done = false)
{
    const LevelBuf& B0 = s->lv[0];
    // From the zero guess phi is never loaded before it is first written
    // (all but variable permittivity on a periodic axis, whose colour kernels
    // update phi in place): the norm passes take a null phi (read as zero: the
    // residual is b-tilde itself), the first cycle starts from zero and the
    // first refinement step reads a null phi.
    const bool no_load = zero_guess && !(s->vc_on && s->periodic);
    int rc;
    if (no_load) {
        if (!init_done && (rc = enqueue_norm(s, nullptr, FIN_INIT, RES_NORM, nullptr, nullptr, 0))) return rc;
        if (max_cycles == 0)   // no cycle will write phi: the last iterate is the guess
            hipLaunchKernelGGL((k_fill<double>), dim3(grid1d(B0.n)), dim3(256), 0, s->stream, phi, B0.n, 0.0);
        else
            hipLaunchKernelGGL(k_zero_if_done, dim3(grid1d(B0.n)), dim3(256), 0, s->stream, phi, B0.n,
                               (const Ctl*)s->ctl);
    } else {
        if (zero_guess)
            hipLaunchKernelGGL((k_fill<double>), dim3(grid1d(B0.n)), dim3(256), 0, s->stream, phi, B0.n, 0.0);
        if ((rc = enqueue_norm(s, phi, FIN_INIT, RES_NORM, nullptr, nullptr, 0))) return rc;
        hipLaunchKernelGGL(k_zero_if_bzero, dim3(grid1d(B0.n)), dim3(256), 0, s->stream, phi, B0.n,
                           (const Ctl*)s->ctl);
    }
    LAUNCHCHK(s);
    CtlHead h;
    int inner = 1;
    if (s->opt.precision == CCMG_FP64) {
        const LevelPtrs<double> H = fp64_ptrs(s, phi);
        rc = run_loop(s, max_cycles, [&](int k) {
            return s->vc_on ? enqueue_vc_cycle(s, phi, k, no_load && k == 1)
                            : enqueue_vcycle<double>(s, H, no_load && k == 1, k);
        }, h);
    } else {
        inner = s->opt.ir_inner_cycles;
        const LevelPtrs<float> H = fp32_ptrs(s);
        // first scaled FP32 residual of the initial guess (re-finalises cycle 0);
        // from the zero guess it is b-tilde, whose norm is finalised above
        if (no_load) {
            hipLaunchKernelGGL(k_first_r32, dim3(grid1d(B0.n / 2 + 1)), dim3(256), 0, s->stream, (const double*)B0.b,
                               s->lv[0].b32, B0.n, s->ctl);
            LAUNCHCHK(s);
        } else {
            rc = enqueue_norm(s, phi, FIN_CYCLE, RES_NORM_R32, nullptr, s->lv[0].b32, 0);
            if (rc) return rc;
        }
        double* tmp = s->lv[0].tmp;
        // Step k reads the iterate written by step k - 1 and writes the other
        // buffer.  From the zero guess the first step reads nothing and may
        // write either one: it is chosen so that the step count of the last
        // solve ends in phi, which spares the final copy when the count repeats.
        const int k_pred = s->last_cycles > 0 ? s->last_cycles : 3;
        const bool flip = no_load && (k_pred & 1);
        auto out_buf = [&](int k) { return (((k & 1) == 0) != flip) ? phi : tmp; };
        auto step = [&](int k) -> int {
            for (int m = 0; m < inner; ++m) {
                int r = enqueue_vcycle<float>(s, H, m == 0, 0);
                if (r) return r;
            }
            PassParams<double> P = base_params<double>(s, 0);
            P.phi_in = k == 1 ? (no_load ? nullptr : phi) : out_buf(k - 1);
            P.phi_out = out_buf(k);
            P.b = s->lv[0].b;
            P.corr = s->lv[0].phi32;
            P.r32_out = s->lv[0].b32;
            P.fin = FIN_CYCLE;
            P.cycle = k;
            if (!dispatch<double>(0, LOAD_CORR, RES_NORM_R32, P, s->stream)) return fail(s, CCMG_E_ARG, "IR pass");
            LAUNCHCHK(s);
            return CCMG_OK;
        };
        rc = run_loop(s, max_cycles, step, h);
        if (rc) return rc;
        if (h.cycles >= 1 && out_buf(h.cycles) == tmp) {
            // the last finished step left the iterate in tmp
            hipLaunchKernelGGL((k_copy<double>), dim3(grid1d(B0.n)), dim3(256), 0, s->stream, (const double*)tmp, phi,
                               B0.n, (const Ctl*)nullptr);
            LAUNCHCHK(s);
        }
    }
    if (rc) return rc;
    return finish_stats(s, h, inner, st, t0);
}

// Carve the workspace: control block, norm partials, then per level the
// FP64 b-tilde / ping-pong / home buffers (finest level, and every level in
// FP64 mode) and the FP32 hierarchy (FP32-IR mode).  With base == nullptr
// only the size is computed.  Returns the bytes used.
// boundary cells of face fc: x faces ny*nz, y faces nx*nz, z faces nx*ny
size_t face_cells(const ccmg_solver* s, int fc)
{
    const size_t nx = s->nx, ny = s->ny, nz = s->nz;
    return fc < 2 ? ny * nz : fc < 4 ? nx * nz : nx * ny;
}

size_t layout_workspace(ccmg_solver* s, char* base)
{
    size_t off = 0;
    auto take = [&](size_t b) -> char* { char* p = base ? base + off : nullptr; off += align256(b); return p; };
    Ctl* ctl = (Ctl*)take(sizeof(Ctl));
    double* part = (double*)take(2 * sizeof(double) * (size_t)s->max_partials);
    if (base) { s->ctl = ctl; s->partials = part; }
    for (int fc = 0; fc < 6; ++fc) {
        double* fv = (double*)take(sizeof(double) * face_cells(s, fc));
        if (base) s->face_vals[fc] = fv;
    }
    if (s->kappa2 > 0.0) {
        double* r = (double*)take(sizeof(double) * s->lv[0].n);
        double* d = (double*)take(sizeof(double) * s->lv[0].n);
        if (base) { s->pb_r = r; s->pb_d = d; }
    }
    if (s->opt.variable_eps) {
        for (int l = 0; l < s->L; ++l) {
            const size_t a = s->lv[l].nx, b = s->lv[l].ny, c = s->lv[l].nz;
            double* kx = (double*)take(sizeof(double) * (a + 1) * b * c);
            double* ky = (double*)take(sizeof(double) * a * (b + 1) * c);
            double* kz = (double*)take(sizeof(double) * a * b * (c + 1));
            if (base) { s->vkx[l] = kx; s->vky[l] = ky; s->vkz[l] = kz; }
        }
    }
    for (int l = 0; l < s->L; ++l) {
        LevelBuf& B = s->lv[l];
        const size_t n = B.n;
        double *b = nullptr, *tmp = nullptr, *phi = nullptr;
        float *b32 = nullptr, *tmp32 = nullptr, *phi32 = nullptr;
        if (l == 0 || s->opt.precision == CCMG_FP64) {
            b = (double*)take(n * 8);
            tmp = (double*)take(n * 8);
            if (l > 0) phi = (double*)take(n * 8);
        }
        if (s->opt.precision == CCMG_FP32_IR) {
            b32 = (float*)take(n * 4);
            tmp32 = (float*)take(n * 4);
            phi32 = (float*)take(n * 4);
        }
        if (base) {
            B.b = b; B.tmp = tmp; B.phi = phi;
            B.b32 = b32; B.tmp32 = tmp32; B.phi32 = phi32;
        }
    }
    return off;
}

int check_ready(ccmg_solver* s)
{
    if (s == nullptr) return CCMG_E_ARG;
    if (s->ws == nullptr) return fail(s, CCMG_E_STATE, "no workspace attached");
    return CCMG_OK;
}

#define NEED_DEV(s, p, name)                                                              \
    do {                                                                                  \
        if (!is_device_ptr(p)) return fail((s), CCMG_E_ARG, "%s must be device memory", name); \
    } while (0)

}  // namespace

// Workspace of the allocation-free solve (ccmg_solve_zero_static): one copy
// per device, resident while the process lives.  In host code this name is
// only a handle for hipGetSymbolAddress, never a device address.
static __device__ __align__(256) char scratch[CCMG_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

// Device address of the current device's scratch array, resolved once per
// device with that device current; also refreshes the CU count the pass
// grids are sized for.
int static_scratch(ccmg_solver* s, char** out)
{
    int dev = 0;
    HIPCHK(s, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(s, CCMG_E_ARG, "device ordinal %d beyond %d", dev, kMaxDevices);
    {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        if (g_scratch_ptr[dev] == nullptr) {
            void* p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || p == nullptr)
                return fail(s, CCMG_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            if (((uintptr_t)p & 255) != 0) return fail(s, CCMG_E_HIP, "internal: scratch not 256-byte aligned");
            g_scratch_ptr[dev] = static_cast<char*>(p);
        }
        *out = g_scratch_ptr[dev];
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0) g_num_cus = ncu;
    (void)hipGetLastError();
    return CCMG_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
namespace {

template <int SF>
void launch_deposit_sub(ccmg_solver* s, int n, const double* c, const double* r, const double* q, double eps, int mode,
                        double* f, double* w)
{
    const LevelBuf& B = s->lv[0];
    hipLaunchKernelGGL((k_deposit_sub<SF>), dim3(n), dim3(kSphereThreads), 0, s->stream, c, r, q, eps, s->h, B.nx,
                       B.ny, B.nz, mode, f, w);
}

template <int SF>
void launch_dq_sub(ccmg_solver* s, int n, const double* c, const double* r, double eps, int mode, const double* lam,
                   double* dq, int accumulate)
{
    const LevelBuf& B = s->lv[0];
    hipLaunchKernelGGL((k_dq_sub<SF>), dim3(n), dim3(kSphereThreads), 0, s->stream, c, r, eps, s->h, B.nx, B.ny,
                       B.nz, mode, lam, dq, accumulate);
}

template <template <int> class K, typename... A>
bool by_subsample(int sf, A... a)
{
    switch (sf) {
    case 1: K<1>::run(a...); return true;
    case 2: K<2>::run(a...); return true;
    case 3: K<3>::run(a...); return true;
    case 4: K<4>::run(a...); return true;
    case 5: K<5>::run(a...); return true;
    case 6: K<6>::run(a...); return true;
    case 7: K<7>::run(a...); return true;
    case 8: K<8>::run(a...); return true;
    default: return false;
    }
}

template <int SF>
struct DepositSub {
    template <typename... A>
    static void run(A... a) { launch_deposit_sub<SF>(a...); }
};

template <int SF>
void launch_coulomb(ccmg_solver* s, const double* phi, GradBc B, int n, const double* c, const double* r,
                    const double* q, int mode, double* force)
{
    hipLaunchKernelGGL((k_coulomb<SF>), dim3(n), dim3(kSphereThreads), 0, s->stream, phi, B, c, r, q, mode, force);
}

template <int SF>
struct Coulomb {
    template <typename... A>
    static void run(A... a) { launch_coulomb<SF>(a...); }
};

template <int SF>
void launch_coulomb_adjoint(ccmg_solver* s, const double* phi, GradBc B, int n, const double* c, const double* r,
                            const double* q, int mode, const double* gF, double* mu, double* direct)
{
    hipLaunchKernelGGL((k_coulomb_adjoint<SF>), dim3(n), dim3(kSphereThreads), 0, s->stream, phi, B, c, r, q, mode, gF,
                       mu, direct);
}

template <int SF>
struct CoulombAdj {
    template <typename... A>
    static void run(A... a) { launch_coulomb_adjoint<SF>(a...); }
};

GradBc grad_bc(const ccmg_solver* s)
{
    GradBc B{};
    B.nx = s->nx;
    B.ny = s->ny;
    B.nz = s->nz;
    B.h = s->h;
    for (int fc = 0; fc < 6; ++fc) {
        B.dirichlet[fc] = s->bc[fc].kind == CCMG_DIRICHLET;
        B.value[fc] = s->bc[fc].value;
        B.face[fc] = s->face_on[fc] ? s->face_vals[fc] : nullptr;
    }
    for (int a = 0; a < 3; ++a) B.per[a] = s->bc[2 * a].kind == CCMG_PERIODIC;
    return B;
}

template <int SF>
struct DqSub {
    template <typename... A>
    static void run(A... a) { launch_dq_sub<SF>(a...); }
};

int check_spheres(ccmg_solver* s, int n, const double* c, const double* r, int subsample, int mode)
{
    if (n < 0) return fail(s, CCMG_E_ARG, "negative sphere count");
    if (subsample < 1 || subsample > CCMG_MAX_SUBSAMPLE)
        return fail(s, CCMG_E_ARG, "subsample must be in 1..%d", CCMG_MAX_SUBSAMPLE);
    if (mode != CCMG_CHARGE_SPREAD && mode != CCMG_CHARGE_VOLUME) return fail(s, CCMG_E_ARG, "unknown charge mode");
    if (n > 0) {
        NEED_DEV(s, c, "d_centers");
        NEED_DEV(s, r, "d_radii");
    }
    return CCMG_OK;
}

}  // namespace

extern "C" {

void ccmg_default_options(ccmg_options* o)
{
    if (!o) return;
    o->nu1 = 2;
    o->nu2 = 2;
    o->levels = 0;
    o->omega = 2.0;
    o->precision = CCMG_FP64;
    o->ir_inner_cycles = 4;
    o->cg_rtol = 1e-13;
    o->cg_maxit = 0;
    o->fuse_sweeps = 2;
    o->bottom_cells = kBottomMaxCells;
    o->variable_eps = 0;
    o->ir_cg_rtol = 1e-6;
    o->kappa2 = 0.0;
}

int ccmg_create(ccmg_solver** out, int nx, int ny, int nz, double h, const ccmg_face bc[6],
                const ccmg_options* opt, void* hip_stream)
{
    g_create_err.clear();
    if (!out || !bc) return fail(nullptr, CCMG_E_ARG, "null argument");
    *out = nullptr;
    if (nx < 2 || ny < 2 || nz < 2) return fail(nullptr, CCMG_E_ARG, "grid must be at least 2 cells per axis");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(nullptr, CCMG_E_ARG, "spacing must be positive");
    ccmg_options o;
    ccmg_default_options(&o);
    if (opt) o = *opt;
    if (o.nu1 < 1 || o.nu1 > 8 || o.nu2 < 1 || o.nu2 > 8) return fail(nullptr, CCMG_E_ARG, "nu1, nu2 must be in 1..8");
    if (o.precision != CCMG_FP64 && o.precision != CCMG_FP32_IR) return fail(nullptr, CCMG_E_ARG, "bad precision");
    if (o.ir_inner_cycles < 1 || o.ir_inner_cycles > 16) return fail(nullptr, CCMG_E_ARG, "ir_inner_cycles in 1..16");
    if (o.fuse_sweeps != 1 && o.fuse_sweeps != 2) return fail(nullptr, CCMG_E_ARG, "fuse_sweeps must be 1 or 2");
    if (!(o.cg_rtol > 0.0) || !(o.ir_cg_rtol > 0.0) || o.cg_maxit < 0) return fail(nullptr, CCMG_E_ARG, "bad CG options");
    if (!std::isfinite(o.omega)) return fail(nullptr, CCMG_E_ARG, "bad omega");
    if (o.bottom_cells < 0 || o.bottom_cells > kBottomMaxCells)
        return fail(nullptr, CCMG_E_ARG, "bottom_cells must be in 0..%d", kBottomMaxCells);
    if (o.variable_eps != 0 && o.variable_eps != 1) return fail(nullptr, CCMG_E_ARG, "variable_eps must be 0 or 1");
    if (o.variable_eps && o.precision != CCMG_FP64)
        return fail(nullptr, CCMG_E_ARG, "variable permittivity is solved in FP64 only");
    bool any_dirichlet = false, any_periodic = false;
    for (int f = 0; f < 6; ++f) {
        if (bc[f].kind != CCMG_DIRICHLET && bc[f].kind != CCMG_NEUMANN && bc[f].kind != CCMG_PERIODIC)
            return fail(nullptr, CCMG_E_ARG, "bad face kind");
        if (!std::isfinite(bc[f].value)) return fail(nullptr, CCMG_E_ARG, "face value not finite");
        any_dirichlet |= bc[f].kind == CCMG_DIRICHLET;
        any_periodic |= bc[f].kind == CCMG_PERIODIC;
    }
    for (int a = 0; a < 3; ++a)
        if ((bc[2 * a].kind == CCMG_PERIODIC) != (bc[2 * a + 1].kind == CCMG_PERIODIC))
            return fail(nullptr, CCMG_E_ARG, "periodic faces come in pairs (axis %d)", a);
    if (any_periodic) {
        // periodic faces run on the stored-stencil operator (unit permittivity
        // unless one is set)
        if (o.precision != CCMG_FP64) return fail(nullptr, CCMG_E_ARG, "periodic faces are solved in FP64 only");
        o.variable_eps = 1;
    }
    if (!(o.kappa2 >= 0.0) || !std::isfinite(o.kappa2)) return fail(nullptr, CCMG_E_ARG, "kappa2 must be finite and >= 0");
    if (o.kappa2 > 0.0 && o.variable_eps)
        return fail(nullptr, CCMG_E_ARG, "the Poisson-Boltzmann term needs constant coefficients (no variable "
                                         "permittivity or periodic faces)");
    if (!any_dirichlet && !(o.kappa2 > 0.0))
        return fail(nullptr, CCMG_E_SINGULAR, "all faces Neumann: the operator is singular");
    // hierarchy depth
    int L = o.levels;
    if (L == 0) {
        L = 1;
        int a = nx, b = ny, c = nz;
        while ((size_t)a * b * c > 512 && a % 2 == 0 && b % 2 == 0 && c % 2 == 0 && a >= 4 && b >= 4 && c >= 4 &&
               L < CCMG_MAX_LEVELS) {
            a /= 2; b /= 2; c /= 2;
            ++L;
        }
    }
    if (L < 2 || L > CCMG_MAX_LEVELS) return fail(nullptr, CCMG_E_DIMS, "levels must be in 2..%d", CCMG_MAX_LEVELS);
    const int div = 1 << (L - 1);
    if (nx % div || ny % div || nz % div)
        return fail(nullptr, CCMG_E_DIMS, "dims %dx%dx%d not divisible by 2^(levels-1) = %d", nx, ny, nz, div);
    const size_t ncoarse = (size_t)(nx / div) * (ny / div) * (nz / div);
    if (ncoarse > CCMG_MAX_COARSE_CELLS)
        return fail(nullptr, CCMG_E_DIMS, "coarsest grid has %zu cells (max %d): use more levels", ncoarse,
                    CCMG_MAX_COARSE_CELLS);
    if ((size_t)nx * ny * nz > (size_t)1 << 34) return fail(nullptr, CCMG_E_DIMS, "grid too large");
    // the smoother addresses one z-plane per buffer descriptor (32-bit byte offsets)
    if ((size_t)nx * ny * sizeof(double) >= (size_t)1 << 31)
        return fail(nullptr, CCMG_E_DIMS, "an x-y plane of %dx%d cells reaches 2 GiB", nx, ny);

    ccmg_solver* s = new ccmg_solver();
    s->nx = nx; s->ny = ny; s->nz = nz; s->h = h;
    for (int f = 0; f < 6; ++f) {
        s->bc[f] = bc[f];
        s->sh[f] = bc[f].kind == CCMG_DIRICHLET ? 1 : -1;
    }
    s->opt = o;
    s->kappa2 = o.kappa2;
    s->periodic = any_periodic;
    s->opt.levels = L;
    s->stream = (hipStream_t)hip_stream;
    s->L = L;
    s->cg_maxit = o.cg_maxit > 0 ? o.cg_maxit : (int)(2 * ncoarse);
    // bottom: first coarse level with <= bottom_cells cells that still has a level below it
    s->lb = -1;
    for (int l = 1; l < L - 1; ++l) {
        const size_t n = (size_t)(nx >> l) * (ny >> l) * (nz >> l);
        if (n <= (size_t)o.bottom_cells && L - l <= kBottomMaxLevels) { s->lb = l; break; }
    }

    s->max_partials = max_pass_blocks(nx, ny, nz);
    for (int l = 0; l < L; ++l) {
        LevelBuf& B = s->lv[l];
        B.nx = nx >> l; B.ny = ny >> l; B.nz = nz >> l;
        B.n = (size_t)B.nx * B.ny * B.nz;
    }
    s->need_bytes = layout_workspace(s, nullptr);
    *out = s;
    return CCMG_OK;
}

size_t ccmg_workspace_bytes(const ccmg_solver* s) { return s ? s->need_bytes : 0; }

namespace {
int vc_unit_faces(ccmg_solver* s);
}  // namespace

int ccmg_set_workspace(ccmg_solver* s, void* d_ptr, size_t bytes)
{
    if (!s) return CCMG_E_ARG;
    if (!d_ptr) return fail(s, CCMG_E_ARG, "null workspace");
    if (((uintptr_t)d_ptr & 255) != 0) return fail(s, CCMG_E_ARG, "workspace must be 256-byte aligned");
    if (bytes < s->need_bytes) return fail(s, CCMG_E_STATE, "workspace of %zu bytes, need %zu", bytes, s->need_bytes);
    NEED_DEV(s, d_ptr, "workspace");
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            g_num_cus = ncu;
        (void)hipGetLastError();
    }
    char* base = (char*)d_ptr;
    if (layout_workspace(s, base) != s->need_bytes) return fail(s, CCMG_E_STATE, "internal: workspace layout mismatch");
    s->ws = base;
    s->ws_bytes = bytes;
    if (s->periodic) return vc_unit_faces(s);
    return CCMG_OK;
}

int ccmg_set_stream(ccmg_solver* s, void* hip_stream)
{
    if (!s) return CCMG_E_ARG;
    s->stream = (hipStream_t)hip_stream;
    return CCMG_OK;
}

int ccmg_num_levels(const ccmg_solver* s) { return s ? s->L : 0; }

int ccmg_level_dims(const ccmg_solver* s, int l, int dims_out[3])
{
    if (!s || !dims_out || l < 0 || l >= s->L) return CCMG_E_ARG;
    dims_out[0] = s->lv[l].nx;
    dims_out[1] = s->lv[l].ny;
    dims_out[2] = s->lv[l].nz;
    return CCMG_OK;
}

int ccmg_deposit_charges(ccmg_solver* s, int n, const double* d_centers, const double* d_radii, const double* d_q,
                         double eps, double* d_f, int* d_counts)
{
    if (!s) return CCMG_E_ARG;
    s->err.clear();
    if (n < 0) return fail(s, CCMG_E_ARG, "negative sphere count");
    if (!(eps > 0.0)) return fail(s, CCMG_E_ARG, "eps must be positive");
    NEED_DEV(s, d_f, "d_f");
    const LevelBuf& B = s->lv[0];
    hipLaunchKernelGGL((k_fill<double>), dim3(grid1d(B.n)), dim3(256), 0, s->stream, d_f, B.n, 0.0);
    if (n > 0) {
        NEED_DEV(s, d_centers, "d_centers");
        NEED_DEV(s, d_radii, "d_radii");
        NEED_DEV(s, d_q, "d_q");
        if (d_counts) NEED_DEV(s, d_counts, "d_counts");
        hipLaunchKernelGGL(k_deposit, dim3(n), dim3(kSphereThreads), 0, s->stream, d_centers, d_radii, d_q, eps, s->h,
                           B.nx, B.ny, B.nz, d_f, d_counts);
    }
    LAUNCHCHK(s);
    return CCMG_OK;
}

int ccmg_deposit_charges_sub(ccmg_solver* s, int n, const double* d_centers, const double* d_radii, const double* d_q,
                             double eps, int subsample, int mode, double* d_f, double* d_weights)
{
    if (!s) return CCMG_E_ARG;
    s->err.clear();
    int rc = check_spheres(s, n, d_centers, d_radii, subsample, mode);
    if (rc) return rc;
    if (!(eps > 0.0)) return fail(s, CCMG_E_ARG, "eps must be positive");
    NEED_DEV(s, d_f, "d_f");
    const LevelBuf& B = s->lv[0];
    hipLaunchKernelGGL((k_fill<double>), dim3(grid1d(B.n)), dim3(256), 0, s->stream, d_f, B.n, 0.0);
    if (n > 0) {
        NEED_DEV(s, d_q, "d_q");
        if (d_weights) NEED_DEV(s, d_weights, "d_weights");
        by_subsample<DepositSub>(subsample, s, n, d_centers, d_radii, d_q, eps, mode, d_f, d_weights);
    }
    LAUNCHCHK(s);
    return CCMG_OK;
}

int ccmg_charge_gradient(ccmg_solver* s, int n, const double* d_centers, const double* d_radii, double eps,
                         int subsample, int mode, const double* d_lambda, double* d_dq)
{
    if (!s) return CCMG_E_ARG;
    s->err.clear();
    int rc = check_spheres(s, n, d_centers, d_radii, subsample, mode);
    if (rc) return rc;
    if (!(eps > 0.0)) return fail(s, CCMG_E_ARG, "eps must be positive");
    if (n == 0) return CCMG_OK;
    NEED_DEV(s, d_lambda, "d_lambda");
    NEED_DEV(s, d_dq, "d_dq");
    by_subsample<DqSub>(subsample, s, n, d_centers, d_radii, eps, mode, d_lambda, d_dq, 0);
    LAUNCHCHK(s);
    return CCMG_OK;
}

int ccmg_gradient(ccmg_solver* s, const double* d_phi, double* d_grad)
{
    int rc = check_ready(s);
    if (rc) return rc;
    s->err.clear();
    NEED_DEV(s, d_phi, "d_phi");
    NEED_DEV(s, d_grad, "d_grad");
    hipLaunchKernelGGL(k_gradient, dim3(grid1d(s->lv[0].n)), dim3(256), 0, s->stream, d_phi, grad_bc(s), d_grad);
    LAUNCHCHK(s);
    return CCMG_OK;
}

int ccmg_coulomb_force(ccmg_solver* s, const double* d_phi, int n, const double* d_centers, const double* d_radii,
                       const double* d_q, int subsample, int mode, double* d_force)
{
    int rc = check_ready(s);
    if (rc) return rc;
    s->err.clear();
    if ((rc = check_spheres(s, n, d_centers, d_radii, subsample, mode))) return rc;
    if (n == 0) return CCMG_OK;
    NEED_DEV(s, d_phi, "d_phi");
    NEED_DEV(s, d_q, "d_q");
    NEED_DEV(s, d_force, "d_force");
    by_subsample<Coulomb>(subsample, s, d_phi, grad_bc(s), n, d_centers, d_radii, d_q, mode, d_force);
    LAUNCHCHK(s);
    return CCMG_OK;
}

int ccmg_coulomb_adjoint(ccmg_solver* s, const double* d_phi, int n, const double* d_centers, const double* d_radii,
                         const double* d_q, int subsample, int mode, const double* d_gF, double* d_mu, double* d_direct)
{
    int rc = check_ready(s);
    if (rc) return rc;
    s->err.clear();
    if ((rc = check_spheres(s, n, d_centers, d_radii, subsample, mode))) return rc;
    NEED_DEV(s, d_mu, "d_mu");
    const size_t n0 = s->lv[0].n;
    hipLaunchKernelGGL((k_fill<double>), dim3(grid1d(n0)), dim3(256), 0, s->stream, d_mu, n0, 0.0);
    if (n > 0) {
        NEED_DEV(s, d_phi, "d_phi");
        NEED_DEV(s, d_q, "d_q");
        NEED_DEV(s, d_gF, "d_gF");
        NEED_DEV(s, d_direct, "d_direct");
        by_subsample<CoulombAdj>(subsample, s, d_phi, grad_bc(s), n, d_centers, d_radii, d_q, mode, d_gF, d_mu,
                                 d_direct);
    }
    LAUNCHCHK(s);
    return CCMG_OK;
}

int ccmg_force_charge_gradient(ccmg_solver* s, const double* d_phi, int n, const double* d_centers,
                               const double* d_radii, const double* d_q, double eps, int force_subsample,
                               int force_mode, int deposit_subsample, int deposit_mode, const double* d_gF,
                               double* d_mu, double* d_lambda, double* d_dq, double rtol, int max_cycles,
                               ccmg_stats* st)
{
    int rc = check_ready(s);
    if (rc) return rc;
    s->err.clear();
    if ((rc = check_spheres(s, n, d_centers, d_radii, force_subsample, force_mode))) return rc;
    if ((rc = check_spheres(s, n, d_centers, d_radii, deposit_subsample, deposit_mode))) return rc;
    if (!(eps > 0.0)) return fail(s, CCMG_E_ARG, "eps must be positive");
    NEED_DEV(s, d_mu, "d_mu");
    NEED_DEV(s, d_lambda, "d_lambda");
    if (n > 0) NEED_DEV(s, d_dq, "d_dq");
    // mu = dL/dphi through the forces; dq = the direct term at fixed phi
    if ((rc = ccmg_coulomb_adjoint(s, d_phi, n, d_centers, d_radii, d_q, force_subsample, force_mode, d_gF, d_mu,
                                   d_dq)))
        return rc;
    // lambda = A^-1 mu (homogeneous boundary values), then dq += the
    // deposition's charge gradient of lambda
    const int src = ccmg_adjoint_solve(s, d_mu, d_lambda, 0, nullptr, nullptr, eps, nullptr, nullptr, rtol,
                                       max_cycles, st);
    if (src != CCMG_OK && src != CCMG_E_NOCONV) return src;
    if (n > 0) {
        by_subsample<DqSub>(deposit_subsample, s, n, d_centers, d_radii, eps, deposit_mode, (const double*)d_lambda,
                            d_dq, 1);
        LAUNCHCHK(s);
    }
    return src;
}

namespace {
// unit permittivity on every level (the periodic solver's default operator)
int vc_unit_faces(ccmg_solver* s)
{
    for (int l = 0; l < s->L; ++l) {
        const LevelBuf& B = s->lv[l];
        const size_t nfx = (size_t)(B.nx + 1) * B.ny * B.nz, nfy = (size_t)B.nx * (B.ny + 1) * B.nz,
                     nfz = (size_t)B.nx * B.ny * (B.nz + 1);
        hipLaunchKernelGGL((k_fill<double>), dim3(grid1d(nfx)), dim3(256), 0, s->stream, s->vkx[l], nfx, 1.0);
        hipLaunchKernelGGL((k_fill<double>), dim3(grid1d(nfy)), dim3(256), 0, s->stream, s->vky[l], nfy, 1.0);
        hipLaunchKernelGGL((k_fill<double>), dim3(grid1d(nfz)), dim3(256), 0, s->stream, s->vkz[l], nfz, 1.0);
    }
    LAUNCHCHK(s);
    s->vc_on = true;
    return CCMG_OK;
}
}  // namespace

int ccmg_set_permittivity(ccmg_solver* s, const double* d_eps)
{
    int rc = check_ready(s);
    if (rc) return rc;
    s->err.clear();
    if (!s->opt.variable_eps) return fail(s, CCMG_E_STATE, "solver created without variable_eps");
    if (d_eps == nullptr) {
        if (s->periodic) return vc_unit_faces(s);
        s->vc_on = false;
        return CCMG_OK;
    }
    NEED_DEV(s, d_eps, "d_eps");
    const LevelBuf& B = s->lv[0];
    const size_t nf = (size_t)(B.nx + 1) * B.ny * B.nz + (size_t)B.nx * (B.ny + 1) * B.nz +
                      (size_t)B.nx * B.ny * (B.nz + 1);
    const VcLevel V0 = vc_level(s, 0);
    hipLaunchKernelGGL(k_vc_faces, dim3(vc_grid(nf)), dim3(256), 0, s->stream, d_eps, s->vkx[0], s->vky[0], s->vkz[0],
                       B.nx, B.ny, B.nz, V0.per[0], V0.per[1], V0.per[2]);
    for (int l = 0; l + 1 < s->L; ++l) {
        const LevelBuf& C = s->lv[l + 1];
        const size_t nc = (size_t)(C.nx + 1) * C.ny * C.nz + (size_t)C.nx * (C.ny + 1) * C.nz +
                          (size_t)C.nx * C.ny * (C.nz + 1);
        hipLaunchKernelGGL(k_vc_coarsen, dim3(vc_grid(nc)), dim3(256), 0, s->stream, vc_level(s, l), s->vkx[l + 1],
                           s->vky[l + 1], s->vkz[l + 1], C.nx, C.ny, C.nz);
    }
    LAUNCHCHK(s);
    s->vc_on = true;
    return CCMG_OK;
}

int ccmg_set_face_values(ccmg_solver* s, int face, const double* d_values)
{
    if (!s) return CCMG_E_ARG;
    s->err.clear();
    if (face < 0 || face > 5) return fail(s, CCMG_E_ARG, "face must be in 0..5");
    if (!s->ws) return fail(s, CCMG_E_STATE, "no workspace set (ccmg_set_workspace)");
    if (d_values == nullptr) {
        s->face_on[face] = false;
        return CCMG_OK;
    }
    NEED_DEV(s, d_values, "d_values");
    HIPCHK(s, hipMemcpyAsync(s->face_vals[face], d_values, sizeof(double) * face_cells(s, face),
                             hipMemcpyDeviceToDevice, s->stream));
    s->face_on[face] = true;
    return CCMG_OK;
}

namespace {

// one cycle (FP64) or one refinement step (FP32-IR) on the folded RHS; with
// `norm` the finest residual norm is reduced into the control block
int enqueue_cycle(ccmg_solver* s, double* d_phi, bool norm)
{
    int rc;
    if (s->vc_on) return enqueue_vc_cycle(s, d_phi, norm ? 1 : 0);
    if (s->opt.precision == CCMG_FP64) return enqueue_vcycle<double>(s, fp64_ptrs(s, d_phi), false, norm ? 1 : 0);
    // FP32 cycles on the scaled residual, FP64 update (the update pass also
    // reduces the next residual norm)
    if ((rc = enqueue_norm(s, d_phi, FIN_INIT, RES_NORM, nullptr, nullptr, 0))) return rc;
    if ((rc = enqueue_norm(s, d_phi, FIN_CYCLE, RES_NORM_R32, nullptr, s->lv[0].b32, 0))) return rc;
    const LevelPtrs<float> H = fp32_ptrs(s);
    for (int m = 0; m < s->opt.ir_inner_cycles; ++m)
        if ((rc = enqueue_vcycle<float>(s, H, m == 0, 0))) return rc;
    PassParams<double> P = base_params<double>(s, 0);
    P.phi_in = d_phi;
    P.phi_out = s->lv[0].tmp;
    P.b = s->lv[0].b;
    P.corr = s->lv[0].phi32;
    P.r32_out = s->lv[0].b32;
    P.fin = FIN_CYCLE;
    P.cycle = 1;
    if (!dispatch<double>(0, LOAD_CORR, RES_NORM_R32, P, s->stream)) return fail(s, CCMG_E_ARG, "IR pass");
    // the update landed in tmp unless a non-finite norm stopped the step (then
    // the update pass did not run, or produced a non-finite residual): the copy
    // is gated on the same flag, so phi never receives stale or broken data
    const size_t n = s->lv[0].n;
    hipLaunchKernelGGL((k_copy<double>), dim3(grid1d(n)), dim3(256), 0, s->stream, (const double*)s->lv[0].tmp, d_phi,
                       n, (const Ctl*)s->ctl);
    LAUNCHCHK(s);
    return CCMG_OK;
}

}  // namespace

int ccmg_vcycle(ccmg_solver* s, double* d_phi, const double* d_f, double* rel_res_out)
{
    int rc = check_ready(s);
    if (rc) return rc;
    s->err.clear();
    NEED_DEV(s, d_phi, "d_phi");
    NEED_DEV(s, d_f, "d_f");
    if ((rc = enqueue_ctl_init(s, -1.0))) return rc;
    if ((rc = enqueue_fold(s, d_f, false))) return rc;
    if ((rc = enqueue_cycle(s, d_phi, rel_res_out != nullptr))) return rc;
    if (rel_res_out) {
        CtlHead h;
        if ((rc = read_ctl(s, h, -1))) return rc;
        *rel_res_out = h.rel;
        if (h.status == -5) return fail(s, CCMG_E_NONFINITE, "residual is not finite");
    }
    return CCMG_OK;
}

int ccmg_vcycles(ccmg_solver* s, double* d_phi, const double* d_f, int ncycles, double* d_rel_out)
{
    int rc = check_ready(s);
    if (rc) return rc;
    s->err.clear();
    if (ncycles < 0 || ncycles > CCMG_MAX_CYCLES) return fail(s, CCMG_E_ARG, "ncycles out of range");
    NEED_DEV(s, d_phi, "d_phi");
    NEED_DEV(s, d_f, "d_f");
    if (d_rel_out) NEED_DEV(s, d_rel_out, "d_rel_out");
    if (ncycles == 0) return CCMG_OK;
    if ((rc = enqueue_ctl_init(s, -1.0))) return rc;
    if ((rc = enqueue_fold(s, d_f, false))) return rc;
    for (int m = 0; m < ncycles; ++m)
        if ((rc = enqueue_cycle(s, d_phi, d_rel_out != nullptr && m == ncycles - 1))) return rc;
    if (d_rel_out)
        HIPCHK(s, hipMemcpyAsync(d_rel_out, &s->ctl->rel, sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    return CCMG_OK;
}

int ccmg_solve_zero(ccmg_solver* s, double* d_phi, const double* d_f, double rtol, int max_cycles, ccmg_stats* st)
{
    const auto t0 = std::chrono::steady_clock::now();
    int rc = check_ready(s);
    if (rc) return rc;
    s->err.clear();
    if (max_cycles < 0 || max_cycles > CCMG_MAX_CYCLES) return fail(s, CCMG_E_ARG, "max_cycles out of range");
    if (!(rtol >= 0.0)) return fail(s, CCMG_E_ARG, "rtol must be >= 0");
    NEED_DEV(s, d_phi, "d_phi");
    NEED_DEV(s, d_f, "d_f");
    if ((rc = enqueue_ctl_init(s, rtol))) return rc;
    const bool fused = !s->vc_on;   // the fold also reduces the initial norm
    if ((rc = enqueue_fold(s, d_f, false, fused))) return rc;
    return solve_folded(s, d_phi, rtol, max_cycles, st, t0, true, fused);
}

int ccmg_solve_zero_static(ccmg_solver* s, double* d_phi, const double* d_f, double rtol, int max_cycles,
                           ccmg_stats* st)
{
    if (!s) return CCMG_E_ARG;
    s->err.clear();
    // host-side checks first: nothing runs on the device for a rejected call
    if (s->need_bytes > CCMG_STATIC_SCRATCH_BYTES)
        return fail(s, CCMG_E_ARG,
                    "workspace of %zu bytes exceeds the static scratch of %zu bytes: attach a workspace and call "
                    "ccmg_solve_zero", s->need_bytes, (size_t)CCMG_STATIC_SCRATCH_BYTES);
    if (s->periodic || s->vc_on)
        return fail(s, CCMG_E_STATE, "periodic faces and variable permittivity keep their face coefficients in "
                                     "the attached workspace: use ccmg_solve_zero");
    for (int fc = 0; fc < 6; ++fc)
        if (s->face_on[fc])
            return fail(s, CCMG_E_STATE, "per-cell boundary values (face %d) live in the attached workspace: use "
                                         "ccmg_solve_zero", fc);
    char* p = nullptr;
    int rc = static_scratch(s, &p);
    if (rc) return rc;
    // carve the workspace from the scratch for this call, then restore the
    // caller's layout (or none: other entry points keep failing with E_STATE)
    char* const old_ws = s->ws;
    const size_t old_bytes = s->ws_bytes;
    layout_workspace(s, p);
    s->ws = p;
    s->ws_bytes = CCMG_STATIC_SCRATCH_BYTES;
    rc = ccmg_solve_zero(s, d_phi, d_f, rtol, max_cycles, st);
    if (rc != CCMG_OK && rc != CCMG_E_NOCONV && rc != CCMG_E_NONFINITE) {
        // an early error return may leave work queued that uses the scratch
        (void)hipStreamSynchronize(s->stream);
        (void)hipGetLastError();
    }
    if (old_ws != nullptr) layout_workspace(s, old_ws);
    s->ws = old_ws;
    s->ws_bytes = old_bytes;
    return rc;
}

int ccmg_solve(ccmg_solver* s, double* d_phi, const double* d_f, double rtol, int max_cycles, ccmg_stats* st)
{
    const auto t0 = std::chrono::steady_clock::now();
    int rc = check_ready(s);
    if (rc) return rc;
    s->err.clear();
    if (max_cycles < 0 || max_cycles > CCMG_MAX_CYCLES) return fail(s, CCMG_E_ARG, "max_cycles out of range");
    if (!(rtol >= 0.0)) return fail(s, CCMG_E_ARG, "rtol must be >= 0");
    NEED_DEV(s, d_phi, "d_phi");
    NEED_DEV(s, d_f, "d_f");
    if ((rc = enqueue_ctl_init(s, rtol))) return rc;
    if ((rc = enqueue_fold(s, d_f, false))) return rc;
    return solve_folded(s, d_phi, rtol, max_cycles, st, t0);
}

int ccmg_solve_pb(ccmg_solver* s, double* d_psi, const double* d_f, double rtol, int max_outer, int inner,
                  ccmg_stats* st)
{
    const auto t0 = std::chrono::steady_clock::now();
    int rc = check_ready(s);
    if (rc) return rc;
    s->err.clear();
    if (!(s->kappa2 > 0.0)) return fail(s, CCMG_E_STATE, "solver created without kappa2 > 0");
    if (s->opt.precision != CCMG_FP64) return fail(s, CCMG_E_ARG, "the Poisson-Boltzmann iteration runs in FP64");
    if (max_outer < 0 || max_outer > CCMG_MAX_CYCLES) return fail(s, CCMG_E_ARG, "max_outer out of range");
    if (inner < 1 || inner > 16) return fail(s, CCMG_E_ARG, "inner must be in 1..16");
    if (!(rtol >= 0.0)) return fail(s, CCMG_E_ARG, "rtol must be >= 0");
    NEED_DEV(s, d_psi, "d_psi");
    NEED_DEV(s, d_f, "d_f");
    const LevelBuf& B0 = s->lv[0];
    if ((rc = enqueue_ctl_init(s, rtol))) return rc;
    if ((rc = enqueue_fold(s, d_f, false))) return rc;
    PbParams P{};
    P.psi = d_psi;
    P.bt = B0.b;
    P.r = s->pb_r;
    P.nx = B0.nx;
    P.ny = B0.ny;
    P.nz = B0.nz;
    for (int f = 0; f < 6; ++f) P.sh[f] = s->sh[f];
    P.hk2 = s->h * s->h * s->kappa2;
    P.partials = s->partials;
    const int nb = std::max(1, std::min({B0.ny * B0.nz, 2 * s->max_partials / 3, kFoldMaxBlocks}));
    // the correction equation: right-hand side the nonlinear residual, unknown
    // delta (level 0), the other levels as for a cycle
    LevelPtrs<double> H = fp64_ptrs(s, s->pb_d);
    H.b[0] = s->pb_r;
    CtlHead h;
    for (int k = 0;; ++k) {
        hipLaunchKernelGGL(k_pb_residual, dim3(nb), dim3(kPbThreads), 0, s->stream, P);
        hipLaunchKernelGGL(k_pb_finish<512>, dim3(1), dim3(512), 0, s->stream, (const double*)s->partials, nb, s->ctl,
                           k);
        LAUNCHCHK(s);
        if ((rc = read_ctl(s, h, -1))) return rc;
        if (h.done || k >= max_outer) break;
        // shifted chord step: (A + cosh(max|psi|) kappa^2 I) delta = r by V-cycles from zero
        s->pb_c = std::cosh(h.pb_max);
        for (int m = 0; m < inner; ++m) {
            rc = enqueue_vcycle<double>(s, H, m == 0, 0);
            if (rc) { s->pb_c = 1.0; return rc; }
        }
        s->pb_c = 1.0;
        hipLaunchKernelGGL(k_axpy, dim3(grid1d(B0.n)), dim3(256), 0, s->stream, d_psi, (const double*)s->pb_d, B0.n);
        LAUNCHCHK(s);
    }
    if (h.bzero) {
        hipLaunchKernelGGL((k_fill<double>), dim3(grid1d(B0.n)), dim3(256), 0, s->stream, d_psi, B0.n, 0.0);
        LAUNCHCHK(s);
    }
    if ((rc = read_all(s, h))) return rc;
    return finish_stats(s, h, inner, st, t0);
}

int ccmg_adjoint_solve(ccmg_solver* s, const double* d_g, double* d_lambda, int n, const double* d_centers,
                       const double* d_radii, double eps, double* d_dq, double* d_drho, double rtol, int max_cycles,
                       ccmg_stats* st)
{
    const auto t0 = std::chrono::steady_clock::now();
    int rc = check_ready(s);
    if (rc) return rc;
    s->err.clear();
    if (max_cycles < 0 || max_cycles > CCMG_MAX_CYCLES) return fail(s, CCMG_E_ARG, "max_cycles out of range");
    if (!(rtol >= 0.0)) return fail(s, CCMG_E_ARG, "rtol must be >= 0");
    if (n < 0) return fail(s, CCMG_E_ARG, "negative sphere count");
    if ((d_dq || d_drho) && !(eps > 0.0)) return fail(s, CCMG_E_ARG, "eps must be positive");
    NEED_DEV(s, d_g, "d_g");
    NEED_DEV(s, d_lambda, "d_lambda");
    const size_t n0 = s->lv[0].n;
    if ((rc = enqueue_ctl_init(s, rtol))) return rc;
    const bool fused = !s->vc_on;   // the fold also reduces the initial norm
    if ((rc = enqueue_fold(s, d_g, true, fused))) return rc;
    const int src = solve_folded(s, d_lambda, rtol, max_cycles, st, t0, true, fused);   // from lambda = 0
    if (src != CCMG_OK && src != CCMG_E_NOCONV) return src;
    if (d_drho) {
        NEED_DEV(s, d_drho, "d_drho");
        hipLaunchKernelGGL(k_scale, dim3(grid1d(n0)), dim3(256), 0, s->stream, (const double*)d_lambda, d_drho, n0,
                           1.0 / eps);
    }
    if (n > 0 && d_dq) {
        NEED_DEV(s, d_centers, "d_centers");
        NEED_DEV(s, d_radii, "d_radii");
        NEED_DEV(s, d_dq, "d_dq");
        const LevelBuf& B = s->lv[0];
        hipLaunchKernelGGL(k_dq, dim3(n), dim3(kSphereThreads), 0, s->stream, d_centers, d_radii, eps, s->h, B.nx, B.ny,
                           B.nz, (const double*)d_lambda, d_dq);
    }
    LAUNCHCHK(s);
    if (st) {
        HIPCHK(s, hipStreamSynchronize(s->stream));
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return src;
}

int ccmg_residual(ccmg_solver* s, const double* d_phi, const double* d_f, double* d_r, double* rel_res_out)
{
    int rc = check_ready(s);
    if (rc) return rc;
    s->err.clear();
    NEED_DEV(s, d_phi, "d_phi");
    NEED_DEV(s, d_f, "d_f");
    if (d_r) NEED_DEV(s, d_r, "d_r");
    if ((rc = enqueue_ctl_init(s, -1.0))) return rc;
    if ((rc = enqueue_fold(s, d_f, false))) return rc;
    if (s->vc_on) {
        if ((rc = enqueue_vc_norm(s, d_phi, FIN_STORE, d_r, 1.0 / (s->h * s->h), 0))) return rc;
    } else {
        PassParams<double> P = base_params<double>(s, 0);
        P.phi_in = d_phi;
        P.b = s->lv[0].b;
        P.fin = FIN_STORE;
        P.r_out = d_r;
        P.rscale = 1.0 / (s->h * s->h);
        if (!dispatch<double>(0, LOAD_PHI, RES_STORE, P, s->stream)) return fail(s, CCMG_E_ARG, "residual pass");
        LAUNCHCHK(s);
    }
    if (rel_res_out) {
        CtlHead h;
        if ((rc = read_ctl(s, h, -1))) return rc;
        *rel_res_out = h.rel;
    }
    return CCMG_OK;
}

int ccmg_smooth(ccmg_solver* s, double* d_phi, const double* d_f, int sweeps)
{
    int rc = check_ready(s);
    if (rc) return rc;
    s->err.clear();
    if (sweeps < 0) return fail(s, CCMG_E_ARG, "negative sweep count");
    NEED_DEV(s, d_phi, "d_phi");
    NEED_DEV(s, d_f, "d_f");
    if (sweeps == 0) return CCMG_OK;
    if ((rc = enqueue_ctl_init(s, -1.0))) return rc;
    if ((rc = enqueue_fold(s, d_f, false))) return rc;
    if (s->vc_on) {
        enqueue_vc_sweeps(s, 0, d_phi, sweeps);
        LAUNCHCHK(s);
        return CCMG_OK;
    }
    const int fuse = s->opt.fuse_sweeps;
    std::vector<PassSpec> ps;
    for (int left = sweeps; left > 0;) {
        const int k = std::min(fuse, left);
        left -= k;
        ps.push_back({2 * k, LOAD_PHI, RES_NONE});
    }
    std::vector<int> dh;
    const bool copy = assign_dst((int)ps.size(), true, dh);
    double* cur = d_phi;
    for (size_t i = 0; i < ps.size(); ++i) {
        PassParams<double> P = base_params<double>(s, 0);
        P.phi_in = cur;
        P.b = s->lv[0].b;
        P.phi_out = dh[i] ? d_phi : s->lv[0].tmp;
        if (!dispatch<double>(ps[i].sphi, ps[i].load, ps[i].res, P, s->stream)) return fail(s, CCMG_E_ARG, "smooth pass");
        cur = P.phi_out;
    }
    if (copy) {
        const size_t n = s->lv[0].n;
        hipLaunchKernelGGL((k_copy<double>), dim3(grid1d(n)), dim3(256), 0, s->stream, (const double*)s->lv[0].tmp,
                           d_phi, n, (const Ctl*)nullptr);
    }
    LAUNCHCHK(s);
    return CCMG_OK;
}

int ccmg_history(const ccmg_solver* s, double* out, int max)
{
    if (!s || !out || max < 0) return CCMG_E_ARG;
    const int n = std::min<int>(max, (int)s->hist.size());
    for (int i = 0; i < n; ++i) out[i] = s->hist[i];
    return n;
}

int ccmg_profile_enable(ccmg_solver* s, int on)
{
    if (!s) return CCMG_E_ARG;
    s->prof = on != 0;
    return CCMG_OK;
}

int ccmg_profile_read(ccmg_solver* s, int which, double* total_ms, int* launches, int reset)
{
    if (!s || which < 0 || which >= 8) return CCMG_E_ARG;
    if (total_ms) *total_ms = s->prof_ms[which];
    if (launches) *launches = s->prof_n[which];
    if (reset) {
        s->prof_ms[which] = 0.0;
        s->prof_n[which] = 0;
    }
    return CCMG_OK;
}

const char* ccmg_last_error(const ccmg_solver* s) { return s ? s->err.c_str() : g_create_err.c_str(); }

void ccmg_destroy(ccmg_solver* s)
{
    if (!s) return;
    for (auto& r : s->prof_recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : s->prof_pool) (void)hipEventDestroy(e);
    delete s;
}

}  // extern "C"
