// Device kernels of the cell-centered multigrid solver (gfx950, wave64).
//
// Every level array is [nz][ny][nx], x fastest.  On the device the operator of
// level l is kept in unscaled integer form
//     (S phi)_c = d_c phi_c - sum of in-domain face neighbours,
// with d_c = 6 + (+1 per Dirichlet face, -1 per Neumann face of the cell):
// the 7-point finite-volume stencil with the boundary entries moved to the
// centre (Sec. 2.4 "Boundary conditions", Sec. 5.3).  The true level operator
// is A_l = s_l S with s_l = 1/(2^l h^2) (Galerkin coarsening with averaging
// restriction and piecewise-constant prolongation keeps this form, Sec. 3), so
// the device stores right-hand sides pre-divided by s_l ("b-tilde").  Cells
// outside the domain read as zero: boundary conditions live only in d_c and in
// the finest right-hand side, never in ghost values (Sec. 2.4 prefers this
// folding because Gauss-Seidel then uses the new values at the boundary).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

// planes of phi and b in flight ahead of the plane being smoothed
#ifndef CCMG_PREFETCH
#define CCMG_PREFETCH 2
#endif

namespace ccmg {

// ---------------------------------------------------------------------------
// Device control block: norms, per-cycle history and the stop flag.  Kernels
// of a solve check `done` on entry, so the host can enqueue several cycles
// without waiting and read the block once.
// ---------------------------------------------------------------------------
constexpr int kMaxHist = 1001;

struct Ctl {
    double rtol;
    double bnorm;       // ||b-tilde|| of the finest level
    double rnorm;       // latest ||r-tilde||
    double rel;         // latest relative residual
    double sig_cur;     // FP32-IR: scale of the correction being solved for
    double sig_next;    // FP32-IR: scale for the next residual
    int done;           // 1: stop (converged, zero RHS or non-finite)
    int status;         // 0 or -5 (non-finite)
    int cycles;         // index of the last finished cycle
    int bzero;          // ||b|| == 0
    unsigned int reserved;  // unused (keeps the layout)
    int cg_iters;       // iterations of the last coarsest-grid CG
    int pad[2];
    double pb_max;      // Poisson-Boltzmann: max |psi| of the iterate whose residual was reduced last
    double hist[kMaxHist];
};

enum Fin : int { FIN_NONE = 0, FIN_INIT = 1, FIN_CYCLE = 2, FIN_STORE = 3 };
enum Load : int { LOAD_PHI = 0, LOAD_ZERO = 1, LOAD_PROLONG = 2, LOAD_CORR = 3 };
enum Res : int { RES_NONE = 0, RES_RESTRICT = 1, RES_NORM = 2, RES_NORM_R32 = 3, RES_STORE = 4 };

// Parameters of the smoother-pass kernel (one struct for every variant).
template <typename T>
struct PassParams {
    const T* phi_in;     // LOAD_PHI / LOAD_PROLONG / LOAD_CORR; null reads as zero
    T* phi_out;          // nullable
    const T* b;          // b-tilde of this level
    const T* ec;         // LOAD_PROLONG: coarse correction (level l+1)
    T omega;             // LOAD_PROLONG
    const float* corr;   // LOAD_CORR: FP32 correction on this level
    T* bc_out;           // RES_RESTRICT: b-tilde of level l+1
    float* r32_out;      // RES_NORM_R32: residual scaled for the FP32 cycles
    T* r_out;            // RES_STORE: residual, scaled by rscale
    T rscale;            // RES_STORE
    double* partials;    // RES_NORM*: 2 doubles per block
    int max_partials;    // capacity of `partials` in blocks (checked on the host)
    Ctl* ctl;            // nullable
    int fin;             // Fin code for k_finish_norm (the launch after a norm pass)
    int cycle;           // FIN_CYCLE: cycle index
    int nx, ny, nz;
    int zc;              // planes per block (even)
    int tiles_x, tiles_y, zchunks;
    int sh[6];           // per-face centre shift: +1 Dirichlet, -1 Neumann
    T shift;             // diagonal shift of the level (linearised Poisson-Boltzmann term), 0 for Poisson
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double pow2_floor(double x)
{
    int e;
    frexp(x, &e);
    return ldexp(1.0, e - 1);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Linear block id remapped so that each XCD (blocks are dealt round-robin to
// the 8 XCDs) receives a contiguous range of tiles: neighbouring tiles then
// share their halos in the same L2.
__device__ __forceinline__ int xcd_block_id(int nblk)
{
    const int bid = blockIdx.x;
    const int q = nblk >> 3, rem = nblk & 7;
    const int xcd = bid & 7, k = bid >> 3;
    return xcd < rem ? xcd * (q + 1) + k : rem * (q + 1) + (xcd - rem) * q + k;
}

// Norm reductions take two kernels.  The producer's blocks each store the
// sums of r^2 and b^2 over their cells (partials[2 blk], partials[2 blk + 1]);
// k_finish_norm, launched next on the same stream, adds them in block order
// (deterministic) and updates the control block.  The kernel boundary orders
// the partials before their reads: no device-scope fence or arrival counter in
// the producer, whose blocks would otherwise each write back their XCD's L2
// and serialise on one atomic.
template <int NT>
__device__ void store_partials(double s_r2, double s_b2, double* partials, int myblk)
{
    __shared__ double red[2][NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    s_r2 = wave_sum(s_r2);
    s_b2 = wave_sum(s_b2);
    if (lane == 0) { red[0][w] = s_r2; red[1][w] = s_b2; }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < NT / 64; ++i) { a += red[0][i]; b += red[1][i]; }
        partials[2 * myblk] = a;
        partials[2 * myblk + 1] = b;
    }
}

// One workgroup of NT threads.  gate != 0: nothing to do when ctl->done was
// already set before the producer ran (the producer then returned at once).
template <int NT>
__global__ __launch_bounds__(NT) void k_finish_norm(const double* partials, int nblk, Ctl* ctl, int fin, int cycle,
                                                     int gate)
{
    if (gate && ctl->done) return;
    __shared__ double red[2][NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double a = 0.0, b = 0.0;
    for (int i = tid; i < nblk; i += NT) {
        a += partials[2 * i];
        b += partials[2 * i + 1];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) { red[0][w] = a; red[1][w] = b; }
    __syncthreads();
    if (tid != 0) return;
    double r2 = 0.0, b2 = 0.0;
    for (int i = 0; i < NT / 64; ++i) { r2 += red[0][i]; b2 += red[1][i]; }
    const double rn = sqrt(r2), bn = sqrt(b2);
    ctl->rnorm = rn;
    // a NaN/Inf anywhere in b or the residual makes one of the sums non-finite
    const bool finite = isfinite(rn) && isfinite(bn);
    const double rel = !finite ? (double)NAN : (bn > 0.0 ? rn / bn : 0.0);
    if (fin == FIN_INIT) {
        ctl->bnorm = bn;
        ctl->rel = rel;
        ctl->hist[0] = rel;
        ctl->cycles = 0;
        ctl->bzero = finite && (bn == 0.0);
        ctl->status = finite ? 0 : -5;
        // a negative rtol marks cycles without a stopping test (single and
        // warm-started cycles): only a non-finite norm stops them, also when
        // b vanishes (phi != 0 still has a residual to correct)
        ctl->done = !finite || (ctl->rtol >= 0.0 && ((bn == 0.0) || !(rel >= ctl->rtol)));
        ctl->sig_next = (finite && rn > 0.0) ? pow2_floor(rn) : 1.0;
    } else if (fin == FIN_CYCLE) {
        ctl->rel = rel;
        if (cycle < kMaxHist) ctl->hist[cycle] = rel;
        ctl->cycles = cycle;
        if (!finite) ctl->status = -5;
        if (!finite || !(rel >= ctl->rtol)) ctl->done = 1;
        ctl->sig_cur = ctl->sig_next;
        ctl->sig_next = (finite && rn > 0.0) ? pow2_floor(rn) : 1.0;
    } else if (fin == FIN_STORE) {
        ctl->bnorm = bn;
        ctl->rel = rel;
        ctl->status = finite ? 0 : -5;
    }
}

// ---------------------------------------------------------------------------
// Cross-lane moves without LDS: DPP wave shifts by one lane.
// lane_prev(v): the value v of lane-1; lane_next(v): the value of lane+1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lane_prev(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_next(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_prev(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_next(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

// an x-pair of cells as one vector access (x even, so 2*sizeof(T)-aligned)
template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

template <typename T>
__device__ __forceinline__ void load2(const T* p, T& a, T& b)
{
    const typename Vec2<T>::type v = *reinterpret_cast<const typename Vec2<T>::type*>(p);
    a = v.x;
    b = v.y;
}
template <typename T>
__device__ __forceinline__ void store2(T* p, T a, T b)
{
    typename Vec2<T>::type v;
    v.x = a;
    v.y = b;
    *reinterpret_cast<typename Vec2<T>::type*>(p) = v;
}

// Raw buffer accesses (gfx9 buffer descriptor, no stride): an access at a
// byte offset at or beyond the descriptor's size reads 0 and a store there is
// dropped by the hardware's range check.  The smoother pass addresses one
// plane per descriptor and gives lanes that must not access (outside the
// domain or the tile) the offset kOob, so its loads and stores need neither a
// branch nor zeroed destination registers.  A plane must stay below 2 GiB.
constexpr unsigned kOob = 0x80000000u;
constexpr int kBufWord3 = 0x00020000;   // gfx9: 32-bit data format, the rest zero
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, size_t plane_bytes, int t, bool in)
{
    const char* p = static_cast<const char*>(base) + (in ? (size_t)t * plane_bytes : 0);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(p), (short)0, in ? (int)plane_bytes : 0, kBufWord3);
}
__device__ __forceinline__ void bload2(__amdgpu_buffer_rsrc_t r, unsigned off, double& a, double& b)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
    a = __hiloint2double((int)v[1], (int)v[0]);
    b = __hiloint2double((int)v[3], (int)v[2]);
}
__device__ __forceinline__ void bload2(__amdgpu_buffer_rsrc_t r, unsigned off, float& a, float& b)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
    a = __uint_as_float(v[0]);
    b = __uint_as_float(v[1]);
}
__device__ __forceinline__ void bload1(__amdgpu_buffer_rsrc_t r, unsigned off, double& a)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
    a = __hiloint2double((int)v[1], (int)v[0]);
}
__device__ __forceinline__ void bload1(__amdgpu_buffer_rsrc_t r, unsigned off, float& a)
{
    a = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
// The FP64 passes' phi outputs are stored non-temporal: the next pass reads
// them back on other XCDs anyway, and the hint keeps the halo rows the
// current pass re-reads longer in L2 (measured: about 1 %).  FP32 outputs keep
// the default policy: their 64 MB arrays profit from staying cached (the hint
// costs the FP32 cycles 7 %).
constexpr int kStoreNT = 2;   // cache-policy operand of the buffer store: nt
__device__ __forceinline__ void bstore2(__amdgpu_buffer_rsrc_t r, unsigned off, double a, double b)
{
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    u4 v;
    v[0] = (unsigned)__double2loint(a);
    v[1] = (unsigned)__double2hiint(a);
    v[2] = (unsigned)__double2loint(b);
    v[3] = (unsigned)__double2hiint(b);
    __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)off, 0, kStoreNT);
}
__device__ __forceinline__ void bstore2(__amdgpu_buffer_rsrc_t r, unsigned off, float a, float b)
{
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    u2 v;
    v[0] = __float_as_uint(a);
    v[1] = __float_as_uint(b);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)off, 0, 0);
}
__device__ __forceinline__ void bstore1(__amdgpu_buffer_rsrc_t r, unsigned off, double a)
{
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    u2 v;
    v[0] = (unsigned)__double2loint(a);
    v[1] = (unsigned)__double2hiint(a);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)off, 0, 0);
}
__device__ __forceinline__ void bstore1(__amdgpu_buffer_rsrc_t r, unsigned off, float a)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(a), r, (int)off, 0, 0);
}

constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }
constexpr int lcm_c(int a, int b) { return a / gcd_c(a, b) * b; }

// ---------------------------------------------------------------------------
// The smoother pass.
//
// One workgroup owns an x-y tile and marches up a chunk of z-planes.  A lane
// holds an x-pair of cells (x even, x+1): one of each colour, so every
// red-black half-sweep updates exactly one cell of the pair and which one is
// known at compile time.  The 64 lanes of a wave form two row groups of 32
// pairs (64 cells along x, coalesced 16-byte accesses); each thread holds M
// consecutive rows, and the 2*WY row strips of the workgroup stack in y.
//
// A pass applies SPHI colour half-sweeps (SPHI/2 full sweeps, red first,
// Sec. 5.3) and optionally a residual stage, reading phi and b once: stage s
// at plane p runs at step t = p + s, so its planes p-1, p, p+1 are in the
// per-thread register ring.  x-neighbours come from the pair itself or from
// the adjacent lane (DPP), y-neighbours from the thread's own rows or, at
// strip edges, from LDS (double-buffered per step: one barrier per step).
// Each stage is exact on a tile that shrinks by one cell per stage, so the
// tile carries an H-cell halo that is loaded but never written.
//
//   LOAD: phi_in | zero | phi_in + omega * e(parent) | phi_in + sigma * corr
//   RES:  none | restriction of the residual to the next level's b-tilde |
//         residual norm | residual norm + residual / sigma as FP32 | store r
// ---------------------------------------------------------------------------
template <typename T, int SPHI, int RES, int M, int WY, int LOAD = LOAD_PHI>
struct PassShape {
    static constexpr int S = SPHI + (RES != RES_NONE ? 1 : 0);   // stages after the load
    static constexpr int H = (S + 1) & ~1;                           // x halo, even (the x-pair lanes)
    // y halo: exactly S rows; a tile then starts at an odd y when S is odd
    // (the colour parity offset YP), and the restriction pairs rows across
    // neighbouring strips.  FP32 restriction passes keep the even halo: their
    // 64-row tiles gain no tile from it and the extra registers spill.
    static constexpr int HY = (RES == RES_RESTRICT && sizeof(T) == 4) ? H : S;
    static constexpr int YP = HY & 1;
    static constexpr bool XSTRIP_RESTRICT = RES == RES_RESTRICT && YP == 1;
    static constexpr int EX = 64;                                    // 32 lanes x 2 cells
    static constexpr int NSTRIP = 2 * WY;
    static constexpr int EY = NSTRIP * M;
    static constexpr int TX = EX - 2 * H;
    static constexpr int TY = EY - 2 * HY;
    // phi ring: S + 2 planes are live; an even ring keeps the unrolled step
    // count U (a multiple of the ring lengths and of the colour period 2)
    // small, so the loop body stays well inside the instruction cache
    static constexpr int RP = (S + 3) & ~1;
    static constexpr int RB = S >= 4 ? RP : S + 1;                   // b ring planes
    // planes in flight: the five-stage passes have no registers to spare for a second one
    static constexpr int PD = CCMG_PREFETCH;
    static constexpr int U = lcm_c(lcm_c(lcm_c(RP, RB), 2), PD);   // unrolled steps
    static constexpr int NT = 64 * WY;
    static constexpr int E1 = SPHI > 0 ? SPHI : 1;                   // single-value edge stages
    // FP64 stages skip planes outside the domain (loaded as zeros, they stay
    // zero); the FP32 passes, at 16 waves per block and 128 registers, keep
    // updating them with a zeroing select instead, which spills nothing there
    static constexpr bool SKIP_OUTSIDE = sizeof(T) == 8;
};

#ifndef CCMG_PASS_WAVES_PER_EU
#define CCMG_PASS_WAVES_PER_EU 1
#endif


template <typename T, int SPHI, int LOAD, int RES, int M, int WY, bool PAD = false>
__global__ __launch_bounds__(64 * WY, CCMG_PASS_WAVES_PER_EU) void k_pass(PassParams<T> P)
{
    // No fused multiply-adds formed by the compiler: every stage is unrolled
    // into U copies and the long marches have a padded variant, and the
    // compiler's choice to fuse a product with a sum can differ between
    // copies, so a cell's rounding would depend on the step position at which
    // its plane is processed, i.e. on where its z-chunk starts.  The fused
    // forms that matter are written out (the residual d phi - sum with one
    // rounding, the prolongation and the refinement update), so every cell is
    // computed the same way under any tiling.
#pragma clang fp contract(off)
    using Sh = PassShape<T, SPHI, RES, M, WY, LOAD>;
    constexpr int S = Sh::S, H = Sh::H, HY = Sh::HY, YP = Sh::YP, TX = Sh::TX, TY = Sh::TY, RP = Sh::RP, RB = Sh::RB,
                  U = Sh::U;
    static_assert(TY % 2 == 0, "tile rows must be even (the row parity of every tile is YP)");
    constexpr int NSTRIP = Sh::NSTRIP;
    static_assert(M % 2 == 0, "rows per thread must be even");
    static_assert(TX > 0 && TY > 0, "tile too small for the halo");

    if (P.ctl != nullptr && P.ctl->done) return;

    // strip-edge exchange: [input of stage j+1][step parity][strip + 1][edge row][pair];
    // slots 0 and NSTRIP + 1 are zero pads, so that the first and the last strip
    // read their missing neighbour rows unconditionally (no per-lane branch)
    __shared__ T edge1[Sh::E1][2][NSTRIP + 2][2][32];
    // both cells of the edge rows, input of the residual stage (same padding)
    __shared__ T edge2[RES != RES_NONE ? 2 : 1][NSTRIP + 2][2][32][2];
    // restriction across strips (odd first row): row-0 pair sums, by step parity;
    // slot NSTRIP is a zero pad
    __shared__ T rq[Sh::XSTRIP_RESTRICT ? 2 : 1][NSTRIP + 1][32];
    {
        constexpr int n1 = Sh::E1 * 2 * 2 * 2 * 32, n2 = (RES != RES_NONE ? 2 : 1) * 2 * 2 * 32 * 2;
        for (int e = threadIdx.x; e < n1; e += 64 * WY) {
            const int xp_ = e & 31, row = (e >> 5) & 1, pad = (e >> 6) & 1, rest = e >> 7;   // rest = stage * 2 + parity
            edge1[rest >> 1][rest & 1][pad ? NSTRIP + 1 : 0][row][xp_] = T(0);
        }
        for (int e = threadIdx.x; e < n2; e += 64 * WY) {
            const int c = e & 1, xp_ = (e >> 1) & 31, row = (e >> 6) & 1, pad = (e >> 7) & 1, par_ = e >> 8;
            edge2[par_][pad ? NSTRIP + 1 : 0][row][xp_][c] = T(0);
        }
        for (int e = threadIdx.x; e < (Sh::XSTRIP_RESTRICT ? 2 : 1) * 32; e += 64 * WY) rq[e >> 5][NSTRIP][e & 31] = T(0);
        __syncthreads();
    }
    static_assert(!Sh::XSTRIP_RESTRICT || M == 2, "cross-strip restriction pairs row 1 with the next strip's row 0");

    const int nblk = P.tiles_x * P.tiles_y * P.zchunks;
    const int blk = xcd_block_id(nblk);
    const int bx = blk % P.tiles_x;
    const int by = (blk / P.tiles_x) % P.tiles_y;
    const int bz = blk / (P.tiles_x * P.tiles_y);

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int xp = lane & 31;
    const int strip = 2 * w + (lane >> 5);
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int xl = bx * TX - H + 2 * xp;             // even: the pair is (xl, xl+1)
    const int ybase = by * TY - HY + strip * M;      // parity YP
    const int z0 = bz * P.zc;
    const int z1 = min(nz, z0 + P.zc);
    const bool vx = (xl >= 0) && (xl < nx);          // nx even: both cells or neither
    const bool xin = (xp >= H / 2) && (xp < H / 2 + TX / 2);

    int dxy[M][2];
    T inv0[M][2];
    bool vrow[M], yin[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const int y = ybase + r;
        vrow[r] = vx && (y >= 0) && (y < ny);
        const int ry = strip * M + r;
        yin[r] = (ry >= HY) && (ry < HY + TY);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int x = xl + c;
            int d = 6;
            if (x == 0) d += P.sh[0];
            if (x == nx - 1) d += P.sh[1];
            if (y == 0) d += P.sh[2];
            if (y == ny - 1) d += P.sh[3];
            dxy[r][c] = d;
            // cells outside the domain get 1/d = 0: their update is exactly 0, no select needed
            inv0[r][c] = vrow[r] ? T(1) / (T(d) + P.shift) : T(0);
        }
    }
    const int cnx = nx >> 1, cny = ny >> 1;
    const size_t plane = (size_t)nx * ny;
    const size_t planeB = plane * sizeof(T), cplaneB = (size_t)cnx * cny * sizeof(T);
    // byte offsets in a plane: loads (in the domain), stores (owned by this
    // tile), parents of the prolongation and coarse cells of the restriction;
    // kOob where the lane must not access
    // b-tilde is read by stage s >= 1 only where that stage is exact, rows
    // [s, EY - 1 - s] of the tile (x pairs [s, EX - 1 - s]): never on the outermost
    // loaded rows, and in a single-stage pass not in the outermost x pairs either
    // (those values feed only cells that are inexact anyway), so they are not loaded
    unsigned offL[M], offS[M], offL4[M], offB[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const unsigned e = (unsigned)((ybase + r) * nx + xl);
        offL[r] = vrow[r] ? e * (unsigned)sizeof(T) : kOob;
        offS[r] = (vrow[r] && yin[r] && xin) ? e * (unsigned)sizeof(T) : kOob;
        offL4[r] = vrow[r] ? e * 4u : kOob;   // the FP32 correction of LOAD_CORR
        const int ry = strip * M + r;
        const bool bskip = ry == 0 || ry == Sh::EY - 1 || (S == 1 && (xp == 0 || xp == 31));
        offB[r] = bskip ? kOob : offL[r];
    }
    auto coarse_off = [&](int r, bool ok) -> unsigned {
        return ok ? (unsigned)((((ybase + r) >> 1) * cnx + (xl >> 1)) * (int)sizeof(T)) : kOob;
    };

    T ph[RP][M][2];
    T bb[RB][M][2];
#pragma unroll
    for (int q = 0; q < RP; ++q)
#pragma unroll
        for (int r = 0; r < M; ++r) { ph[q][r][0] = T(0); ph[q][r][1] = T(0); }
#pragma unroll
    for (int q = 0; q < RB; ++q)
#pragma unroll
        for (int r = 0; r < M; ++r) { bb[q][r][0] = T(0); bb[q][r][1] = T(0); }

    T sig_cur = T(0);
    double inv_sig_next = 1.0;
    if constexpr (LOAD == LOAD_CORR) sig_cur = (T)P.ctl->sig_cur;
    if constexpr (RES == RES_NORM_R32) inv_sig_next = 1.0 / P.ctl->sig_next;

    double acc_r2 = 0.0, acc_b2 = 0.0;
    T racc[M / 2];
#pragma unroll
    for (int r = 0; r < M / 2; ++r) racc[r] = T(0);

    // Prefetch: raw loads of planes t+1 .. t+PD are in flight while plane t's
    // stages run; they are combined (prolongation / correction) only when the
    // plane enters the ring, so no load is waited for early.
    constexpr int PD = Sh::PD;
    // parent rows of the prolongation: rows r, r+1 share one when the tile starts at an even y
    constexpr int NE = YP ? M : M / 2;
    T nph[PD][M][2], nbb[PD][M][2], nex[PD][NE];
    float ncr[PD][M][2];
    // parent values of plane t (zero outside the domain)
    unsigned offE[NE];
#pragma unroll
    for (int r = 0; r < M; r += (YP ? 1 : 2)) offE[YP ? r : r / 2] = coarse_off(r, vrow[r]);
    // PAD: planes at or beyond `tlim` are not needed; their loads read zeros
    // through a size-0 descriptor (no branch, so no register joins that would
    // make the compiler wait for loads still in flight)
    auto load_parents = [&](int t, T* e, int tlim) {
        const bool zin = (t >= 0) && (t < nz) && (!PAD || t < tlim);
        const auto re = plane_rsrc(P.ec, cplaneB, t >> 1, zin);
#pragma unroll
        for (int i = 0; i < NE; ++i) bload1(re, offE[i], e[i]);
    };
    // The two planes 2k, 2k+1 share their parent plane: an odd plane reuses
    // the parents of the even plane below it (kept in elast), so only even
    // planes load them.  The parity of a plane is fixed by its unrolled step.
    T elast[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) elast[i] = T(0);
    auto load_plane = [&](int t, int k, auto oddt, int tlim) {
        const bool zin = (t >= 0) && (t < nz) && (!PAD || t < tlim);
        const auto rb = plane_rsrc(P.b, planeB, t, zin);
        // a null phi_in reads as zero (the zero initial guess: no load is made)
        const auto rp = plane_rsrc(P.phi_in, planeB, t, zin && LOAD != LOAD_ZERO && P.phi_in != nullptr);
        const auto rc = plane_rsrc(P.corr, plane * sizeof(float), t, zin && LOAD == LOAD_CORR);
#pragma unroll
        for (int r = 0; r < M; ++r) {
            bload2(rb, offB[r], nbb[k][r][0], nbb[k][r][1]);
            if constexpr (LOAD != LOAD_ZERO) bload2(rp, offL[r], nph[k][r][0], nph[k][r][1]);
            else { nph[k][r][0] = T(0); nph[k][r][1] = T(0); }
            if constexpr (LOAD == LOAD_CORR) bload2(rc, offL4[r], ncr[k][r][0], ncr[k][r][1]);
        }
        if constexpr (LOAD == LOAD_PROLONG && !decltype(oddt)::value) load_parents(t, nex[k], tlim);
    };

    // tbeg has the parity of S (z0 is even); a cross-strip restriction
    // finishes each plane one step after its residual, hence one more step
    const int tbeg = z0 - S, tend = z1 + S + (Sh::XSTRIP_RESTRICT ? 1 : 0);
    T q1p = T(0);                                   // row-1 pair sum of the previous step's plane
#pragma unroll
    for (int k = 0; k < PD; ++k) {
        if ((S + k) & 1) load_plane(tbeg + k, k, std::true_type{}, tend);
        else load_plane(tbeg + k, k, std::false_type{}, tend);
    }
    // the first plane is odd when S is: its parents are those of plane tbeg - 1
    if constexpr (LOAD == LOAD_PROLONG && (S & 1)) load_parents(tbeg - 1, elast, tend);

    // PAD: the march runs a whole number of unrolled blocks of U steps; the
    // steps past tend load zeros (size-0 descriptors) and find every stage,
    // output, residual and restriction outside its z range, so they only move
    // the rings and pass the barrier.  Without it every step tests t < tend,
    // which joins every ring register after every step; the compiler's
    // copies at those joins wait for the prefetched planes, so a long march
    // loses its prefetch (the finest post-smoothing pass ran 10 % slower),
    // while a short one (coarse levels) would lose more to the padding.
    const int tstop = PAD ? tbeg + U * ((tend - tbeg + U - 1) / U) : tend;
    // Two copies of the unrolled block of U steps: blocks whose steps all lie
    // in [max(z0, 1) + S + 1, min(z1 + SPHI, nz)) run a copy with CK = false,
    // where every stage's plane is inside its needed range and the domain and
    // off the z faces, and the output, residual and restriction planes inside
    // the chunk, so those tests (scalar compares, selects and branches in
    // every stage) are compiled out; the other blocks run the checked copy.
    // The arithmetic is the same in both.  Long marches only: the padded ones
    // and the single-stage FP64 passes (the second copy costs registers, which
    // the FP32 and the short five-stage passes do not have to spare).
    const int t_lo = max(z0, 1) + S + 1, t_hi = min(z1 + SPHI, nz);
    constexpr int NCOPY = (PAD || (sizeof(T) == 8 && SPHI == 0)) ? 2 : 1;
    for (int tb = tbeg; tb < tstop; tb += U) {
    const bool interior = NCOPY == 2 && tb >= t_lo && tb + U <= t_hi;
#pragma unroll
    for (int copy = 0; copy < NCOPY; ++copy) {
    const bool CK = NCOPY == 1 || copy == 1;
    if (NCOPY == 2 && (copy == 0) != interior) continue;
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int t = tb + q;
            if (!CK || PAD || t < tend) {
                const int par = t & 1;
                // ---- stage 0: the prefetched plane t enters the rings; plane t+PD is requested
                {
                    const int s0 = q % RP, sb0 = q % RB, k = q % PD;
                    if constexpr (LOAD == LOAD_PROLONG) {
                        if (((S + q) & 1) == 0) {
#pragma unroll
                            for (int i = 0; i < NE; ++i) elast[i] = nex[k][i];
                        }
                    }
#pragma unroll
                    for (int r = 0; r < M; ++r) {
                        T v0 = nph[k][r][0], v1 = nph[k][r][1];
                        if constexpr (LOAD == LOAD_PROLONG) {
                            const T e = elast[YP ? r : r / 2];
                            v0 = fma(P.omega, e, v0);
                            v1 = fma(P.omega, e, v1);
                        }
                        if constexpr (LOAD == LOAD_CORR) {
                            v0 = fma(sig_cur, (T)ncr[k][r][0], v0);
                            v1 = fma(sig_cur, (T)ncr[k][r][1], v1);
                        }
                        ph[s0][r][0] = v0; ph[s0][r][1] = v1;
                        bb[sb0][r][0] = nbb[k][r][0]; bb[sb0][r][1] = nbb[k][r][1];
                    }
                    if constexpr (PAD) {
                        // the slot's old contents are consumed above: issue its next loads
                        // only now, so that they reuse the slot's registers (a load hoisted
                        // above those uses would land in other registers, and the copies
                        // back into the slot would wait for it); planes past tend read zeros
                        __builtin_amdgcn_sched_barrier(0);
                        if ((S + q + PD) & 1) load_plane(t + PD, k, std::true_type{}, tend);
                        else load_plane(t + PD, k, std::false_type{}, tend);
                    } else if (t + PD < tend) {
                        if ((S + q + PD) & 1) load_plane(t + PD, k, std::true_type{}, tend);
                        else load_plane(t + PD, k, std::false_type{}, tend);
                    }
                    const int ppar = (S + q) & 1;
                    if constexpr (SPHI > 0) {
                        const int o0 = (1 + 0 + ppar + YP) & 1, o1 = (1 + (M - 1) + ppar + YP) & 1;
                        edge1[0][par][strip + 1][0][xp] = ph[s0][0][o0];
                        edge1[0][par][strip + 1][1][xp] = ph[s0][M - 1][o1];
                    } else if constexpr (RES != RES_NONE) {
                        edge2[par][strip + 1][0][xp][0] = ph[s0][0][0];
                        edge2[par][strip + 1][0][xp][1] = ph[s0][0][1];
                        edge2[par][strip + 1][1][xp][0] = ph[s0][M - 1][0];
                        edge2[par][strip + 1][1][xp][1] = ph[s0][M - 1][1];
                    }
                }
                // ---- all strip-edge inputs of this step were written before the last
                // barrier (other parity buffer): read them at once, one LDS latency
                T e_lo[Sh::E1], e_hi[Sh::E1];
#pragma unroll
                for (int s = 1; s <= SPHI; ++s) {
                    const T* ein = &edge1[s - 1][par ^ 1][0][0][0];
                    e_lo[s - 1] = ein[(strip * 2 + 1) * 32 + xp];          // row 1 of strip - 1 (or the pad)
                    e_hi[s - 1] = ein[((strip + 2) * 2 + 0) * 32 + xp];    // row 0 of strip + 1 (or the pad)
                }
                T e2lo[2], e2hi[2];
                if constexpr (RES != RES_NONE) {
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        e2lo[c] = edge2[par ^ 1][strip][1][xp][c];
                        e2hi[c] = edge2[par ^ 1][strip + 2][0][xp][c];
                    }
                }
                // ---- stages 1..SPHI: colour half-sweeps, red ((x+y+z) even) first
#pragma unroll
                for (int s = 1; s <= SPHI; ++s) {
                    const int p = t - s;
                    const int sc = (q - s + 2 * U) % RP;
                    const int sm = (q - s - 1 + 2 * U) % RP;
                    const int sp = (q - s + 1 + 2 * U) % RP;
                    const int sb = (q - s + 2 * U) % RB;
                    const int cs = (s + 1) & 1;
                    const int ppar = (S + q - s) & 1;
                    int dz = 0;
                    if (CK && p == 0) dz += P.sh[4];
                    if (CK && p == nz - 1) dz += P.sh[5];
                    // Stage s is needed on planes [z0 - (S - s), z1 + (S - s)); outside, its
                    // values are read only by later stages that are skipped as well
                    // (the needed ranges nest), so the halo steps at the chunk ends run
                    // only the stages that matter.  Planes outside the domain are skipped
                    // too (see SKIP_OUTSIDE): they were loaded as zeros and must stay zero.
                    if (CK && (p < z0 - (S - s) || p >= z1 + (S - s))) continue;
                    const bool pin = (p >= 0) && (p < nz);
                    if (CK && Sh::SKIP_OUTSIDE && !pin) continue;
                    const T elo = e_lo[s - 1];
                    const T ehi = e_hi[s - 1];
                    // 1/diagonal of the updated cell of each row; planes at a z face
                    // (dz != 0, uniform over the workgroup) take a short branch that
                    // recomputes it, so the update itself exists once in the code
                    T invz[M];
#pragma unroll
                    for (int r = 0; r < M; ++r) invz[r] = inv0[r][(cs + r + ppar + YP) & 1];
                    if (CK && dz != 0) {
#pragma unroll
                        for (int r = 0; r < M; ++r) {
                            const int o = (cs + r + ppar + YP) & 1;
                            invz[r] = vrow[r] ? T(1) / (T(dxy[r][o] + dz) + P.shift) : T(0);
                        }
                    }
#pragma unroll
                    for (int r = 0; r < M; ++r) {
                        const int o = (cs + r + ppar + YP) & 1;
                        T xm, xq;
                        if (o == 0) { xm = lane_prev(ph[sc][r][1]); xq = ph[sc][r][1]; }
                        else        { xm = ph[sc][r][0]; xq = lane_next(ph[sc][r][0]); }
                        const T ym = r > 0 ? ph[sc][r - 1][o] : elo;
                        const T yp = r < M - 1 ? ph[sc][r + 1][o] : ehi;
                        const T sum = ((((xm + xq) + ym) + yp) + ph[sm][r][o]) + ph[sp][r][o];
                        // cells outside the domain have 1/d = 0: they stay zero
                        const T nv = (bb[sb][r][o] + sum) * invz[r];
                        if constexpr (Sh::SKIP_OUTSIDE) ph[sc][r][o] = nv;
                        else ph[sc][r][o] = (!CK || pin) ? nv : T(0);
                    }
                    // keep the stages apart in the schedule (bounds register live ranges)
                    __builtin_amdgcn_sched_barrier(0);
                    if (s < SPHI) {
                        const int o0 = (cs + 0 + ppar + YP) & 1, o1 = (cs + (M - 1) + ppar + YP) & 1;
                        edge1[s][par][strip + 1][0][xp] = ph[sc][0][o0];
                        edge1[s][par][strip + 1][1][xp] = ph[sc][M - 1][o1];
                    } else if (RES != RES_NONE) {
                        edge2[par][strip + 1][0][xp][0] = ph[sc][0][0];
                        edge2[par][strip + 1][0][xp][1] = ph[sc][0][1];
                        edge2[par][strip + 1][1][xp][0] = ph[sc][M - 1][0];
                        edge2[par][strip + 1][1][xp][1] = ph[sc][M - 1][1];
                    }
                }
                // ---- output of the smoothed plane t - SPHI
                if (P.phi_out != nullptr) {
                    const int po = t - SPHI;
                    if (!CK || (po >= z0 && po < z1)) {
                        const int so = (q - SPHI + 2 * U) % RP;
                        const auto rs = plane_rsrc(P.phi_out, planeB, po, true);
#pragma unroll
                        for (int r = 0; r < M; ++r) bstore2(rs, offS[r], ph[so][r][0], ph[so][r][1]);
                    }
                }
                // ---- restriction across strips of the plane whose residual the
                // previous step computed: children rows y (this thread's row 1) and
                // y + 1 (the next strip's row 0), planes paired in z as above
                if constexpr (Sh::XSTRIP_RESTRICT) if (!CK || (t - 1 - S >= z0 && t - 1 - S < z1)) {
                    const int pp = t - 1 - S;
                    const T q0n = rq[par ^ 1][strip + 1][xp];             // the pad after the last strip
                    const T s4 = q1p + q0n;
                    if ((pp & 1) == 0) {
                        racc[0] = s4;
                    } else {
                        const auto rr = plane_rsrc(P.bc_out, cplaneB, pp >> 1, true);
                        bstore1(rr, coarse_off(1, xin && vrow[1] && yin[1]), T(0.25) * (racc[0] + s4));
                    }
                }
                // ---- residual stage at plane t - S (both cells of every pair)
                if constexpr (RES != RES_NONE) if (!CK || (t - S >= z0 && t - S < z1)) {
                    const int p = t - S;
                    const int sc = (q - S + 2 * U) % RP;
                    const int sm = (q - S - 1 + 2 * U) % RP;
                    const int sp = (q - S + 1 + 2 * U) % RP;
                    const int sb = (q - S + 2 * U) % RB;
                    const bool pok = !CK || ((p >= z0) && (p < z1));
                    int dz = 0;
                    if (CK && p == 0) dz += P.sh[4];
                    if (CK && p == nz - 1) dz += P.sh[5];
                    const T* elo = e2lo;
                    const T* ehi = e2hi;
                    T res[M][2];
#pragma unroll
                    for (int r = 0; r < M; ++r) {
                        const T xm0 = lane_prev(ph[sc][r][1]);
                        const T xp1 = lane_next(ph[sc][r][0]);
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const T xm = c == 0 ? xm0 : ph[sc][r][0];
                            const T xq = c == 0 ? ph[sc][r][1] : xp1;
                            const T ym = r > 0 ? ph[sc][r - 1][c] : elo[c];
                            const T yp = r < M - 1 ? ph[sc][r + 1][c] : ehi[c];
                            const T sum = ((((xm + xq) + ym) + yp) + ph[sm][r][c]) + ph[sp][r][c];
                            res[r][c] = bb[sb][r][c] - fma(T(dxy[r][c] + dz) + P.shift, ph[sc][r][c], -sum);
                        }
                    }
                    if constexpr (Sh::XSTRIP_RESTRICT) {
                        // row 0 (odd y) pairs with the previous strip's row 1, row 1 with
                        // the next strip's row 0: publish row 0, keep row 1 for the next step
                        rq[par][strip][xp] = res[0][0] + res[0][1];
                        q1p = res[1][0] + res[1][1];
                    } else if constexpr (RES == RES_RESTRICT) {
                        // children: the pair (x), rows r, r+1 (y), planes p, p+1 (z)
                        // p lies in [z0, z1) here
#pragma unroll
                        for (int r = 0; r < M; r += 2) {
                            const T s4 = (res[r][0] + res[r][1]) + (res[r + 1][0] + res[r + 1][1]);
                            if ((p & 1) == 0) {
                                racc[r / 2] = s4;
                            } else {
                                const auto rr = plane_rsrc(P.bc_out, cplaneB, p >> 1, true);
                                bstore1(rr, coarse_off(r, xin && vrow[r] && yin[r]), T(0.25) * (racc[r / 2] + s4));
                            }
                        }
                    } else {
                        if (pok && xin) {
#pragma unroll
                            for (int r = 0; r < M; ++r) {
                                if (vrow[r] && yin[r]) {
                                    const double r0 = (double)res[r][0], r1 = (double)res[r][1];
                                    const double b0 = (double)bb[sb][r][0], b1 = (double)bb[sb][r][1];
                                    acc_r2 += r0 * r0 + r1 * r1;
                                    acc_b2 += b0 * b0 + b1 * b1;
                                    const size_t idx = (size_t)p * plane + (size_t)(ybase + r) * nx + xl;
                                    if constexpr (RES == RES_NORM_R32)
                                        store2(P.r32_out + idx, (float)(r0 * inv_sig_next), (float)(r1 * inv_sig_next));
                                    if constexpr (RES == RES_STORE)
                                        if (P.r_out) store2(P.r_out + idx, res[r][0] * P.rscale, res[r][1] * P.rscale);
                                }
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
    }

    if constexpr (RES == RES_NORM || RES == RES_NORM_R32 || RES == RES_STORE) {
        store_partials<64 * WY>(acc_r2, acc_b2, P.partials, blk);
    }
}

// ---------------------------------------------------------------------------
// Coarsest level: conjugate gradients in FP64 by one workgroup (Sec. 5.3),
// search direction resident in LDS.  Solves (S + shift) x = b-tilde from x = 0
// until ||r|| <= rtol ||b|| or maxit, and writes x (as T).
// ---------------------------------------------------------------------------
constexpr int kCgThreads = 256;

template <typename T, int NPT>
__global__ __launch_bounds__(kCgThreads) void k_coarse_cg(const T* b, T* x_out, int nx, int ny, int nz,
                                                          int sh0, int sh1, int sh2, int sh3, int sh4, int sh5,
                                                          double shift, double rtol, int maxit, Ctl* ctl)
{
    if (ctl != nullptr && ctl->done) return;
    __shared__ double pl[kCgThreads * NPT];
    __shared__ double red[2][kCgThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int n = nx * ny * nz;
    double xr[NPT], rr_[NPT], qv[NPT];
    int dg[NPT], nb[NPT][6];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int c = tid + k * kCgThreads;
        const bool v = c < n;
        const int i = v ? c % nx : 0, j = v ? (c / nx) % ny : 0, kk = v ? c / (nx * ny) : 0;
        int d = 6;
        if (i == 0) d += sh0;
        if (i == nx - 1) d += sh1;
        if (j == 0) d += sh2;
        if (j == ny - 1) d += sh3;
        if (kk == 0) d += sh4;
        if (kk == nz - 1) d += sh5;
        dg[k] = v ? d : 0;
        nb[k][0] = (v && i > 0) ? c - 1 : -1;
        nb[k][1] = (v && i < nx - 1) ? c + 1 : -1;
        nb[k][2] = (v && j > 0) ? c - nx : -1;
        nb[k][3] = (v && j < ny - 1) ? c + nx : -1;
        nb[k][4] = (v && kk > 0) ? c - nx * ny : -1;
        nb[k][5] = (v && kk < nz - 1) ? c + nx * ny : -1;
        xr[k] = 0.0;
        rr_[k] = v ? (double)b[c] : 0.0;
        pl[c] = rr_[k];
    }
    auto block_sum = [&](double v, int slot) -> double {
        v = wave_sum(v);
        if (lane == 0) red[slot][w] = v;
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < kCgThreads / 64; ++i) s += red[slot][i];
        return s;
    };
    double loc = 0.0;
#pragma unroll
    for (int k = 0; k < NPT; ++k) loc += rr_[k] * rr_[k];
    double rr = block_sum(loc, 0);
    const double bnorm = sqrt(rr);
    int it = 0;
    if (bnorm > 0.0) {
        while (it < maxit) {
            // q = S p
            double pq = 0.0;
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int c = tid + k * kCgThreads;
                double s = 0.0;
#pragma unroll
                for (int f = 0; f < 6; ++f) s += nb[k][f] >= 0 ? pl[nb[k][f]] : 0.0;
                const double pc = dg[k] ? pl[c] : 0.0;
                qv[k] = dg[k] ? ((double)dg[k] + shift) * pc - s : 0.0;
                pq += pc * qv[k];
            }
            pq = block_sum(pq, 1);
            const double alpha = rr / pq;
            double loc2 = 0.0;
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int c = tid + k * kCgThreads;
                const double pc = dg[k] ? pl[c] : 0.0;
                xr[k] += alpha * pc;
                rr_[k] -= alpha * qv[k];
                loc2 += rr_[k] * rr_[k];
            }
            const double rr_new = block_sum(loc2, 0);
            ++it;
            if (sqrt(rr_new) <= rtol * bnorm) break;
            const double beta = rr_new / rr;
            rr = rr_new;
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int c = tid + k * kCgThreads;
                if (dg[k]) pl[c] = rr_[k] + beta * pl[c];
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int c = tid + k * kCgThreads;
        if (c < n) x_out[c] = (T)xr[k];
    }
    if (tid == 0 && ctl != nullptr) ctl->cg_iters = it;
}

// ---------------------------------------------------------------------------
// Wave-level building blocks for the single-workgroup bottom of the cycle.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Index of cell (i,j,k) in an LDS array with a one-cell zero ghost layer.
__device__ __forceinline__ int padded(int i, int j, int k, int nx, int ny)
{
    return ((k + 1) * (ny + 2) + (j + 1)) * (nx + 2) + (i + 1);
}

// floor(c / d) for 0 <= c < 2^16 and 1 <= d < 2^16 by one high multiply with
// m = ceil(2^32 / d): c m / 2^32 exceeds c / d by less than c / 2^32 < 1 / d,
// too little to reach the next integer.  Replaces the long integer division
// sequence in the index arithmetic of the small-grid kernels.
struct SmallDiv {
    unsigned d, m;
    __device__ explicit SmallDiv(int den) : d((unsigned)den), m(den > 1 ? 0xFFFFFFFFu / (unsigned)den + 1u : 0u) {}
    __device__ __forceinline__ int div(int c) const { return d > 1 ? (int)__umulhi((unsigned)c, m) : c; }
};

// (i, j, k) of the plain index c = (k ny + j) nx + i, with dx = nx, dy = ny
__device__ __forceinline__ void split3(int c, const SmallDiv& dx, const SmallDiv& dy, int& i, int& j, int& k)
{
    const int q = dx.div(c);
    i = c - q * (int)dx.d;
    k = dy.div(q);
    j = q - k * (int)dy.d;
}

__device__ __forceinline__ int cell_diag(int i, int j, int k, int nx, int ny, int nz, const int* sh)
{
    int d = 6;
    if (i == 0) d += sh[0];
    if (i == nx - 1) d += sh[1];
    if (j == 0) d += sh[2];
    if (j == ny - 1) d += sh[3];
    if (k == 0) d += sh[4];
    if (k == nz - 1) d += sh[5];
    return d;
}

// 1/x to full double precision: hardware reciprocal estimate and two Newton
// steps (each doubles the correct bits); no IEEE division sequence on the
// critical path of the one-wave CG.
__device__ __forceinline__ double fast_rcp(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// x + (the value of lane l ^ 16) and x + (lane l ^ 32), the lower lane's value
// first: gfx950's 16- and 32-lane swaps give both operands in every lane.
__device__ __forceinline__ double add_swap16(double x)
{
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(x), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(x), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double add_swap32(double x)
{
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(x), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(x), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double first_lane(double x)
{
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(x)),
                            __builtin_amdgcn_readfirstlane(__double2loint(x)));
}
// Two wave sums over the 64 lanes at once (independent chains interleave),
// the same value in every lane, in a fixed association (deterministic):
// quads, rows of 16 by rotation, then the four row sums of lanes 0, 16, 32
// and 48 combined as (r0 + r1) + (r2 + r3) by the lane swaps, and lane 0's
// result taken.
__device__ __forceinline__ void wave_sum2(double& a, double& b)
{
    a += dpp_d<0xB1>(a); b += dpp_d<0xB1>(b);
    a += dpp_d<0x4E>(a); b += dpp_d<0x4E>(b);
    a += dpp_d<0x124>(a); b += dpp_d<0x124>(b);
    a += dpp_d<0x128>(a); b += dpp_d<0x128>(b);
    a = add_swap16(a); b = add_swap16(b);
    a = add_swap32(a); b = add_swap32(b);
    a = first_lane(a); b = first_lane(b);
}

// Conjugate gradients in FP64 by ONE wave on a level of n <= 512 cells
// (Sec. 5.3: CG on the coarsest grid).  Solves S x = b from x = 0 until
// ||r|| <= rtol ||b|| or maxit.  The recurrences are arranged as in
// Chronopoulos and Gear (1989): the matrix product is taken of the residual,
// and both inner products of an iteration, (r,r) and (r,S r), come from one
// combined reduction; in exact arithmetic the iterates are those of standard
// CG.  The residual lives in LDS with a zero ghost layer (rl,
// (nx+2)(ny+2)(nz+2) doubles, ghosts already zero), so every neighbour read is
// unconditional; b is read with get_b(c) and x written with put_x(c, value),
// c the unpadded index.  No workgroup barrier: the wave's own LDS accesses are
// ordered.
constexpr int kCgWaveMax = 512;

template <typename GetB, typename PutX>
__device__ int cg_one_wave(GetB get_b, PutX put_x, double* rl, int nx, int ny, int nz, const int* sh, double shift,
                           double rtol, int maxit)
{
    constexpr int NPT = kCgWaveMax / 64;
    const int lane = threadIdx.x & 63;
    const int n = nx * ny * nz;
    const int sy = nx + 2, sz = (nx + 2) * (ny + 2);
    double xr[NPT], rv[NPT], pv[NPT], sv[NPT];
    int pc_[NPT], dg[NPT];
    const SmallDiv dx(nx), dy(ny);
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int c = lane + 64 * k;
        const bool v = c < n;
        int i, j, kk;
        split3(v ? c : 0, dx, dy, i, j, kk);
        dg[k] = v ? cell_diag(i, j, kk, nx, ny, nz, sh) : 0;
        // lanes without a cell point at the corner ghost (index 0): they read
        // zeros and only ever store their residual, which stays 0
        pc_[k] = v ? padded(i, j, kk, nx, ny) : 0;
        xr[k] = 0.0;
        pv[k] = 0.0;
        sv[k] = 0.0;
        rv[k] = v ? (double)get_b(c) : 0.0;
        if (v) rl[pc_[k]] = rv[k];
    }
    // Each iteration reduces (r, r) and (r, S r) of the current residual in one
    // combined wave sum; the stopping test on (r, r) therefore sits at the top
    // of the next iteration, after its matrix product (one spare product at
    // the end).  Sums and their order are those of the two-reduction form.
    double gamma_old = 1.0, alpha_old = 1.0, bound = 0.0;
    int it = 0;
    while (true) {
        // w = S r, gamma = (r, r), delta = (w, r)
        double wv[NPT], nbs[NPT][6];
        double gamma = 0.0, delta = 0.0;
        // all neighbour loads first (unconditional), then the arithmetic
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int c = dg[k] ? pc_[k] : sz + sy + 1;   // a ghost-surrounded safe index
            nbs[k][0] = rl[c - 1];
            nbs[k][1] = rl[c + 1];
            nbs[k][2] = rl[c - sy];
            nbs[k][3] = rl[c + sy];
            nbs[k][4] = rl[c - sz];
            nbs[k][5] = rl[c + sz];
        }
#pragma unroll
        for (int k = 0; k < NPT; ++k) gamma += rv[k] * rv[k];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const double sum = ((((nbs[k][0] + nbs[k][1]) + nbs[k][2]) + nbs[k][3]) + nbs[k][4]) + nbs[k][5];
            const double mask = dg[k] ? 1.0 : 0.0;
            wv[k] = mask * (((double)dg[k] + shift) * rv[k] - sum);
            delta += rv[k] * wv[k];
        }
        wave_sum2(gamma, delta);
        if (it == 0) {
            if (!(gamma > 0.0)) break;                // b = 0: x = 0
            bound = rtol * rtol * gamma;              // ||r||^2 <= rtol^2 ||b||^2
        } else if (gamma <= bound) {
            break;
        }
        if (it >= maxit) break;
        const double beta = it == 0 ? 0.0 : gamma * fast_rcp(gamma_old);
        const double alpha = gamma * fast_rcp(delta - beta * gamma * fast_rcp(alpha_old));
        __builtin_amdgcn_wave_barrier();   // all lanes' reads of r precede its update below
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            pv[k] = rv[k] + beta * pv[k];
            sv[k] = wv[k] + beta * sv[k];
            xr[k] += alpha * pv[k];
            rv[k] -= alpha * sv[k];
            rl[pc_[k]] = rv[k];
        }
        __builtin_amdgcn_wave_barrier();
        ++it;
        gamma_old = gamma;
        alpha_old = alpha;
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int c = lane + 64 * k;
        if (c < n) put_x(c, xr[k]);
    }
    return it;
}


// Standalone coarsest-grid CG for n <= 512 cells: one wave.
template <typename T>
__global__ __launch_bounds__(64) void k_coarse_cg_wave(const T* b, T* x_out, int nx, int ny, int nz, int sh0,
                                                       int sh1, int sh2, int sh3, int sh4, int sh5, double shift,
                                                       double rtol, int maxit, Ctl* ctl)
{
    if (ctl != nullptr && ctl->done) return;
    extern __shared__ double pl[];
    const int sh[6] = {sh0, sh1, sh2, sh3, sh4, sh5};
    const int np = (nx + 2) * (ny + 2) * (nz + 2);
    for (int c = threadIdx.x; c < np; c += 64) pl[c] = 0.0;
    __syncthreads();
    const int it = cg_one_wave([&](int c) { return b[c]; }, [&](int c, double v) { x_out[c] = (T)v; }, pl, nx, ny,
                               nz, sh, shift, rtol, maxit);
    if (threadIdx.x == 0 && ctl != nullptr) ctl->cg_iters = it;
}

// ---------------------------------------------------------------------------
// The bottom of the V-cycle in one workgroup.  Levels lb..L-1, where level lb
// has at most 4096 cells, live entirely in LDS (phi with a zero ghost layer,
// b-tilde, the CG direction): one kernel runs the pre-smoothing, residual
// restriction, coarsest CG (one wave), prolongation with the magnified
// correction and post-smoothing of all of them (Sec. 3), reading b-tilde of
// level lb and writing its correction phi (the guess on every coarse level is
// zero).  It replaces two pass launches per level and the CG launch, whose
// cost on such small grids is latency, not bandwidth.
// ---------------------------------------------------------------------------
constexpr int kBottomThreads = 512;
constexpr int kBottomMaxCells = 4096;
constexpr int kBottomMaxLevels = 6;
constexpr int kBottomCpt = kBottomMaxCells / 2 / kBottomThreads;   // cells of one colour per thread

template <typename T>
struct BottomParams {
    const T* b_in;      // b-tilde of level lb (global)
    T* phi_out;         // phi of level lb (global, its home buffer)
    int nlev;           // levels in the bottom (>= 2; the last one is solved by CG)
    int nx[kBottomMaxLevels], ny[kBottomMaxLevels], nz[kBottomMaxLevels];
    int poff[kBottomMaxLevels];   // offsets of the padded phi arrays
    int boff[kBottomMaxLevels];   // offsets of the b-tilde arrays
    int sh[6];
    double shift[kBottomMaxLevels];   // per-level diagonal shift (Poisson-Boltzmann term), 0 for Poisson
    T omega;
    int nu1, nu2;
    double cg_rtol;
    int cg_maxit;
    Ctl* ctl;
};

// LDS footprint (elements of T) of the padded phi and plain b arrays of a bottom
template <typename T>
__host__ __device__ inline void bottom_layout(BottomParams<T>& B, int& nphi, int& nb)
{
    nphi = 0;
    nb = 0;
    for (int l = 0; l < B.nlev; ++l) {
        B.poff[l] = nphi;
        B.boff[l] = nb;
        nphi += (B.nx[l] + 2) * (B.ny[l] + 2) * (B.nz[l] + 2);
        nb += B.nx[l] * B.ny[l] * B.nz[l];
    }
}

// `sweeps` red-black sweeps on one level in LDS; each thread owns fixed cells
// of each colour, their padded index and diagonal computed once per call.
template <typename T>
__device__ void bottom_smooth(T* ph, const T* bt, int nx, int ny, int nz, const int* sh, double shift, int sweeps)
{
    const int hx = nx / 2, half = hx * ny * nz;   // nx even: each colour has half the cells
    const int sy = nx + 2, sz = (nx + 2) * (ny + 2);
    int pidx[2][kBottomCpt], bidx[2][kBottomCpt], dg[2][kBottomCpt];
    const SmallDiv dhx(hx), dny(ny);
#pragma unroll
    for (int colour = 0; colour < 2; ++colour)
#pragma unroll
        for (int u = 0; u < kBottomCpt; ++u) {
            const int m = threadIdx.x + u * kBottomThreads;
            const bool v = m < half;
            int ip, j, k;
            split3(v ? m : 0, dhx, dny, ip, j, k);
            const int i = 2 * ip + ((j + k + colour) & 1);   // entries without a cell only load (cell 0 or 1)
            pidx[colour][u] = padded(i, j, k, nx, ny);
            bidx[colour][u] = (k * ny + j) * nx + i;
            dg[colour][u] = v ? cell_diag(i, j, k, nx, ny, nz, sh) : 0;
        }
    T inv[2][kBottomCpt];
#pragma unroll
    for (int colour = 0; colour < 2; ++colour)
#pragma unroll
        for (int u = 0; u < kBottomCpt; ++u)
            inv[colour][u] = dg[colour][u] ? T(1) / (T(dg[colour][u]) + T(shift)) : T(0);
    for (int sw = 0; sw < sweeps; ++sw) {
#pragma unroll
        for (int colour = 0; colour < 2; ++colour) {
            // loads of every owned cell first, then the updates (cells of one colour are independent)
            T nv[kBottomCpt];
#pragma unroll
            for (int u = 0; u < kBottomCpt; ++u) {
                const int c = pidx[colour][u];
                const T sum = ((((ph[c - 1] + ph[c + 1]) + ph[c - sy]) + ph[c + sy]) + ph[c - sz]) + ph[c + sz];
                nv[u] = (bt[bidx[colour][u]] + sum) * inv[colour][u];
            }
#pragma unroll
            for (int u = 0; u < kBottomCpt; ++u)
                if (dg[colour][u]) ph[pidx[colour][u]] = nv[u];
            __syncthreads();
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBottomThreads) void k_bottom(const BottomParams<T> P)
{
    if (P.ctl != nullptr && P.ctl->done) return;
    extern __shared__ char lds_raw[];
    const int lc = P.nlev - 1;
    // offsets were laid out on the host by bottom_layout
    const int nphi = P.poff[lc] + (P.nx[lc] + 2) * (P.ny[lc] + 2) * (P.nz[lc] + 2);
    const int nb = P.boff[lc] + P.nx[lc] * P.ny[lc] * P.nz[lc];
    T* ph_all = reinterpret_cast<T*>(lds_raw);
    T* b_all = ph_all + nphi;
    double* pl = reinterpret_cast<double*>(lds_raw + (((size_t)(nphi + nb) * sizeof(T) + 7) & ~(size_t)7));
    const int npl = (P.nx[lc] + 2) * (P.ny[lc] + 2) * (P.nz[lc] + 2);
    // zero every phi (ghosts stay zero) and the CG direction
    for (int c = threadIdx.x; c < nphi; c += kBottomThreads) ph_all[c] = T(0);
    for (int c = threadIdx.x; c < npl; c += kBottomThreads) pl[c] = 0.0;
    const int n0 = P.nx[0] * P.ny[0] * P.nz[0];
    {
        // every load issued before the first LDS store, so that the thread
        // waits for one memory latency rather than one per cell (n0 is at
        // most kBottomMaxCells, checked on the host)
        constexpr int kLd = kBottomMaxCells / kBottomThreads;
        T v[kLd];
#pragma unroll
        for (int u = 0; u < kLd; ++u) {
            const int c = threadIdx.x + u * kBottomThreads;
            v[u] = c < n0 ? P.b_in[c] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kLd; ++u) {
            const int c = threadIdx.x + u * kBottomThreads;
            if (c < n0) b_all[c] = v[u];
        }
    }
    __syncthreads();
    // descend
    for (int l = 0; l < lc; ++l) {
        const int nx = P.nx[l], ny = P.ny[l], nz = P.nz[l];
        T* ph = ph_all + P.poff[l];
        const T* bt = b_all + P.boff[l];
        bottom_smooth(ph, bt, nx, ny, nz, P.sh, P.shift[l], P.nu1);
        // b-tilde of level l+1 = 1/4 sum of the children's residuals
        const int cnx = nx / 2, cny = ny / 2, cnz = nz / 2, nc = cnx * cny * cnz;
        const int sy = nx + 2, sz = (nx + 2) * (ny + 2);
        T* bc = b_all + P.boff[l + 1];
        const SmallDiv dcx(cnx), dcy(cny);
        for (int C = threadIdx.x; C < nc; C += kBottomThreads) {
            int I, J, K;
            split3(C, dcx, dcy, I, J, K);
            T acc[2][2];
#pragma unroll
            for (int dk = 0; dk < 2; ++dk)
#pragma unroll
                for (int dj = 0; dj < 2; ++dj) {
                    T pair = T(0);
#pragma unroll
                    for (int di = 0; di < 2; ++di) {
                        const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                        const int c = padded(i, j, k, nx, ny);
                        const T sum =
                            ((((ph[c - 1] + ph[c + 1]) + ph[c - sy]) + ph[c + sy]) + ph[c - sz]) + ph[c + sz];
                        const T r = bt[(k * ny + j) * nx + i] -
                                    ((T(cell_diag(i, j, k, nx, ny, nz, P.sh)) + T(P.shift[l])) * ph[c] - sum);
                        pair = di == 0 ? r : pair + r;
                    }
                    acc[dk][dj] = pair;
                }
            bc[C] = T(0.25) * ((acc[0][0] + acc[0][1]) + (acc[1][0] + acc[1][1]));
        }
        __syncthreads();
    }
    // coarsest level: CG by wave 0, from the b-tilde in LDS into phi's interior
    if (threadIdx.x < 64) {
        const int nx = P.nx[lc], ny = P.ny[lc];
        const T* bt = b_all + P.boff[lc];
        T* ph = ph_all + P.poff[lc];
        const SmallDiv dx(nx), dy(ny);
        const int it = cg_one_wave(
            [&](int c) { return bt[c]; },
            [&](int c, double v) {
                int i, j, k;
                split3(c, dx, dy, i, j, k);
                ph[padded(i, j, k, nx, ny)] = (T)v;
            },
            pl, nx, ny, P.nz[lc], P.sh, P.shift[lc], P.cg_rtol, P.cg_maxit);
        if (threadIdx.x == 0 && P.ctl != nullptr) P.ctl->cg_iters = it;
    }
    __syncthreads();
    // ascend
    for (int l = lc - 1; l >= 0; --l) {
        const int nx = P.nx[l], ny = P.ny[l], nz = P.nz[l], n = nx * ny * nz;
        const int cnx = nx / 2, cny = ny / 2;
        T* ph = ph_all + P.poff[l];
        const T* pc = ph_all + P.poff[l + 1];
        const SmallDiv dx(nx), dy(ny);
        for (int c = threadIdx.x; c < n; c += kBottomThreads) {
            int i, j, k;
            split3(c, dx, dy, i, j, k);
            ph[padded(i, j, k, nx, ny)] += P.omega * pc[padded(i >> 1, j >> 1, k >> 1, cnx, cny)];
        }
        __syncthreads();
        bottom_smooth(ph, b_all + P.boff[l], nx, ny, nz, P.sh, P.shift[l], P.nu2);
    }
    {
        const int nx = P.nx[0], ny = P.ny[0];
        const T* ph = ph_all + P.poff[0];
        const SmallDiv dx(nx), dy(ny);
        for (int c = threadIdx.x; c < n0; c += kBottomThreads) {
            int i, j, k;
            split3(c, dx, dy, i, j, k);
            P.phi_out[c] = ph[padded(i, j, k, nx, ny)];
        }
    }
}

// ---------------------------------------------------------------------------
// Elementwise kernels
// ---------------------------------------------------------------------------

// Finest right-hand side with the boundary terms folded in (Sec. 2.4, Sec. 5.3):
// b-tilde = h^2 (f + sum over the cell's boundary faces of term_f), where
// term_f = 2 g_d / h^2 (Dirichlet) or g_n / h (Neumann), faces added in the
// order x-, x+, y-, y+, z-, z+.  A face with a value array takes g per
// boundary cell: x faces [nz][ny], y faces [nz][nx], z faces [ny][nx].
struct FoldParams {
    const double* f;
    double* bt;
    int nx, ny, nz;
    double h, h2;
    double t[6];              // constant terms of faces without a value array
    const double* face[6];    // per-cell boundary values, or null
    int dirichlet[6];
};

__device__ __forceinline__ double fold_term(const FoldParams& P, int fc, size_t at)
{
#pragma clang fp contract(off)
    if (P.face[fc] == nullptr) return P.t[fc];
    const double g = P.face[fc][at];
    return P.dirichlet[fc] ? 2.0 * g / (P.h * P.h) : g / P.h;
}

// One block per x-row at a time (rows z-major, grid-stride over the nz*ny
// rows): the row's y and z faces are uniform, so only x needs per-cell tests
// and no cell index is divided.  NORM: the block also sums b-tilde^2 over its
// rows and stores it as both norm partials (the residual of the zero guess is
// b-tilde itself), for k_finish_norm in block order.
constexpr int kFoldThreads = 256;
template <bool NORM>
__global__ __launch_bounds__(kFoldThreads) void k_fold(FoldParams P, double* partials)
{
#pragma clang fp contract(off)
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int rows = ny * nz;
    double acc = 0.0;
    for (int row = blockIdx.x; row < rows; row += gridDim.x) {
        const int j = row % ny, k = row / ny;
        const size_t base = (size_t)row * nx;
        for (int i = threadIdx.x; i < nx; i += kFoldThreads) {
            const size_t c = base + i;
            double v = P.f[c];
            if (i == 0) v += fold_term(P, 0, (size_t)k * ny + j);
            if (i == nx - 1) v += fold_term(P, 1, (size_t)k * ny + j);
            if (j == 0) v += fold_term(P, 2, (size_t)k * nx + i);
            if (j == ny - 1) v += fold_term(P, 3, (size_t)k * nx + i);
            if (k == 0) v += fold_term(P, 4, (size_t)j * nx + i);
            if (k == nz - 1) v += fold_term(P, 5, (size_t)j * nx + i);
            const double bt = v * P.h2;
            P.bt[c] = bt;
            if constexpr (NORM) acc += bt * bt;
        }
    }
    if constexpr (NORM) store_partials<kFoldThreads>(acc, acc, partials, blockIdx.x);
}

template <typename T>
__global__ void k_fill(T* a, size_t n, T v)
{
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x)
        a[c] = v;
}

// zero phi when a solve from the zero initial guess stopped before its first
// cycle (zero right-hand side, rtol >= 1, non-finite input): that guess is
// never loaded, so nothing else writes phi then
__global__ void k_zero_if_done(double* a, size_t n, const Ctl* ctl)
{
    if (!ctl->done) return;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x)
        a[c] = 0.0;
}

// zero phi when the finest right-hand side vanished (then phi = 0 is the solution)
__global__ void k_zero_if_bzero(double* a, size_t n, const Ctl* ctl)
{
    if (!ctl->bzero) return;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x)
        a[c] = 0.0;
}

template <typename T>
__global__ void k_copy(const T* src, T* dst, size_t n, const Ctl* ctl)
{
    if (ctl != nullptr && ctl->done) return;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x)
        dst[c] = src[c];
}

// First scaled FP32 residual of a refinement from the zero guess: the
// residual is b-tilde itself, whose norm and scale the initial norm already
// finalised (cycle 0), so the stencil pass reduces to this stream:
// dst = (float)(src / sig_next), and sig_cur takes sig_next, as the
// finalisation of cycle 0 does.
__global__ __launch_bounds__(256) void k_first_r32(const double* __restrict__ src, float* __restrict__ dst, size_t n,
                                                   Ctl* ctl)
{
    if (ctl->done) return;
    const double inv = 1.0 / ctl->sig_next;
    const size_t n2 = n / 2;
    const double2* s2 = reinterpret_cast<const double2*>(src);
    float2* d2 = reinterpret_cast<float2*>(dst);
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n2; c += (size_t)gridDim.x * blockDim.x) {
        const double2 v = s2[c];
        d2[c] = make_float2((float)(v.x * inv), (float)(v.y * inv));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (n & 1) dst[n - 1] = (float)(src[n - 1] * inv);
        ctl->sig_cur = ctl->sig_next;
    }
}

__global__ void k_scale(const double* src, double* dst, size_t n, double a)
{
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x)
        dst[c] = src[c] * a;
}

__global__ void k_ctl_init(Ctl* ctl, double rtol)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->rtol = rtol;
        ctl->bnorm = 0.0;
        ctl->rnorm = 0.0;
        ctl->rel = 0.0;
        ctl->sig_cur = 1.0;
        ctl->sig_next = 1.0;
        ctl->done = 0;
        ctl->status = 0;
        ctl->cycles = 0;
        ctl->bzero = 0;
        ctl->reserved = 0u;
        ctl->cg_iters = 0;
    }
}

// ---------------------------------------------------------------------------
// Poisson-Boltzmann (extension; the outlook of Sec. 9 names the equation for
// charged particles in an electrolyte, with double layers, without writing it
// out).  In the b-tilde scale of the finest level the nonlinear equation
// -Lap(psi) + kappa^2 sinh(psi) = f reads S psi + h^2 kappa^2 sinh(psi) = b-tilde.
// k_pb_residual: r = b-tilde - S psi - h^2 kappa^2 sinh(psi) by x-rows, with
// per-block partials (sum r^2, sum b-tilde^2, max |psi|) for k_pb_finish.
// ---------------------------------------------------------------------------
constexpr int kPbThreads = 256;

struct PbParams {
    const double* psi;
    const double* bt;
    double* r;
    int nx, ny, nz;
    int sh[6];
    double hk2;          // h^2 kappa^2
    double* partials;    // 3 per block
};

__global__ __launch_bounds__(kPbThreads) void k_pb_residual(PbParams P)
{
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int rows = ny * nz;
    const size_t plane = (size_t)nx * ny;
    double r2 = 0.0, b2 = 0.0, m = 0.0;
    for (int row = blockIdx.x; row < rows; row += gridDim.x) {
        const int j = row % ny, k = row / ny;
        const size_t base = (size_t)row * nx;
        for (int i = threadIdx.x; i < nx; i += kPbThreads) {
            const size_t c = base + i;
            const double p = P.psi[c];
            // neighbours in the order x-, x+, y-, y+, z-, z+; outside the domain the
            // face's condition moves to the centre (folded boundary conditions)
            double nb = 0.0;
            int d = 6;
            if (i > 0) nb += P.psi[c - 1]; else d += P.sh[0];
            if (i < nx - 1) nb += P.psi[c + 1]; else d += P.sh[1];
            if (j > 0) nb += P.psi[c - nx]; else d += P.sh[2];
            if (j < ny - 1) nb += P.psi[c + nx]; else d += P.sh[3];
            if (k > 0) nb += P.psi[c - plane]; else d += P.sh[4];
            if (k < nz - 1) nb += P.psi[c + plane]; else d += P.sh[5];
            const double b = P.bt[c];
            const double r = b - ((double)d * p - nb) - P.hk2 * sinh(p);
            P.r[c] = r;
            r2 += r * r;
            b2 += b * b;
            m = fmax(m, fabs(p));
        }
    }
    __shared__ double red[3][kPbThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    r2 = wave_sum(r2);
    b2 = wave_sum(b2);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if (lane == 0) { red[0][w] = r2; red[1][w] = b2; red[2][w] = m; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0, mm = 0.0;
        for (int i = 0; i < kPbThreads / 64; ++i) { a += red[0][i]; b += red[1][i]; mm = fmax(mm, red[2][i]); }
        P.partials[3 * blockIdx.x] = a;
        P.partials[3 * blockIdx.x + 1] = b;
        P.partials[3 * blockIdx.x + 2] = mm;
    }
}

// One block: the partials in block order; relative nonlinear residual of
// step `cycle` into the control block (cycle 0 also records ||b-tilde||).
// done: converged (rel < rtol), b-tilde = 0 (psi = 0 solves it), or not finite.
template <int NT>
__global__ __launch_bounds__(NT) void k_pb_finish(const double* partials, int nblk, Ctl* ctl, int cycle)
{
    __shared__ double red[3][NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double a = 0.0, b = 0.0, m = 0.0;
    for (int i = tid; i < nblk; i += NT) {
        a += partials[3 * i];
        b += partials[3 * i + 1];
        m = fmax(m, partials[3 * i + 2]);
    }
    a = wave_sum(a);
    b = wave_sum(b);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if (lane == 0) { red[0][w] = a; red[1][w] = b; red[2][w] = m; }
    __syncthreads();
    if (tid != 0) return;
    double r2 = 0.0, b2 = 0.0, mm = 0.0;
    for (int i = 0; i < NT / 64; ++i) { r2 += red[0][i]; b2 += red[1][i]; mm = fmax(mm, red[2][i]); }
    const double rn = sqrt(r2), bn = sqrt(b2);
    const bool finite = isfinite(rn) && isfinite(bn) && isfinite(mm);
    const double rel = !finite ? (double)NAN : (bn > 0.0 ? rn / bn : 0.0);
    ctl->rnorm = rn;
    ctl->rel = rel;
    ctl->pb_max = mm;
    if (cycle < kMaxHist) ctl->hist[cycle] = rel;
    ctl->cycles = cycle;
    if (cycle == 0) {
        ctl->bnorm = bn;
        ctl->bzero = finite && bn == 0.0;
    }
    if (!finite) ctl->status = -5;
    ctl->done = !finite || ctl->bzero || !(rel >= ctl->rtol);
}

__global__ void k_axpy(double* y, const double* x, size_t n)
{
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x)
        y[c] += x[c];
}

// ---------------------------------------------------------------------------
// Charged spheres (Sec. 2.4, naive volume mapping)
// ---------------------------------------------------------------------------
constexpr int kSphereThreads = 256;

// Is the centre of cell (i,j,k) in the closed ball?  Same expression and
// order as a plain evaluation, and no contraction, so every implementation
// following the definition selects the same cells.
__device__ __forceinline__ bool cell_in_ball(int i, int j, int k, double h, double cx, double cy, double cz, double R)
{
#pragma clang fp contract(off)
    const double dx = ((double)i + 0.5) * h - cx;
    const double dy = ((double)j + 0.5) * h - cy;
    const double dz = ((double)k + 0.5) * h - cz;
    const double d2 = dx * dx + dy * dy + dz * dz;
    return d2 <= R * R;
}

struct Box { int i0, i1, j0, j1, k0, k1; };

__device__ __forceinline__ void ball_box(double c, double R, double h, int n, int& lo, int& hi)
{
    int a = (int)floor((c - R) / h - 0.5) - 1;
    int b = (int)ceil((c + R) / h - 0.5) + 1;
    lo = a < 0 ? 0 : a;
    hi = b > n - 1 ? n - 1 : b;
}

template <int NT>
__device__ double block_sum_d(double v)
{
    __shared__ double red[NT / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;
}

// one workgroup per sphere: count its cells, then add q/(eps n_s h^3) to each
__global__ __launch_bounds__(kSphereThreads) void k_deposit(const double* centers, const double* radii,
                                                           const double* q, double eps, double h, int nx,
                                                           int ny, int nz, double* f, int* counts)
{
    const int s = blockIdx.x;
    const double cx = centers[3 * s], cy = centers[3 * s + 1], cz = centers[3 * s + 2], R = radii[s];
    Box B;
    ball_box(cx, R, h, nx, B.i0, B.i1);
    ball_box(cy, R, h, ny, B.j0, B.j1);
    ball_box(cz, R, h, nz, B.k0, B.k1);
    const int bx = B.i1 - B.i0 + 1, by = B.j1 - B.j0 + 1, bz = B.k1 - B.k0 + 1;
    const long long nbox = (bx > 0 && by > 0 && bz > 0) ? (long long)bx * by * bz : 0;
    double cnt = 0.0;
    for (long long c = threadIdx.x; c < nbox; c += kSphereThreads) {
        const int i = B.i0 + (int)(c % bx), j = B.j0 + (int)((c / bx) % by), k = B.k0 + (int)(c / ((long long)bx * by));
        cnt += cell_in_ball(i, j, k, h, cx, cy, cz, R) ? 1.0 : 0.0;
    }
    const double ns = block_sum_d<kSphereThreads>(cnt);
    if (threadIdx.x == 0 && counts != nullptr) counts[s] = (int)ns;
    if (ns == 0.0) return;
    double val;
    {
#pragma clang fp contract(off)
        val = q[s] / (eps * ns * h * h * h);
    }
    for (long long c = threadIdx.x; c < nbox; c += kSphereThreads) {
        const int i = B.i0 + (int)(c % bx), j = B.j0 + (int)((c / bx) % by), k = B.k0 + (int)(c / ((long long)bx * by));
        if (cell_in_ball(i, j, k, h, cx, cy, cz, R))
            atomicAdd(&f[((size_t)k * ny + j) * nx + i], val);
    }
}

// dL/dq_s = sum over the sphere's cells of lambda_c / (eps n_s h^3)
__global__ __launch_bounds__(kSphereThreads) void k_dq(const double* centers, const double* radii, double eps,
                                                      double h, int nx, int ny, int nz, const double* lam,
                                                      double* dq)
{
    const int s = blockIdx.x;
    const double cx = centers[3 * s], cy = centers[3 * s + 1], cz = centers[3 * s + 2], R = radii[s];
    Box B;
    ball_box(cx, R, h, nx, B.i0, B.i1);
    ball_box(cy, R, h, ny, B.j0, B.j1);
    ball_box(cz, R, h, nz, B.k0, B.k1);
    const int bx = B.i1 - B.i0 + 1, by = B.j1 - B.j0 + 1, bz = B.k1 - B.k0 + 1;
    const long long nbox = (bx > 0 && by > 0 && bz > 0) ? (long long)bx * by * bz : 0;
    double cnt = 0.0, acc = 0.0;
    for (long long c = threadIdx.x; c < nbox; c += kSphereThreads) {
        const int i = B.i0 + (int)(c % bx), j = B.j0 + (int)((c / bx) % by), k = B.k0 + (int)(c / ((long long)bx * by));
        if (cell_in_ball(i, j, k, h, cx, cy, cz, R)) {
            cnt += 1.0;
            acc += lam[((size_t)k * ny + j) * nx + i];
        }
    }
    const double ns = block_sum_d<kSphereThreads>(cnt);
    const double sum = block_sum_d<kSphereThreads>(acc);
    if (threadIdx.x == 0) {
#pragma clang fp contract(off)
        dq[s] = ns > 0.0 ? sum / (eps * ns * h * h * h) : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Sub-sampled deposition (Sec. 2.4, "Subsampling"): the overlap ratio of a
// cell is the fraction of its SF^3 equidistant sub-cell centres
// ((i + (a + 1/2)/SF) h, ...) inside the closed ball.  The distance test is
// (dx*dx + dy*dy) + dz*dz <= R*R, uncontracted, so every implementation of
// the definition counts the same sub-cells.
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846;

template <int SF>
__device__ __forceinline__ int sub_cells_in_ball(int i, int j, int k, double h, double cx, double cy, double cz,
                                                 double R2)
{
#pragma clang fp contract(off)
    double dx2[SF], dy2[SF], dz2[SF];
#pragma unroll
    for (int a = 0; a < SF; ++a) {
        const double o = ((double)a + 0.5) / (double)SF;
        const double dx = ((double)i + o) * h - cx;
        const double dy = ((double)j + o) * h - cy;
        const double dz = ((double)k + o) * h - cz;
        dx2[a] = dx * dx;
        dy2[a] = dy * dy;
        dz2[a] = dz * dz;
    }
    int cnt = 0;
#pragma unroll
    for (int c = 0; c < SF; ++c)
#pragma unroll
        for (int b = 0; b < SF; ++b)
#pragma unroll
            for (int a = 0; a < SF; ++a) cnt += (dx2[a] + dy2[b] + dz2[c] <= R2) ? 1 : 0;
    return cnt;
}

// charge normalisation of sphere s: spread (q W h^3 = q: the charge is kept)
// or volume (the paper's density q / (4/3 pi R^3) times the overlap ratio)
__device__ __forceinline__ double sphere_norm(int mode, double eps, double W, double R, double h)
{
#pragma clang fp contract(off)
    return mode == 0 ? eps * W * h * h * h : eps * ((4.0 / 3.0) * kPi * R * R * R);
}

// one workgroup per sphere: total sub-cell count W_s SF^3 (an exact integer
// sum), then q_s w_c / norm_s added to every overlapped cell
template <int SF>
__global__ __launch_bounds__(kSphereThreads) void k_deposit_sub(const double* centers, const double* radii,
                                                               const double* q, double eps, double h, int nx,
                                                               int ny, int nz, int mode, double* f,
                                                               double* weights)
{
#pragma clang fp contract(off)
    const int s = blockIdx.x;
    const double cx = centers[3 * s], cy = centers[3 * s + 1], cz = centers[3 * s + 2], R = radii[s];
    const double R2 = R * R;
    Box B;
    ball_box(cx, R, h, nx, B.i0, B.i1);
    ball_box(cy, R, h, ny, B.j0, B.j1);
    ball_box(cz, R, h, nz, B.k0, B.k1);
    const int bx = B.i1 - B.i0 + 1, by = B.j1 - B.j0 + 1, bz = B.k1 - B.k0 + 1;
    const long long nbox = (bx > 0 && by > 0 && bz > 0) ? (long long)bx * by * bz : 0;
    // the counting pass gives W_s: needed for the spread normalisation and when
    // the caller asks for it; the volume normalisation does without (a sphere
    // covering no sub-cell centre then adds nothing either way)
    double W = 0.0;
    if (mode == 0 || weights != nullptr) {
        double cnt = 0.0;
        for (long long c = threadIdx.x; c < nbox; c += kSphereThreads) {
            const int i = B.i0 + (int)(c % bx), j = B.j0 + (int)((c / bx) % by),
                      k = B.k0 + (int)(c / ((long long)bx * by));
            cnt += (double)sub_cells_in_ball<SF>(i, j, k, h, cx, cy, cz, R2);
        }
        W = block_sum_d<kSphereThreads>(cnt) / (double)(SF * SF * SF);
        if (threadIdx.x == 0 && weights != nullptr) weights[s] = W;
        if (W == 0.0) return;
    }
    const double norm = sphere_norm(mode, eps, W, R, h);
    const double qs = q[s];
    for (long long c = threadIdx.x; c < nbox; c += kSphereThreads) {
        const int i = B.i0 + (int)(c % bx), j = B.j0 + (int)((c / bx) % by), k = B.k0 + (int)(c / ((long long)bx * by));
        const int m = sub_cells_in_ball<SF>(i, j, k, h, cx, cy, cz, R2);
        if (m > 0) {
            const double w = (double)m / (double)(SF * SF * SF);
            atomicAdd(&f[((size_t)k * ny + j) * nx + i], qs * w / norm);
        }
    }
}

// dL/dq_s = sum_c lambda_c w_c / norm_s for the sub-sampled deposition;
// accumulate != 0 adds it to the value already in dq[s] (dq[s] + term)
template <int SF>
__global__ __launch_bounds__(kSphereThreads) void k_dq_sub(const double* centers, const double* radii, double eps,
                                                          double h, int nx, int ny, int nz, int mode,
                                                          const double* lam, double* dq, int accumulate)
{
#pragma clang fp contract(off)
    const int s = blockIdx.x;
    const double cx = centers[3 * s], cy = centers[3 * s + 1], cz = centers[3 * s + 2], R = radii[s];
    const double R2 = R * R;
    Box B;
    ball_box(cx, R, h, nx, B.i0, B.i1);
    ball_box(cy, R, h, ny, B.j0, B.j1);
    ball_box(cz, R, h, nz, B.k0, B.k1);
    const int bx = B.i1 - B.i0 + 1, by = B.j1 - B.j0 + 1, bz = B.k1 - B.k0 + 1;
    const long long nbox = (bx > 0 && by > 0 && bz > 0) ? (long long)bx * by * bz : 0;
    double cnt = 0.0, acc = 0.0;
    for (long long c = threadIdx.x; c < nbox; c += kSphereThreads) {
        const int i = B.i0 + (int)(c % bx), j = B.j0 + (int)((c / bx) % by), k = B.k0 + (int)(c / ((long long)bx * by));
        const int m = sub_cells_in_ball<SF>(i, j, k, h, cx, cy, cz, R2);
        if (m > 0) {
            cnt += (double)m;
            acc += lam[((size_t)k * ny + j) * nx + i] * ((double)m / (double)(SF * SF * SF));
        }
    }
    const double W = block_sum_d<kSphereThreads>(cnt) / (double)(SF * SF * SF);
    const double sum = block_sum_d<kSphereThreads>(acc);
    if (threadIdx.x == 0) {
        const double g = (mode == 0 && W == 0.0) ? 0.0 : sum / sphere_norm(mode, eps, W, R, h);
        dq[s] = accumulate ? dq[s] + g : g;
    }
}

// ---------------------------------------------------------------------------
// Potential gradient and electrostatic force (Sec. 2.4, "Coulomb force")
// ---------------------------------------------------------------------------
struct GradBc {
    int nx, ny, nz;
    double h;
    int dirichlet[6];
    double value[6];
    const double* face[6];   // per-cell boundary values, or null
    int per[3];              // periodic axes
};

// indices on periodic axes taken modulo the extent
__device__ __forceinline__ void wrap3(const int* per, int nx, int ny, int nz, int& i, int& j, int& k)
{
    if (per[0]) i = i < 0 ? i + nx : (i >= nx ? i - nx : i);
    if (per[1]) j = j < 0 ? j + ny : (j >= ny ? j - ny : j);
    if (per[2]) k = k < 0 ? k + nz : (k >= nz ? k - nz : k);
}

// phi at (i,j,k), or the ghost value one layer outside across one face:
// Dirichlet 2 g - phi_b, Neumann phi_b + h g_n (g_n the outward derivative)
__device__ __forceinline__ double phi_or_ghost(const double* phi, const GradBc& B, int i, int j, int k)
{
#pragma clang fp contract(off)
    wrap3(B.per, B.nx, B.ny, B.nz, i, j, k);
    int fc = -1, ii = i, jj = j, kk = k;
    if (i < 0) { fc = 0; ii = 0; }
    else if (i >= B.nx) { fc = 1; ii = B.nx - 1; }
    else if (j < 0) { fc = 2; jj = 0; }
    else if (j >= B.ny) { fc = 3; jj = B.ny - 1; }
    else if (k < 0) { fc = 4; kk = 0; }
    else if (k >= B.nz) { fc = 5; kk = B.nz - 1; }
    const double in = phi[((size_t)kk * B.ny + jj) * B.nx + ii];
    if (fc < 0) return in;
    double g = B.value[fc];
    if (B.face[fc] != nullptr) {
        const size_t at = fc < 2 ? (size_t)kk * B.ny + jj : fc < 4 ? (size_t)kk * B.nx + ii : (size_t)jj * B.nx + ii;
        g = B.face[fc][at];
    }
    return B.dirichlet[fc] ? 2.0 * g - in : in + B.h * g;
}

// D3Q19 lattice gradient 3 sum_q w_q phi(x + h c_q) c_q / h (w = 1/18 along
// the axes, 1/36 along the face diagonals) where all 18 neighbours exist,
// D3Q7 central differences with boundary ghosts on the boundary layer
__device__ __forceinline__ void grad_at(const double* phi, const GradBc& B, int i, int j, int k, double& gx,
                                        double& gy, double& gz)
{
#pragma clang fp contract(off)
    const size_t sy = (size_t)B.nx, sz = (size_t)B.nx * B.ny;
    const bool in_x = i > 0 && i < B.nx - 1, in_y = j > 0 && j < B.ny - 1, in_z = k > 0 && k < B.nz - 1;
    if ((in_x || B.per[0]) && (in_y || B.per[1]) && (in_z || B.per[2]) && !(in_x && in_y && in_z)) {
        // D3Q19 across a periodic boundary: neighbours by wrapped index
        auto P = [&](int dx, int dy, int dz) {
            int a = i + dx, b = j + dy, c = k + dz;
            wrap3(B.per, B.nx, B.ny, B.nz, a, b, c);
            return phi[(size_t)c * sz + (size_t)b * sy + a];
        };
        const double ax = P(1, 0, 0) - P(-1, 0, 0), ay = P(0, 1, 0) - P(0, -1, 0), az = P(0, 0, 1) - P(0, 0, -1);
        const double xya = P(1, 1, 0) - P(-1, -1, 0), xyb = P(1, -1, 0) - P(-1, 1, 0);
        const double xza = P(1, 0, 1) - P(-1, 0, -1), xzb = P(1, 0, -1) - P(-1, 0, 1);
        const double yza = P(0, 1, 1) - P(0, -1, -1), yzb = P(0, 1, -1) - P(0, -1, 1);
        const double s = 3.0 / B.h;
        gx = s * (ax * (1.0 / 18.0) + ((xya + xyb) + (xza + xzb)) * (1.0 / 36.0));
        gy = s * (ay * (1.0 / 18.0) + ((xya - xyb) + (yza + yzb)) * (1.0 / 36.0));
        gz = s * (az * (1.0 / 18.0) + ((xza - xzb) + (yza - yzb)) * (1.0 / 36.0));
        return;
    }
    if (in_x && in_y && in_z) {
        const double* p = phi + (k * sz + j * sy + i);
        const double ax = p[1] - p[-1];
        const double ay = p[sy] - p[-(ptrdiff_t)sy];
        const double az = p[sz] - p[-(ptrdiff_t)sz];
        const double xya = p[1 + sy] - p[-1 - (ptrdiff_t)sy];   // (1,1,0) - (-1,-1,0)
        const double xyb = p[1 - (ptrdiff_t)sy] - p[-1 + (ptrdiff_t)sy];   // (1,-1,0) - (-1,1,0)
        const double xza = p[1 + sz] - p[-1 - (ptrdiff_t)sz];
        const double xzb = p[1 - (ptrdiff_t)sz] - p[-1 + (ptrdiff_t)sz];
        const double yza = p[sy + sz] - p[-(ptrdiff_t)sy - (ptrdiff_t)sz];
        const double yzb = p[sy - (ptrdiff_t)sz] - p[-(ptrdiff_t)sy + (ptrdiff_t)sz];
        const double s = 3.0 / B.h;
        gx = s * (ax * (1.0 / 18.0) + ((xya + xyb) + (xza + xzb)) * (1.0 / 36.0));
        gy = s * (ay * (1.0 / 18.0) + ((xya - xyb) + (yza + yzb)) * (1.0 / 36.0));
        gz = s * (az * (1.0 / 18.0) + ((xza - xzb) + (yza - yzb)) * (1.0 / 36.0));
        return;
    }
    const double d = 2.0 * B.h;
    gx = (phi_or_ghost(phi, B, i + 1, j, k) - phi_or_ghost(phi, B, i - 1, j, k)) / d;
    gy = (phi_or_ghost(phi, B, i, j + 1, k) - phi_or_ghost(phi, B, i, j - 1, k)) / d;
    gz = (phi_or_ghost(phi, B, i, j, k + 1) - phi_or_ghost(phi, B, i, j, k - 1)) / d;
}

__global__ void k_gradient(const double* phi, GradBc B, double* grad)
{
    const size_t n = (size_t)B.nx * B.ny * B.nz;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % B.nx), j = (int)((c / B.nx) % B.ny), k = (int)(c / ((size_t)B.nx * B.ny));
        double gx, gy, gz;
        grad_at(phi, B, i, j, k, gx, gy, gz);
        grad[c] = gx;
        grad[n + c] = gy;
        grad[2 * n + c] = gz;
    }
}

// F_s = -h^3 sum_b grad(phi)(x_b) rho_s(x_b), rho_s = q_s w_b / norm_s (the
// sphere's own density of the sub-sampled deposition): one workgroup per
// sphere, one pass over its box
template <int SF>
__global__ __launch_bounds__(kSphereThreads) void k_coulomb(const double* phi, GradBc B, const double* centers,
                                                           const double* radii, const double* q, int mode,
                                                           double* force)
{
#pragma clang fp contract(off)
    const int s = blockIdx.x;
    const double cx = centers[3 * s], cy = centers[3 * s + 1], cz = centers[3 * s + 2], R = radii[s];
    const double R2 = R * R, h = B.h;
    Box X;
    ball_box(cx, R, h, B.nx, X.i0, X.i1);
    ball_box(cy, R, h, B.ny, X.j0, X.j1);
    ball_box(cz, R, h, B.nz, X.k0, X.k1);
    const int bx = X.i1 - X.i0 + 1, by = X.j1 - X.j0 + 1, bz = X.k1 - X.k0 + 1;
    const long long nbox = (bx > 0 && by > 0 && bz > 0) ? (long long)bx * by * bz : 0;
    double cnt = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
    for (long long c = threadIdx.x; c < nbox; c += kSphereThreads) {
        const int i = X.i0 + (int)(c % bx), j = X.j0 + (int)((c / bx) % by), k = X.k0 + (int)(c / ((long long)bx * by));
        const int m = sub_cells_in_ball<SF>(i, j, k, h, cx, cy, cz, R2);
        if (m > 0) {
            double gx, gy, gz;
            grad_at(phi, B, i, j, k, gx, gy, gz);
            const double w = (double)m / (double)(SF * SF * SF);
            cnt += (double)m;
            ax += gx * w;
            ay += gy * w;
            az += gz * w;
        }
    }
    const double W = block_sum_d<kSphereThreads>(cnt) / (double)(SF * SF * SF);
    ax = block_sum_d<kSphereThreads>(ax);
    ay = block_sum_d<kSphereThreads>(ay);
    az = block_sum_d<kSphereThreads>(az);
    if (threadIdx.x == 0) {
        double* F = force + 3 * (size_t)s;
        if (W == 0.0) {
            F[0] = F[1] = F[2] = 0.0;
        } else {
            const double norm = sphere_norm(mode, 1.0, W, R, h);
            const double h3 = h * h * h;
            F[0] = -h3 * ax * q[s] / norm;
            F[1] = -h3 * ay * q[s] / norm;
            F[2] = -h3 * az * q[s] / norm;
        }
    }
}

// Adjoint of the force for a loss with dL/dF_s = gF_s: mu += G_lin^T of
// -h^3 (q_s / norm_s) w_b gF_s at every overlapped cell (the transposed
// D3Q19 / boundary-layer D3Q7 stencil, ghosts contributing their linear part
// -phi_b (Dirichlet) or +phi_b (Neumann)), and direct[s] = gF_s . F_s / q_s.
__device__ __forceinline__ void scatter_grad_t(const GradBc& B, int i, int j, int k, double vx, double vy,
                                               double vz, double* mu)
{
    const size_t sy = (size_t)B.nx, sz = (size_t)B.nx * B.ny;
    const size_t c = (size_t)k * sz + (size_t)j * sy + i;
    const bool in_x = i > 0 && i < B.nx - 1, in_y = j > 0 && j < B.ny - 1, in_z = k > 0 && k < B.nz - 1;
    if ((in_x || B.per[0]) && (in_y || B.per[1]) && (in_z || B.per[2]) && !(in_x && in_y && in_z)) {
        auto A = [&](int dx, int dy, int dz, double v) {
            int a = i + dx, b = j + dy, cc = k + dz;
            wrap3(B.per, B.nx, B.ny, B.nz, a, b, cc);
            atomicAdd(&mu[(size_t)cc * sz + (size_t)b * sy + a], v);
        };
        const double s = 3.0 / B.h;
        const double ax = s * vx * (1.0 / 18.0), ay = s * vy * (1.0 / 18.0), az = s * vz * (1.0 / 18.0);
        const double d = s * (1.0 / 36.0);
        A(1, 0, 0, ax); A(-1, 0, 0, -ax); A(0, 1, 0, ay); A(0, -1, 0, -ay); A(0, 0, 1, az); A(0, 0, -1, -az);
        A(1, 1, 0, d * (vx + vy)); A(-1, -1, 0, -d * (vx + vy)); A(1, -1, 0, d * (vx - vy)); A(-1, 1, 0, -d * (vx - vy));
        A(1, 0, 1, d * (vx + vz)); A(-1, 0, -1, -d * (vx + vz)); A(1, 0, -1, d * (vx - vz)); A(-1, 0, 1, -d * (vx - vz));
        A(0, 1, 1, d * (vy + vz)); A(0, -1, -1, -d * (vy + vz)); A(0, 1, -1, d * (vy - vz)); A(0, -1, 1, -d * (vy - vz));
        return;
    }
    if (in_x && in_y && in_z) {
        const double s = 3.0 / B.h;
        const double ax = s * vx * (1.0 / 18.0), ay = s * vy * (1.0 / 18.0), az = s * vz * (1.0 / 18.0);
        atomicAdd(&mu[c + 1], ax);
        atomicAdd(&mu[c - 1], -ax);
        atomicAdd(&mu[c + sy], ay);
        atomicAdd(&mu[c - sy], -ay);
        atomicAdd(&mu[c + sz], az);
        atomicAdd(&mu[c - sz], -az);
        const double d = s * (1.0 / 36.0);
        atomicAdd(&mu[c + 1 + sy], d * (vx + vy));
        atomicAdd(&mu[c - 1 - sy], -d * (vx + vy));
        atomicAdd(&mu[c + 1 - sy], d * (vx - vy));
        atomicAdd(&mu[c - 1 + sy], -d * (vx - vy));
        atomicAdd(&mu[c + 1 + sz], d * (vx + vz));
        atomicAdd(&mu[c - 1 - sz], -d * (vx + vz));
        atomicAdd(&mu[c + 1 - sz], d * (vx - vz));
        atomicAdd(&mu[c - 1 + sz], -d * (vx - vz));
        atomicAdd(&mu[c + sy + sz], d * (vy + vz));
        atomicAdd(&mu[c - sy - sz], -d * (vy + vz));
        atomicAdd(&mu[c + sy - sz], d * (vy - vz));
        atomicAdd(&mu[c - sy + sz], -d * (vy - vz));
        return;
    }
    const double inv2h = 1.0 / (2.0 * B.h);
    const double v[3] = {vx, vy, vz};
    const int pos[3] = {i, j, k};
    const int n[3] = {B.nx, B.ny, B.nz};
    const size_t st[3] = {1, sy, sz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double cf = v[a] * inv2h;
        const size_t wrapv = (size_t)(n[a] - 1) * st[a];   // periodic: across to the opposite side
        if (pos[a] + 1 < n[a]) atomicAdd(&mu[c + st[a]], cf);
        else if (B.per[a]) atomicAdd(&mu[c - wrapv], cf);
        else atomicAdd(&mu[c], B.dirichlet[2 * a + 1] ? -cf : cf);
        if (pos[a] - 1 >= 0) atomicAdd(&mu[c - st[a]], -cf);
        else if (B.per[a]) atomicAdd(&mu[c + wrapv], -cf);
        else atomicAdd(&mu[c], B.dirichlet[2 * a] ? cf : -cf);
    }
}

template <int SF>
__global__ __launch_bounds__(kSphereThreads) void k_coulomb_adjoint(const double* phi, GradBc B,
                                                                   const double* centers, const double* radii,
                                                                   const double* q, int mode, const double* gF,
                                                                   double* mu, double* direct)
{
#pragma clang fp contract(off)
    const int s = blockIdx.x;
    const double cx = centers[3 * s], cy = centers[3 * s + 1], cz = centers[3 * s + 2], R = radii[s];
    const double R2 = R * R, h = B.h;
    Box X;
    ball_box(cx, R, h, B.nx, X.i0, X.i1);
    ball_box(cy, R, h, B.ny, X.j0, X.j1);
    ball_box(cz, R, h, B.nz, X.k0, X.k1);
    const int bx = X.i1 - X.i0 + 1, by = X.j1 - X.j0 + 1, bz = X.k1 - X.k0 + 1;
    const long long nbox = (bx > 0 && by > 0 && bz > 0) ? (long long)bx * by * bz : 0;
    // pass 1: W_s (the scatter needs the normalisation)
    double cnt = 0.0;
    for (long long c = threadIdx.x; c < nbox; c += kSphereThreads) {
        const int i = X.i0 + (int)(c % bx), j = X.j0 + (int)((c / bx) % by), k = X.k0 + (int)(c / ((long long)bx * by));
        cnt += (double)sub_cells_in_ball<SF>(i, j, k, h, cx, cy, cz, R2);
    }
    const double W = block_sum_d<kSphereThreads>(cnt) / (double)(SF * SF * SF);
    if (W == 0.0) {
        if (threadIdx.x == 0) direct[s] = 0.0;
        return;
    }
    const double pre = -(h * h * h) / sphere_norm(mode, 1.0, W, R, h);
    const double g0 = gF[3 * s], g1 = gF[3 * s + 1], g2 = gF[3 * s + 2], qs = q[s];
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (long long c = threadIdx.x; c < nbox; c += kSphereThreads) {
        const int i = X.i0 + (int)(c % bx), j = X.j0 + (int)((c / bx) % by), k = X.k0 + (int)(c / ((long long)bx * by));
        const int m = sub_cells_in_ball<SF>(i, j, k, h, cx, cy, cz, R2);
        if (m > 0) {
            const double w = (double)m / (double)(SF * SF * SF);
            double gx, gy, gz;
            grad_at(phi, B, i, j, k, gx, gy, gz);
            ax += gx * w;
            ay += gy * w;
            az += gz * w;
            const double f = pre * qs * w;
            scatter_grad_t(B, i, j, k, f * g0, f * g1, f * g2, mu);
        }
    }
    ax = block_sum_d<kSphereThreads>(ax);
    ay = block_sum_d<kSphereThreads>(ay);
    az = block_sum_d<kSphereThreads>(az);
    if (threadIdx.x == 0) direct[s] = pre * (ax * g0 + ay * g1 + az * g2);
}

// ---------------------------------------------------------------------------
// Variable permittivity: -div(eps grad phi) = rho with stored face
// coefficients (Galerkin coarsening with the cell-centred transfers, Sec. 3;
// per-unknown stencils, Sec. 5.3).  Level l's operator is s_l times the
// 7-point stencil with normalised face coefficients k (k = harmonic-mean eps
// on the finest level, the mean of the 4 fine faces on a coarse face):
//     d_c phi_c - sum over in-domain faces k_f phi_n,
//     d_c = sum over in-domain faces k_f + 2 k_f per Dirichlet boundary face.
// Face arrays: x faces [nz][ny][nx+1], y faces [nz][ny+1][nx], z faces
// [nz+1][ny][nx] (face i between cells i-1 and i).
// ---------------------------------------------------------------------------
struct VcLevel {
    const double* kx;
    const double* ky;
    const double* kz;
    int nx, ny, nz;
    int dir[6];   // 1: Dirichlet face
    int per[3];   // periodic axes: the boundary face couples cell n-1 and cell 0
};

// Cell coordinates of a grid-stride loop over c = (k ny + j) nx + i: the start
// and the stride are split once, then every step adds the stride's (i, j, k)
// parts with carries, so the loop body divides nothing (a 64-bit division per
// cell would dominate these memory-light kernels).
struct Walk3 {
    int i, j, k;
    int si, sj, sk, nx, ny;
    __device__ Walk3(size_t c0, size_t stride, int nx_, int ny_) : nx(nx_), ny(ny_)
    {
        const size_t pl = (size_t)nx * ny;
        i = (int)(c0 % nx);
        j = (int)((c0 / nx) % ny);
        k = (int)(c0 / pl);
        si = (int)(stride % nx);
        sj = (int)((stride / nx) % ny);
        sk = (int)(stride / pl);
    }
    __device__ __forceinline__ void next()
    {
        i += si;          // < 2 nx: at most one carry
        j += sj;
        k += sk;
        if (i >= nx) { i -= nx; ++j; }
        if (j >= ny) { j -= ny; ++k; }   // j <= 2 ny - 1 before
    }
};

__device__ __forceinline__ size_t vc_ix(const VcLevel& L, int i, int j, int k)
{
    return ((size_t)k * L.ny + j) * (size_t)(L.nx + 1) + i;
}
__device__ __forceinline__ size_t vc_iy(const VcLevel& L, int i, int j, int k)
{
    return ((size_t)k * (L.ny + 1) + j) * (size_t)L.nx + i;
}
__device__ __forceinline__ size_t vc_iz(const VcLevel& L, int i, int j, int k)
{
    return ((size_t)k * L.ny + j) * (size_t)L.nx + i;
}

// diagonal and weighted neighbour sum of cell (i,j,k)
__device__ __forceinline__ void vc_row(const VcLevel& L, const double* phi, int i, int j, int k, double& d,
                                       double& sum)
{
    const size_t sy = (size_t)L.nx, sz = (size_t)L.nx * L.ny;
    const size_t c = (size_t)k * sz + (size_t)j * sy + i;
    const double kxm = L.kx[vc_ix(L, i, j, k)], kxp = L.kx[vc_ix(L, i + 1, j, k)];
    const double kym = L.ky[vc_iy(L, i, j, k)], kyp = L.ky[vc_iy(L, i, j + 1, k)];
    const double kzm = L.kz[vc_iz(L, i, j, k)], kzp = L.kz[vc_iz(L, i, j, k + 1)];
    const size_t wx = (size_t)(L.nx - 1), wy = (size_t)(L.ny - 1) * sy, wz = (size_t)(L.nz - 1) * sz;
    double dd = 0.0, ss = 0.0;
    if (i > 0) { dd += kxm; ss += kxm * phi[c - 1]; }
    else if (L.per[0]) { dd += kxm; ss += kxm * phi[c + wx]; } else if (L.dir[0]) dd += 2.0 * kxm;
    if (i < L.nx - 1) { dd += kxp; ss += kxp * phi[c + 1]; }
    else if (L.per[0]) { dd += kxp; ss += kxp * phi[c - wx]; } else if (L.dir[1]) dd += 2.0 * kxp;
    if (j > 0) { dd += kym; ss += kym * phi[c - sy]; }
    else if (L.per[1]) { dd += kym; ss += kym * phi[c + wy]; } else if (L.dir[2]) dd += 2.0 * kym;
    if (j < L.ny - 1) { dd += kyp; ss += kyp * phi[c + sy]; }
    else if (L.per[1]) { dd += kyp; ss += kyp * phi[c - wy]; } else if (L.dir[3]) dd += 2.0 * kyp;
    if (k > 0) { dd += kzm; ss += kzm * phi[c - sz]; }
    else if (L.per[2]) { dd += kzm; ss += kzm * phi[c + wz]; } else if (L.dir[4]) dd += 2.0 * kzm;
    if (k < L.nz - 1) { dd += kzp; ss += kzp * phi[c + sz]; }
    else if (L.per[2]) { dd += kzp; ss += kzp * phi[c - wz]; } else if (L.dir[5]) dd += 2.0 * kzp;
    d = dd;
    sum = ss;
}

__device__ __forceinline__ double harmonic_mean(double a, double b) { return 2.0 * a * b / (a + b); }

// finest-level face coefficients from the cell permittivity: one thread per
// face of each orientation (boundary faces take their cell's value)
__global__ void k_vc_faces(const double* eps, double* kx, double* ky, double* kz, int nx, int ny, int nz, int px,
                           int py, int pz)
{
    const size_t nfx = (size_t)(nx + 1) * ny * nz, nfy = (size_t)nx * (ny + 1) * nz, nfz = (size_t)nx * ny * (nz + 1);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    auto E = [&](int i, int j, int k) { return eps[((size_t)k * ny + j) * nx + i]; };
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < nfx + nfy + nfz; t += stride) {
        if (t < nfx) {
            const int i = (int)(t % (nx + 1)), j = (int)((t / (nx + 1)) % ny), k = (int)(t / ((size_t)(nx + 1) * ny));
            kx[t] = (i == 0 || i == nx) ? (px ? harmonic_mean(E(nx - 1, j, k), E(0, j, k)) : E(i == 0 ? 0 : nx - 1, j, k))
                                        : harmonic_mean(E(i - 1, j, k), E(i, j, k));
        } else if (t < nfx + nfy) {
            const size_t u = t - nfx;
            const int i = (int)(u % nx), j = (int)((u / nx) % (ny + 1)), k = (int)(u / ((size_t)nx * (ny + 1)));
            ky[u] = (j == 0 || j == ny) ? (py ? harmonic_mean(E(i, ny - 1, k), E(i, 0, k)) : E(i, j == 0 ? 0 : ny - 1, k))
                                        : harmonic_mean(E(i, j - 1, k), E(i, j, k));
        } else {
            const size_t u = t - nfx - nfy;
            const int i = (int)(u % nx), j = (int)((u / nx) % ny), k = (int)(u / ((size_t)nx * ny));
            kz[u] = (k == 0 || k == nz) ? (pz ? harmonic_mean(E(i, j, nz - 1), E(i, j, 0)) : E(i, j, k == 0 ? 0 : nz - 1))
                                        : harmonic_mean(E(i, j, k - 1), E(i, j, k));
        }
    }
}

// Galerkin coarsening: every coarse face coefficient is the mean of the 4
// fine face coefficients on that face (F: fine level, C: coarse level)
__global__ void k_vc_coarsen(VcLevel F, double* ckx, double* cky, double* ckz, int cnx, int cny, int cnz)
{
    const size_t nfx = (size_t)(cnx + 1) * cny * cnz, nfy = (size_t)cnx * (cny + 1) * cnz,
                 nfz = (size_t)cnx * cny * (cnz + 1);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < nfx + nfy + nfz; t += stride) {
        if (t < nfx) {
            const int I = (int)(t % (cnx + 1)), J = (int)((t / (cnx + 1)) % cny), K = (int)(t / ((size_t)(cnx + 1) * cny));
            ckx[t] = (F.kx[vc_ix(F, 2 * I, 2 * J, 2 * K)] + F.kx[vc_ix(F, 2 * I, 2 * J + 1, 2 * K)] +
                      F.kx[vc_ix(F, 2 * I, 2 * J, 2 * K + 1)] + F.kx[vc_ix(F, 2 * I, 2 * J + 1, 2 * K + 1)]) * 0.25;
        } else if (t < nfx + nfy) {
            const size_t u = t - nfx;
            const int I = (int)(u % cnx), J = (int)((u / cnx) % (cny + 1)), K = (int)(u / ((size_t)cnx * (cny + 1)));
            cky[u] = (F.ky[vc_iy(F, 2 * I, 2 * J, 2 * K)] + F.ky[vc_iy(F, 2 * I + 1, 2 * J, 2 * K)] +
                      F.ky[vc_iy(F, 2 * I, 2 * J, 2 * K + 1)] + F.ky[vc_iy(F, 2 * I + 1, 2 * J, 2 * K + 1)]) * 0.25;
        } else {
            const size_t u = t - nfx - nfy;
            const int I = (int)(u % cnx), J = (int)((u / cnx) % cny), K = (int)(u / ((size_t)cnx * cny));
            ckz[u] = (F.kz[vc_iz(F, 2 * I, 2 * J, 2 * K)] + F.kz[vc_iz(F, 2 * I + 1, 2 * J, 2 * K)] +
                      F.kz[vc_iz(F, 2 * I, 2 * J + 1, 2 * K)] + F.kz[vc_iz(F, 2 * I + 1, 2 * J + 1, 2 * K)]) * 0.25;
        }
    }
}

// b-tilde = h^2 (f + boundary terms): Dirichlet 2 k_f g / h^2, Neumann k_f g_n / h,
// per-cell face values when given, faces added in the order x-, x+, y-, y+, z-, z+
struct VcFold {
    const double* f;
    double* bt;
    double h;
    double value[6];
    const double* face[6];
    int homogeneous;
};

__device__ __forceinline__ double vc_bterm(const VcFold& P, const VcLevel& L, int fc, size_t at, double kf)
{
    if (P.homogeneous || L.per[fc / 2]) return 0.0;
    const double g = P.face[fc] != nullptr ? P.face[fc][at] : P.value[fc];
    return L.dir[fc] ? 2.0 * kf * g / (P.h * P.h) : kf * g / P.h;
}

__global__ void k_vc_fold(VcFold P, VcLevel L)
{
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const size_t n = (size_t)nx * ny * nz;
    const size_t c0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    Walk3 w(c0, stride, nx, ny);
    for (size_t c = c0; c < n; c += stride, w.next()) {
        const int i = w.i, j = w.j, k = w.k;
        double v = P.f[c];
        if (i == 0) v += vc_bterm(P, L, 0, (size_t)k * ny + j, L.kx[vc_ix(L, 0, j, k)]);
        if (i == nx - 1) v += vc_bterm(P, L, 1, (size_t)k * ny + j, L.kx[vc_ix(L, nx, j, k)]);
        if (j == 0) v += vc_bterm(P, L, 2, (size_t)k * nx + i, L.ky[vc_iy(L, i, 0, k)]);
        if (j == ny - 1) v += vc_bterm(P, L, 3, (size_t)k * nx + i, L.ky[vc_iy(L, i, ny, k)]);
        if (k == 0) v += vc_bterm(P, L, 4, (size_t)j * nx + i, L.kz[vc_iz(L, i, j, 0)]);
        if (k == nz - 1) v += vc_bterm(P, L, 5, (size_t)j * nx + i, L.kz[vc_iz(L, i, j, nz)]);
        P.bt[c] = v * (P.h * P.h);
    }
}

// one colour of a red-black Gauss-Seidel sweep (red = (i+j+k) even):
// phi_c <- (b~_c + sum k_f phi_n) / d_c
__global__ void k_vc_sweep(VcLevel L, double* phi, const double* bt, int colour, const Ctl* ctl)
{
    if (ctl != nullptr && ctl->done) return;
    const int nx = L.nx, ny = L.ny;
    const int hx = (nx + 1) / 2;                      // cells of one colour per row (at most)
    const size_t total = (size_t)hx * ny * L.nz;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    Walk3 w(t0, stride, hx, ny);   // (m, j, k): the m-th cell of the colour in row (j, k)
    for (size_t t = t0; t < total; t += stride, w.next()) {
        const int j = w.j, k = w.k;
        const int i = 2 * w.i + ((j + k + colour) & 1);
        if (i >= nx) continue;
        double d, sum;
        vc_row(L, phi, i, j, k, d, sum);
        const size_t c = ((size_t)k * ny + j) * nx + i;
        phi[c] = (bt[c] + sum) / d;
    }
}

// residual of the 8 children of every coarse cell, averaged into the coarse
// b-tilde (b~_{l+1} = (1/4) sum of the children's r~ = r / s_l, since
// s_{l+1} = s_l / 2 and R averages), and the coarse initial guess set to zero
__global__ void k_vc_restrict(VcLevel L, const double* phi, const double* bt, double* bc, double* phic,
                              const Ctl* ctl)
{
    if (ctl != nullptr && ctl->done) return;
    const int cnx = L.nx / 2, cny = L.ny / 2, cnz = L.nz / 2;
    const size_t nc = (size_t)cnx * cny * cnz;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    Walk3 w(t0, stride, cnx, cny);
    for (size_t t = t0; t < nc; t += stride, w.next()) {
        const int I = w.i, J = w.j, K = w.k;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = 2 * K + (q >> 2);
            const size_t c = ((size_t)k * L.ny + j) * L.nx + i;
            double d, sum;
            vc_row(L, phi, i, j, k, d, sum);
            acc += bt[c] - (d * phi[c] - sum);
        }
        bc[t] = 0.25 * acc;
        phic[t] = 0.0;
    }
}

// nearest-neighbour prolongation with the magnified correction
__global__ void k_vc_prolong(double* phi, const double* ec, int nx, int ny, int nz, double omega, const Ctl* ctl)
{
    if (ctl != nullptr && ctl->done) return;
    const int cnx = nx / 2, cny = ny / 2;
    const size_t n = (size_t)nx * ny * nz;
    const size_t c0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    Walk3 w(c0, stride, nx, ny);
    for (size_t c = c0; c < n; c += stride, w.next()) {
        const int i = w.i, j = w.j, k = w.k;
        phi[c] += omega * ec[((size_t)(k >> 1) * cny + (j >> 1)) * cnx + (i >> 1)];
    }
}

// finest residual norm (and ||b~||) as block partials for k_finish_norm (grid-stride form:
// periodic axes, residual output); r_out (nullable) receives the residual times rscale
constexpr int kVcNormThreads = 256;
__global__ __launch_bounds__(kVcNormThreads) void k_vc_norm(VcLevel L, const double* phi, const double* bt,
                                                           double* r_out, double rscale, double* partials, Ctl* ctl,
                                                           int fin, int cycle)
{
    if (fin == FIN_CYCLE && ctl->done) return;
    const int nx = L.nx, ny = L.ny;
    const size_t n = (size_t)nx * ny * L.nz;
    double r2 = 0.0, b2 = 0.0;
    const size_t c0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    Walk3 w(c0, stride, nx, ny);
    for (size_t c = c0; c < n; c += stride, w.next()) {
        double d, sum;
        vc_row(L, phi, w.i, w.j, w.k, d, sum);
        const double r = bt[c] - (d * phi[c] - sum);
        r2 += r * r;
        b2 += bt[c] * bt[c];
        if (r_out != nullptr) r_out[c] = r * rscale;
    }
    store_partials<kVcNormThreads>(r2, b2, partials, (int)blockIdx.x);
}

// One red-black Gauss-Seidel sweep on the stored stencil in a single pass
// (variable permittivity without periodic axes).  The z-marching scheme of
// k_pass with two stages, red on plane t-1 and black on plane t-2: a lane
// holds an x-pair, and the face coefficients of its rows travel in register
// rings beside phi and b-tilde, so a sweep reads phi, b-tilde and the three
// face arrays once instead of once per colour.  The arithmetic is that of
// k_vc_sweep: d = the in-domain faces' k plus 2k per Dirichlet boundary face
// (face weights 1, 2 or 0, exact), the neighbour sum, both in the order x-,
// x+, y-, y+, z-, z+, and phi = (b-tilde + sum) / d.
struct VcPassParams {
    VcLevel L;
    const double* phi_in;
    double* phi_out;
    const double* b;
    const double* ec;    // PROLONG: correction of level l+1, added as omega * e(parent) on loading
    double omega;
    const Ctl* ctl;
    int zc, tiles_x, tiles_y, zchunks;
};
constexpr int kVcPassWaves = 8;
constexpr int kVcPassRows = 2;
constexpr int kVcPassTX = 64 - 2 * 2;                                // x halo 2 (two stages)
constexpr int kVcPassTY = 2 * kVcPassWaves * kVcPassRows - 2 * 2;   // y halo 2

template <bool PROLONG>
__global__ __launch_bounds__(64 * kVcPassWaves, 1) void k_vc_pass(VcPassParams P)
{
    // No implicit fusion of products and sums (the same reason as in k_pass:
    // the unrolled copies of a stage must round alike); the fused forms are
    // written out.
#pragma clang fp contract(off)
    using T = double;
    constexpr int M = kVcPassRows, WY = kVcPassWaves, S = 2, H = 2, HY = 2;
    constexpr int NSTRIP = 2 * WY, TX = kVcPassTX, TY = kVcPassTY;
    constexpr int RP = 4, RF = 3, U = 12;   // ring lengths (b-tilde and faces share RF); U = lcm(RP, RF, 2)
    if (P.ctl != nullptr && P.ctl->done) return;

    // strip-edge exchange as in k_pass: [stage input][step parity][strip + 1][edge row][pair]
    __shared__ T edge1[S][2][NSTRIP + 2][2][32];
    for (int e = threadIdx.x; e < S * 2 * 2 * 2 * 32; e += 64 * WY) {
        const int xp_ = e & 31, row = (e >> 5) & 1, pad = (e >> 6) & 1, rest = e >> 7;
        edge1[rest >> 1][rest & 1][pad ? NSTRIP + 1 : 0][row][xp_] = T(0);
    }
    __syncthreads();

    const VcLevel& L = P.L;
    const int nblk = P.tiles_x * P.tiles_y * P.zchunks;
    const int blk = xcd_block_id(nblk);
    const int bx = blk % P.tiles_x;
    const int by = (blk / P.tiles_x) % P.tiles_y;
    const int bz = blk / (P.tiles_x * P.tiles_y);
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int xp = lane & 31;
    const int strip = 2 * w + (lane >> 5);
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int xl = bx * TX - H + 2 * xp;
    const int ybase = by * TY - HY + strip * M;   // even
    const int z0 = bz * P.zc;
    const int z1 = min(nz, z0 + P.zc);
    const bool vx = (xl >= 0) && (xl < nx);
    const bool xin = (xp >= H / 2) && (xp < H / 2 + TX / 2);

    auto wb = [&](int f) { return L.dir[f] ? T(2) : T(0); };   // boundary face weight
    bool vrow[M], yin[M];
    // face weights of the in-domain cells: x and y of the pair and of row 0 are
    // even and the dims are even, so only the x- face of cell 0, the x+ face of
    // cell 1, the y- face of row 0 and the y+ face of row 1 can lie on the
    // boundary; every other weight is 1
    const T wx0 = xl == 0 ? wb(0) : T(1), wx1 = xl + 1 == nx - 1 ? wb(1) : T(1);
    const T wy0 = ybase == 0 ? wb(2) : T(1), wy1 = ybase + 1 == ny - 1 ? wb(3) : T(1);
    static_assert(M == 2, "the boundary weights assume two rows per thread");
    const size_t planeP = (size_t)nx * ny * sizeof(T);         // phi, b-tilde, one z-face plane
    const size_t planeX = (size_t)(nx + 1) * ny * sizeof(T);   // x faces of one plane
    const size_t planeY = (size_t)nx * (ny + 1) * sizeof(T);   // y faces of one plane
    unsigned offP[M], offS[M], offX[M], offX1[M], offY[M + 1];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const int y = ybase + r;
        vrow[r] = vx && (y >= 0) && (y < ny);
        const int ry = strip * M + r;
        yin[r] = (ry >= HY) && (ry < HY + TY);
        offP[r] = vrow[r] ? (unsigned)((y * nx + xl) * (int)sizeof(T)) : kOob;
        offS[r] = (vrow[r] && yin[r] && xin) ? offP[r] : kOob;
        // x faces xl and xl + 1, also for the lane just beyond the domain's last
        // cell (xl = nx), whose face xl is the domain's x+ boundary face
        const bool vf = (xl >= 0) && (xl <= nx) && (y >= 0) && (y < ny);
        offX[r] = vf ? (unsigned)((y * (nx + 1) + xl) * (int)sizeof(T)) : kOob;
        offX1[r] = (vf && xl + 1 <= nx) ? offX[r] + (unsigned)sizeof(T) : kOob;
    }
#pragma unroll
    for (int r = 0; r <= M; ++r) {   // y faces below rows 0..M-1 and above row M-1
        const int y = ybase + r;
        offY[r] = (vx && y >= 0 && y <= ny) ? (unsigned)((y * nx + xl) * (int)sizeof(T)) : kOob;
    }

    // rings: phi (planes t-3..t), b-tilde and faces (planes t-2..t); per row the
    // x faces xl, xl+1 (face xl+2 from the next lane), the y faces below the
    // rows and above the last, the z faces below the plane
    T ph[RP][M][2], bb[RF][M][2], fx[RF][M][2], fy[RF][M + 1][2], fz[RF][M][2];
#pragma unroll
    for (int q = 0; q < RP; ++q)
#pragma unroll
        for (int r = 0; r < M; ++r) ph[q][r][0] = ph[q][r][1] = T(0);
    // phi and the z faces of plane t are read in the step in which the plane
    // enters (stage 1 of that step needs them as plane t-1's upper neighbours):
    // they are requested one step ahead into nph / nfz.  b-tilde and the x and
    // y faces are first read one step later: they are loaded straight into
    // their ring slot at the end of the previous step, after stage 2 has
    // finished with the plane that slot held.
    T nph[M][2], nfz[M][2];
    // PROLONG: the parent (level l+1) of the pair's rows; planes 2k and 2k+1
    // share it, so even planes load it (nex) and odd planes reuse it (elast)
    const int cnx = nx >> 1, cny = ny >> 1;
    const size_t cplaneP = (size_t)cnx * cny * sizeof(T);
    const unsigned offE = vrow[0] ? (unsigned)(((ybase >> 1) * cnx + (xl >> 1)) * (int)sizeof(T)) : kOob;
    T nex = T(0), elast = T(0);
    auto load_early = [&](int t, bool even) {
        const bool zin = (t >= 0) && (t < nz);
        const bool zinf = (t >= 0) && (t <= nz);   // z faces: nz + 1 planes
        const auto rp = plane_rsrc(P.phi_in, planeP, t, zin && P.phi_in != nullptr);   // null: zero guess
        const auto rz = plane_rsrc(L.kz, planeP, t, zinf);
#pragma unroll
        for (int r = 0; r < M; ++r) {
            bload2(rp, offP[r], nph[r][0], nph[r][1]);
            bload2(rz, offP[r], nfz[r][0], nfz[r][1]);
        }
        if constexpr (PROLONG)
            if (even) bload1(plane_rsrc(P.ec, cplaneP, t >> 1, zin), offE, nex);
    };
    auto load_late = [&](int t, int slot) {
        const bool zin = (t >= 0) && (t < nz);
        const auto rb = plane_rsrc(P.b, planeP, t, zin);
        const auto rx = plane_rsrc(L.kx, planeX, t, zin);
        const auto ry = plane_rsrc(L.ky, planeY, t, zin);
#pragma unroll
        for (int r = 0; r < M; ++r) {
            bload2(rb, offP[r], bb[slot][r][0], bb[slot][r][1]);
            bload1(rx, offX[r], fx[slot][r][0]);
            bload1(rx, offX1[r], fx[slot][r][1]);
        }
#pragma unroll
        for (int r = 0; r <= M; ++r) bload2(ry, offY[r], fy[slot][r][0], fy[slot][r][1]);
    };

    const int tbeg = z0 - S, tend = z1 + S;   // tbeg even (z0 even, S = 2): plane t has the parity of q
    load_early(tbeg, true);
    load_late(tbeg, 0);
    for (int tb = tbeg; tb < tend; tb += U) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int t = tb + q;
            if (t < tend) {
                const int par = t & 1;
                // ---- stage 0: plane t enters the rings; plane t + 1 is requested
                {
                    const int s0 = q % RP, sf0 = q % RF;
                    if constexpr (PROLONG)
                        if ((q & 1) == 0) elast = nex;
#pragma unroll
                    for (int r = 0; r < M; ++r) {
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            ph[s0][r][c] = PROLONG ? fma(P.omega, elast, nph[r][c]) : nph[r][c];
                            fz[sf0][r][c] = nfz[r][c];
                        }
                    }
                    if (t + 1 < tend) load_early(t + 1, (q & 1) == 1);
                    const int ppar = q & 1;   // parity of plane t
                    // black cells of the edge rows: the neighbours the red stage needs
                    edge1[0][par][strip + 1][0][xp] = ph[s0][0][(1 + 0 + ppar) & 1];
                    edge1[0][par][strip + 1][1][xp] = ph[s0][M - 1][(1 + (M - 1) + ppar) & 1];
                }
                T e_lo[S], e_hi[S];
#pragma unroll
                for (int s = 1; s <= S; ++s) {
                    const T* ein = &edge1[s - 1][par ^ 1][0][0][0];
                    e_lo[s - 1] = ein[(strip * 2 + 1) * 32 + xp];
                    e_hi[s - 1] = ein[((strip + 2) * 2 + 0) * 32 + xp];
                }
                // ---- stages 1 (red) and 2 (black)
#pragma unroll
                for (int s = 1; s <= S; ++s) {
                    const int p = t - s;
                    const int sc = (q - s + 2 * U) % RP;
                    const int sm = (q - s - 1 + 2 * U) % RP;
                    const int sp = (q - s + 1 + 2 * U) % RP;
                    const int sf = (q - s + 2 * U) % RF;
                    const int sfp = (q - s + 1 + 2 * U) % RF;   // faces of plane p + 1 (its lower z face)
                    const int cs = (s + 1) & 1;
                    const int ppar = (q - s) & 1;
                    if (p < z0 - (S - s) || p >= z1 + (S - s)) continue;
                    if (p < 0 || p >= nz) continue;   // planes outside the domain stay zero
                    const T wzm = p == 0 ? wb(4) : T(1);
                    const T wzp = p == nz - 1 ? wb(5) : T(1);
#pragma unroll
                    for (int r = 0; r < M; ++r) {
                        const int o = (cs + r + ppar) & 1;
                        T xm, xq;
                        if (o == 0) { xm = lane_prev(ph[sc][r][1]); xq = ph[sc][r][1]; }
                        else        { xm = ph[sc][r][0]; xq = lane_next(ph[sc][r][0]); }
                        const T kxm = fx[sf][r][o], kxp = o == 0 ? fx[sf][r][1] : lane_next(fx[sf][r][0]);
                        const T ym = r > 0 ? ph[sc][r - 1][o] : e_lo[s - 1];
                        const T yq = r < M - 1 ? ph[sc][r + 1][o] : e_hi[s - 1];
                        const T kym = fy[sf][r][o], kyp = fy[sf][r + 1][o];
                        const T kzm = fz[sf][r][o], kzp = fz[sfp][r][o];
                        T dd = (o == 0 ? wx0 : T(1)) * kxm;
                        dd = fma(o == 1 ? wx1 : T(1), kxp, dd);
                        dd = fma(r == 0 ? wy0 : T(1), kym, dd);
                        dd = fma(r == 1 ? wy1 : T(1), kyp, dd);
                        dd = fma(wzm, kzm, dd);
                        dd = fma(wzp, kzp, dd);
                        // neighbours outside the domain are zero: their terms add nothing
                        T ss = kxm * xm;
                        ss = fma(kxp, xq, ss);
                        ss = fma(kym, ym, ss);
                        ss = fma(kyp, yq, ss);
                        ss = fma(kzm, ph[sm][r][o], ss);
                        ss = fma(kzp, ph[sp][r][o], ss);
                        const T nv = (bb[sf][r][o] + ss) / dd;
                        ph[sc][r][o] = vrow[r] ? nv : T(0);   // cells outside the domain have d = 0
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    if (s < S) {
                        edge1[s][par][strip + 1][0][xp] = ph[sc][0][(cs + 0 + ppar) & 1];
                        edge1[s][par][strip + 1][1][xp] = ph[sc][M - 1][(cs + (M - 1) + ppar) & 1];
                    }
                }
                // ---- output of the swept plane t - 2
                {
                    const int po = t - S;
                    if (po >= z0 && po < z1) {
                        const int so = (q - S + 2 * U) % RP;
                        const auto rs = plane_rsrc(P.phi_out, planeP, po, true);
#pragma unroll
                        for (int r = 0; r < M; ++r) bstore2(rs, offS[r], ph[so][r][0], ph[so][r][1]);
                    }
                }
                if (t + 1 < tend) load_late(t + 1, (q + 1) % RF);
                __syncthreads();
            }
        }
    }
}

// The stored-stencil residual r = b-tilde - (d phi - sum k phi_nb) of every
// cell in one z-marching pass (same layout, descriptors and strip-edge
// exchange as k_vc_pass, one stage: the residual of plane t-1 at step t),
// either restricted (RESTRICT: b-tilde of level l+1 = 1/4 of the sum over the
// 8 children, the coarse phi set to zero) or reduced to block partials of
// ||r||^2 and ||b-tilde||^2 for k_finish_norm.
struct VcResParams {
    VcLevel L;
    const double* phi;
    const double* b;
    double* bc_out;      // RESTRICT: b-tilde of level l+1
    double* phic;        // RESTRICT: phi of level l+1 (zeroed)
    double* partials;    // norm: 2 doubles per block
    const Ctl* ctl;
    int fin;             // norm: FIN_CYCLE skips when ctl->done
    int zc, tiles_x, tiles_y, zchunks;
};

template <bool RESTRICT>
__global__ __launch_bounds__(64 * kVcPassWaves, 1) void k_vc_res(VcResParams P)
{
    // No implicit fusion of products and sums (the same reason as in k_pass:
    // the unrolled copies of a stage must round alike); the fused forms are
    // written out.
#pragma clang fp contract(off)
    using T = double;
    constexpr int M = kVcPassRows, WY = kVcPassWaves, S = 1, H = 2, HY = 2;
    constexpr int NSTRIP = 2 * WY, TX = kVcPassTX, TY = kVcPassTY;
    constexpr int RP = 4, RF = 2, U = 4;   // phi: planes t-3..t (t-2..t used); b-tilde, faces: t-1, t
    if (RESTRICT ? (P.ctl != nullptr && P.ctl->done) : (P.fin == FIN_CYCLE && P.ctl->done)) return;

    // both cells of the edge rows of the plane that entered in the previous step
    __shared__ T edge2[2][NSTRIP + 2][2][32][2];
    for (int e = threadIdx.x; e < 2 * 2 * 2 * 32 * 2; e += 64 * WY) {
        const int c = e & 1, xp_ = (e >> 1) & 31, row = (e >> 6) & 1, pad = (e >> 7) & 1, par_ = e >> 8;
        edge2[par_][pad ? NSTRIP + 1 : 0][row][xp_][c] = T(0);
    }
    __syncthreads();

    const VcLevel& L = P.L;
    const int nblk = P.tiles_x * P.tiles_y * P.zchunks;
    const int blk = xcd_block_id(nblk);
    const int bx = blk % P.tiles_x;
    const int by = (blk / P.tiles_x) % P.tiles_y;
    const int bz = blk / (P.tiles_x * P.tiles_y);
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int xp = lane & 31;
    const int strip = 2 * w + (lane >> 5);
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int xl = bx * TX - H + 2 * xp;
    const int ybase = by * TY - HY + strip * M;   // even
    const int z0 = bz * P.zc;
    const int z1 = min(nz, z0 + P.zc);
    const bool vx = (xl >= 0) && (xl < nx);
    const bool xin = (xp >= H / 2) && (xp < H / 2 + TX / 2);

    auto wb = [&](int f) { return L.dir[f] ? T(2) : T(0); };
    const T wx0 = xl == 0 ? wb(0) : T(1), wx1 = xl + 1 == nx - 1 ? wb(1) : T(1);
    const T wy0 = ybase == 0 ? wb(2) : T(1), wy1 = ybase + 1 == ny - 1 ? wb(3) : T(1);
    static_assert(M == 2, "the boundary weights and the restriction assume two rows per thread");
    bool vrow[M], own[M];
    const size_t planeP = (size_t)nx * ny * sizeof(T);
    const size_t planeX = (size_t)(nx + 1) * ny * sizeof(T);
    const size_t planeY = (size_t)nx * (ny + 1) * sizeof(T);
    unsigned offP[M], offX[M], offX1[M], offY[M + 1];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const int y = ybase + r;
        vrow[r] = vx && (y >= 0) && (y < ny);
        const int ry = strip * M + r;
        own[r] = vrow[r] && xin && (ry >= HY) && (ry < HY + TY);
        offP[r] = vrow[r] ? (unsigned)((y * nx + xl) * (int)sizeof(T)) : kOob;
        const bool vf = (xl >= 0) && (xl <= nx) && (y >= 0) && (y < ny);
        offX[r] = vf ? (unsigned)((y * (nx + 1) + xl) * (int)sizeof(T)) : kOob;
        offX1[r] = (vf && xl + 1 <= nx) ? offX[r] + (unsigned)sizeof(T) : kOob;
    }
#pragma unroll
    for (int r = 0; r <= M; ++r) {
        const int y = ybase + r;
        offY[r] = (vx && y >= 0 && y <= ny) ? (unsigned)((y * nx + xl) * (int)sizeof(T)) : kOob;
    }
    // the coarse cell of the pair's rows (0, 1): written by the owning lanes
    const int cnx = nx >> 1, cny = ny >> 1;
    const size_t cplane = (size_t)cnx * cny * sizeof(T);
    const unsigned offC = own[0] ? (unsigned)(((ybase >> 1) * cnx + (xl >> 1)) * (int)sizeof(T)) : kOob;

    T ph[RP][M][2], bb[RF][M][2], fx[RF][M][2], fy[RF][M + 1][2], fz[RF][M][2];
#pragma unroll
    for (int q = 0; q < RP; ++q)
#pragma unroll
        for (int r = 0; r < M; ++r) ph[q][r][0] = ph[q][r][1] = T(0);
    T nph[M][2], nfz[M][2];
    auto load_early = [&](int t) {
        const bool zin = (t >= 0) && (t < nz);
        const bool zinf = (t >= 0) && (t <= nz);
        const auto rp = plane_rsrc(P.phi, planeP, t, zin && P.phi != nullptr);   // null: zero guess
        const auto rz = plane_rsrc(L.kz, planeP, t, zinf);
#pragma unroll
        for (int r = 0; r < M; ++r) {
            bload2(rp, offP[r], nph[r][0], nph[r][1]);
            bload2(rz, offP[r], nfz[r][0], nfz[r][1]);
        }
    };
    auto load_late = [&](int t, int slot) {
        const bool zin = (t >= 0) && (t < nz);
        const auto rb = plane_rsrc(P.b, planeP, t, zin);
        const auto rx = plane_rsrc(L.kx, planeX, t, zin);
        const auto ry = plane_rsrc(L.ky, planeY, t, zin);
#pragma unroll
        for (int r = 0; r < M; ++r) {
            bload2(rb, offP[r], bb[slot][r][0], bb[slot][r][1]);
            bload1(rx, offX[r], fx[slot][r][0]);
            bload1(rx, offX1[r], fx[slot][r][1]);
        }
#pragma unroll
        for (int r = 0; r <= M; ++r) bload2(ry, offY[r], fy[slot][r][0], fy[slot][r][1]);
    };

    double acc_r2 = 0.0, acc_b2 = 0.0;
    T racc = T(0);
    const int tbeg = z0 - S - 1, tend = z1 + S;   // tbeg even: plane z0 - 1 enters first (the residual needs z0 - 1)
    load_early(tbeg);
    load_late(tbeg, 0);
    for (int tb = tbeg; tb < tend; tb += U) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int t = tb + q;
            if (t < tend) {
                const int par = t & 1;
                {
                    const int s0 = q % RP, sf0 = q % RF;
#pragma unroll
                    for (int r = 0; r < M; ++r) {
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            ph[s0][r][c] = nph[r][c];
                            fz[sf0][r][c] = nfz[r][c];
                        }
                    }
                    if (t + 1 < tend) load_early(t + 1);
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        edge2[par][strip + 1][0][xp][c] = ph[s0][0][c];
                        edge2[par][strip + 1][1][xp][c] = ph[s0][M - 1][c];
                    }
                }
                // ---- the residual of plane p = t - 1
                const int p = t - 1;
                if (p >= z0 && p < z1) {
                    const int sc = (q - 1 + 2 * U) % RP, sm = (q - 2 + 2 * U) % RP, sp = q % RP;
                    const int sf = (q - 1 + 2 * U) % RF;
                    const int szm = sf, szp = q % RF;   // z faces below plane p and below plane p + 1
                    const T wzm = p == 0 ? wb(4) : T(1);
                    const T wzp = p == nz - 1 ? wb(5) : T(1);
                    T elo[2], ehi[2];
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        elo[c] = edge2[par ^ 1][strip][1][xp][c];
                        ehi[c] = edge2[par ^ 1][strip + 2][0][xp][c];
                    }
                    T res[M][2];
#pragma unroll
                    for (int r = 0; r < M; ++r) {
                        const T pm = lane_prev(ph[sc][r][1]);
                        const T pn = lane_next(ph[sc][r][0]);
                        const T kn = lane_next(fx[sf][r][0]);
#pragma unroll
                        for (int o = 0; o < 2; ++o) {
                            const T xm = o == 0 ? pm : ph[sc][r][0];
                            const T xq = o == 0 ? ph[sc][r][1] : pn;
                            const T kxm = fx[sf][r][o], kxp = o == 0 ? fx[sf][r][1] : kn;
                            const T ym = r > 0 ? ph[sc][r - 1][o] : elo[o];
                            const T yq = r < M - 1 ? ph[sc][r + 1][o] : ehi[o];
                            const T kym = fy[sf][r][o], kyp = fy[sf][r + 1][o];
                            const T kzm = fz[szm][r][o], kzp = fz[szp][r][o];
                            T dd = (o == 0 ? wx0 : T(1)) * kxm;
                            dd = fma(o == 1 ? wx1 : T(1), kxp, dd);
                            dd = fma(r == 0 ? wy0 : T(1), kym, dd);
                            dd = fma(r == 1 ? wy1 : T(1), kyp, dd);
                            dd = fma(wzm, kzm, dd);
                            dd = fma(wzp, kzp, dd);
                            T ss = kxm * xm;
                            ss = fma(kxp, xq, ss);
                            ss = fma(kym, ym, ss);
                            ss = fma(kyp, yq, ss);
                            ss = fma(kzm, ph[sm][r][o], ss);
                            ss = fma(kzp, ph[sp][r][o], ss);
                            res[r][o] = bb[sf][r][o] - fma(dd, ph[sc][r][o], -ss);
                        }
                    }
                    if constexpr (RESTRICT) {
                        // children: the pair (x), rows 0 and 1 (y), planes p and p + 1 (z)
                        const T s4 = (res[0][0] + res[0][1]) + (res[1][0] + res[1][1]);
                        if ((p & 1) == 0) {
                            racc = s4;
                        } else {
                            const int pc = p >> 1;
                            const auto rc = plane_rsrc(P.bc_out, cplane, pc, true);
                            const auto rz = plane_rsrc(P.phic, cplane, pc, true);
                            bstore1(rc, offC, T(0.25) * (racc + s4));
                            bstore1(rz, offC, T(0));
                        }
                    } else {
#pragma unroll
                        for (int r = 0; r < M; ++r) {
                            if (own[r]) {
                                acc_r2 += res[r][0] * res[r][0] + res[r][1] * res[r][1];
                                acc_b2 += bb[sf][r][0] * bb[sf][r][0] + bb[sf][r][1] * bb[sf][r][1];
                            }
                        }
                    }
                }
                if (t + 1 < tend) load_late(t + 1, (q + 1) % RF);
                __syncthreads();
            }
        }
    }
    if constexpr (!RESTRICT) store_partials<64 * WY>(acc_r2, acc_b2, P.partials, blk);
}

constexpr int kVcCgThreads = 512;

// Coarsest-level CG on the stored stencil with one cell per thread (n <=
// kVcCgThreads, Sec. 5.3): the cell's face coefficients, diagonal and
// neighbour indices (as vc_row, periodic wrap included) stay in registers and
// only the residual passes through LDS.  Arranged as cg_one_wave
// (Chronopoulos and Gear): (r, r) and (r, S r) in one combined reduction per
// iteration, two workgroup barriers per iteration; x = 0 to ||r|| <= rtol ||b||
// or maxit.
__global__ __launch_bounds__(kVcCgThreads) void k_vc_cg_cell(VcLevel L, const double* b, double* x_out, double rtol,
                                                            int maxit, const Ctl* ctl)
{
    if (ctl != nullptr && ctl->done) return;
    constexpr int NW = kVcCgThreads / 64;
    __shared__ double rl[kVcCgThreads];
    __shared__ double red[2][NW];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nx = L.nx, ny = L.ny, nz = L.nz, n = nx * ny * nz;
    const bool v = tid < n;
    int i, j, k;
    split3(v ? tid : 0, SmallDiv(nx), SmallDiv(ny), i, j, k);
    const int c = tid, sy = nx, sz = nx * ny;
    const int wx = nx - 1, wy = (ny - 1) * sy, wz = (nz - 1) * sz;
    double kf[6];
    int nb[6];
    double d = 0.0;
    // face f with coefficient kk: an in-domain (or periodic) neighbour at index m,
    // or a boundary face (no term; 2 kk on the diagonal when Dirichlet)
    auto face = [&](int f, double kk, bool inside, bool wrap, int m_in, int m_wrap) {
        if (inside) { d += kk; kf[f] = kk; nb[f] = m_in; }
        else if (wrap) { d += kk; kf[f] = kk; nb[f] = m_wrap; }
        else { if (L.dir[f]) d += 2.0 * kk; kf[f] = 0.0; nb[f] = c; }
    };
    if (v) {
        face(0, L.kx[vc_ix(L, i, j, k)], i > 0, L.per[0] != 0, c - 1, c + wx);
        face(1, L.kx[vc_ix(L, i + 1, j, k)], i < nx - 1, L.per[0] != 0, c + 1, c - wx);
        face(2, L.ky[vc_iy(L, i, j, k)], j > 0, L.per[1] != 0, c - sy, c + wy);
        face(3, L.ky[vc_iy(L, i, j + 1, k)], j < ny - 1, L.per[1] != 0, c + sy, c - wy);
        face(4, L.kz[vc_iz(L, i, j, k)], k > 0, L.per[2] != 0, c - sz, c + wz);
        face(5, L.kz[vc_iz(L, i, j, k + 1)], k < nz - 1, L.per[2] != 0, c + sz, c - wz);
    } else {
#pragma unroll
        for (int f = 0; f < 6; ++f) { kf[f] = 0.0; nb[f] = 0; }
    }
    double rv = v ? b[tid] : 0.0, xr = 0.0, pv = 0.0, sv = 0.0;
    rl[tid] = rv;
    double gamma_old = 1.0, alpha_old = 1.0, bound = 0.0;
    int it = 0;
    while (true) {
        __syncthreads();   // the residual in LDS is complete
        double ss = kf[0] * rl[nb[0]];
        ss += kf[1] * rl[nb[1]];
        ss += kf[2] * rl[nb[2]];
        ss += kf[3] * rl[nb[3]];
        ss += kf[4] * rl[nb[4]];
        ss += kf[5] * rl[nb[5]];
        const double wv = v ? d * rv - ss : 0.0;
        double gamma = rv * rv, delta = rv * wv;
        gamma = wave_sum(gamma);
        delta = wave_sum(delta);
        if (lane == 0) { red[0][w] = gamma; red[1][w] = delta; }
        __syncthreads();   // every wave's sums are in LDS; every read of rl above is done
        gamma = 0.0;
        delta = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) { gamma += red[0][q]; delta += red[1][q]; }
        // every thread holds the same sums: the exits are uniform
        if (it == 0) {
            if (!(gamma > 0.0)) break;
            bound = rtol * rtol * gamma;
        } else if (gamma <= bound) {
            break;
        }
        if (it >= maxit) break;
        const double beta = it == 0 ? 0.0 : gamma / gamma_old;
        const double alpha = gamma / (delta - beta * gamma / alpha_old);
        pv = rv + beta * pv;
        sv = wv + beta * sv;
        xr += alpha * pv;
        rv -= alpha * sv;
        rl[tid] = rv;
        ++it;
        gamma_old = gamma;
        alpha_old = alpha;
    }
    if (v) x_out[tid] = xr;
}

// coarsest level: conjugate gradients by one workgroup (Sec. 5.3) on the
// stored stencil, from x = 0 until ||r|| <= rtol ||b|| or maxit; vectors in LDS
__global__ __launch_bounds__(kVcCgThreads) void k_vc_cg(VcLevel L, const double* b, double* x_out, double rtol,
                                                       int maxit, const Ctl* ctl)
{
    if (ctl != nullptr && ctl->done) return;
    extern __shared__ double vcg[];
    const int n = L.nx * L.ny * L.nz;
    double* x = vcg;
    double* r = x + n;
    double* p = r + n;
    double* q = p + n;
    const int tid = threadIdx.x;
    double rr = 0.0;
    for (int c = tid; c < n; c += kVcCgThreads) {
        x[c] = 0.0;
        r[c] = b[c];
        p[c] = b[c];
        rr += b[c] * b[c];
    }
    rr = block_sum_d<kVcCgThreads>(rr);
    const double bn = sqrt(rr);
    if (bn > 0.0) {
        for (int it = 0; it < maxit; ++it) {
            double pq = 0.0;
            for (int c = tid; c < n; c += kVcCgThreads) {
                const int i = c % L.nx, j = (c / L.nx) % L.ny, k = c / (L.nx * L.ny);
                double d, sum;
                vc_row(L, p, i, j, k, d, sum);
                q[c] = d * p[c] - sum;
                pq += p[c] * q[c];
            }
            pq = block_sum_d<kVcCgThreads>(pq);
            const double alpha = rr / pq;
            double rn = 0.0;
            for (int c = tid; c < n; c += kVcCgThreads) {
                x[c] += alpha * p[c];
                r[c] -= alpha * q[c];
                rn += r[c] * r[c];
            }
            rn = block_sum_d<kVcCgThreads>(rn);
            if (sqrt(rn) <= rtol * bn) break;
            const double beta = rn / rr;
            rr = rn;
            for (int c = tid; c < n; c += kVcCgThreads) p[c] = r[c] + beta * p[c];
            __syncthreads();
        }
    }
    __syncthreads();
    for (int c = tid; c < n; c += kVcCgThreads) x_out[c] = x[c];
}

}  // namespace ccmg
