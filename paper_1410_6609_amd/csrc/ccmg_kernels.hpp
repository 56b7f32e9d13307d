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
    unsigned int counter;  // blocks finished in the current reduction
    int cg_iters;       // iterations of the last coarsest-grid CG
    int pad[2];
    double hist[kMaxHist];
};

enum Fin : int { FIN_NONE = 0, FIN_INIT = 1, FIN_CYCLE = 2, FIN_STORE = 3 };
enum Load : int { LOAD_PHI = 0, LOAD_ZERO = 1, LOAD_PROLONG = 2, LOAD_CORR = 3 };
enum Res : int { RES_NONE = 0, RES_RESTRICT = 1, RES_NORM = 2, RES_NORM_R32 = 3, RES_STORE = 4 };

// Parameters of the smoother-pass kernel (one struct for every variant).
template <typename T>
struct PassParams {
    const T* phi_in;     // LOAD_PHI / LOAD_PROLONG / LOAD_CORR
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
    Ctl* ctl;            // nullable
    int fin;             // Fin code for the last block
    int cycle;           // FIN_CYCLE: cycle index
    int nx, ny, nz;
    int zc;              // planes per block (even)
    int tiles_x, tiles_y, zchunks;
    int sh[6];           // per-face centre shift: +1 Dirichlet, -1 Neumann
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

// Last-block reduction epilogue.  Every block stores its two partial sums;
// the block that finishes last adds all partials in block order (deterministic)
// and updates the control block.
template <int NT>
__device__ void finish_norm(double s_r2, double s_b2, double* partials, Ctl* ctl, int fin, int cycle,
                            int nblk, int myblk)
{
    __shared__ double red[2][NT / 64];
    __shared__ int last;
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
        __threadfence();
        const unsigned prev = atomicAdd(&ctl->counter, 1u);
        last = (prev == (unsigned)nblk - 1u);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double a = 0.0, b = 0.0;
    for (int i = tid; i < nblk; i += NT) {
        a += __hip_atomic_load(&partials[2 * i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        b += __hip_atomic_load(&partials[2 * i + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    a = wave_sum(a);
    b = wave_sum(b);
    __syncthreads();
    if (lane == 0) { red[0][w] = a; red[1][w] = b; }
    __syncthreads();
    if (tid != 0) return;
    double r2 = 0.0, b2 = 0.0;
    for (int i = 0; i < NT / 64; ++i) { r2 += red[0][i]; b2 += red[1][i]; }
    const double rn = sqrt(r2), bn = sqrt(b2);
    ctl->counter = 0u;
    ctl->rnorm = rn;
    if (fin == FIN_INIT) {
        ctl->bnorm = bn;
        const double rel = bn > 0.0 ? rn / bn : 0.0;
        ctl->rel = rel;
        ctl->hist[0] = rel;
        ctl->cycles = 0;
        ctl->bzero = (bn == 0.0);
        const bool finite = isfinite(rel);
        ctl->status = finite ? 0 : -5;
        ctl->done = (bn == 0.0) || !(rel >= ctl->rtol);
        ctl->sig_next = rn > 0.0 ? pow2_floor(rn) : 1.0;
    } else if (fin == FIN_CYCLE) {
        const double rel = bn > 0.0 ? rn / bn : 0.0;
        ctl->rel = rel;
        if (cycle < kMaxHist) ctl->hist[cycle] = rel;
        ctl->cycles = cycle;
        const bool finite = isfinite(rel);
        if (!finite) ctl->status = -5;
        if (!(rel >= ctl->rtol)) ctl->done = 1;
        ctl->sig_cur = ctl->sig_next;
        ctl->sig_next = rn > 0.0 ? pow2_floor(rn) : 1.0;
    } else if (fin == FIN_STORE) {
        ctl->bnorm = bn;
        ctl->rel = bn > 0.0 ? rn / bn : 0.0;
    }
}

// ---------------------------------------------------------------------------
// The smoother pass.
//
// One workgroup owns an x-y tile and marches up a chunk of z-planes.  Lanes
// run along x (coalesced rows), each thread holds M consecutive y-rows, WY
// waves stack in y.  A pass applies SPHI red-black colour half-sweeps (SPHI/2
// full sweeps) and optionally a residual stage, all in one read of phi and b:
// stage s at plane p runs at step t = p + s, so every stage finds the planes
// p-1, p, p+1 it needs in the per-thread register ring.  The x-neighbours come
// from the adjacent lanes, y-neighbours from the thread's own rows or, at the
// edges of its row strip, from LDS (double-buffered per step, one barrier per
// step).  Each stage is exact on a tile that shrinks by one cell per stage, so
// the tile carries an H-cell halo that is loaded but not written.
//
//   LOAD: phi_in | zero | phi_in + omega * e(parent) | phi_in + sigma * corr
//   RES:  none | restriction of the residual to the next level's b-tilde |
//         residual norm | residual norm + residual / sigma as FP32 | store r
// ---------------------------------------------------------------------------
template <typename T, int SPHI, int RES, int M, int WY>
struct PassShape {
    static constexpr int S = SPHI + (RES != RES_NONE ? 1 : 0);   // stages after the load
    static constexpr int H = (S + 1) & ~1;                           // halo, even (restriction pairs)
    static constexpr int EX = 64;
    static constexpr int EY = M * WY;
    static constexpr int TX = EX - 2 * H;
    static constexpr int TY = EY - 2 * H;
    static constexpr int R = S + 2;                                  // ring planes
    static constexpr int NT = 64 * WY;
    static constexpr int LDS_STAGES = S > 0 ? S : 1;
};

template <typename T, int SPHI, int LOAD, int RES, int M, int WY>
__global__ __launch_bounds__(64 * WY) void k_pass(PassParams<T> P)
{
    using Sh = PassShape<T, SPHI, RES, M, WY>;
    constexpr int S = Sh::S, H = Sh::H, TX = Sh::TX, TY = Sh::TY, R = Sh::R;
    static_assert(M % 2 == 0, "rows per thread must be even");
    static_assert(TX > 0 && TY > 0, "tile too small for the halo");

    if (P.ctl != nullptr && P.ctl->done) return;

    __shared__ T edge[Sh::LDS_STAGES][2][WY][2][64];

    const int nblk = P.tiles_x * P.tiles_y * P.zchunks;
    const int blk = xcd_block_id(nblk);
    const int bx = blk % P.tiles_x;
    const int by = (blk / P.tiles_x) % P.tiles_y;
    const int bz = blk / (P.tiles_x * P.tiles_y);

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int x = bx * TX - H + lane;
    const int ybase = by * TY - H + w * M;
    const int z0 = bz * P.zc;
    const int z1 = min(nz, z0 + P.zc);
    const bool vx = (x >= 0) && (x < nx);
    const bool xin = (lane >= H) && (lane < H + TX);

    // per-row geometry: validity, interior membership and 1/d without the z faces
    int dxy[M];
    T invd[M];
    bool vrow[M], yin[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const int y = ybase + r;
        vrow[r] = vx && (y >= 0) && (y < ny);
        const int ry = w * M + r;
        yin[r] = (ry >= H) && (ry < H + TY);
        int d = 6;
        if (x == 0) d += P.sh[0];
        if (x == nx - 1) d += P.sh[1];
        if (y == 0) d += P.sh[2];
        if (y == ny - 1) d += P.sh[3];
        dxy[r] = d;
        invd[r] = T(1) / T(d);
    }
    const int cnx = nx >> 1, cny = ny >> 1;
    const size_t plane = (size_t)nx * ny;

    T ph[R][M];
    T bb[R][M];
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int r = 0; r < M; ++r) { ph[q][r] = T(0); bb[q][r] = T(0); }

    // FP32-IR scales
    T sig_cur = T(0);
    double inv_sig_next = 1.0;
    if constexpr (LOAD == LOAD_CORR) sig_cur = (T)P.ctl->sig_cur;
    if constexpr (RES == RES_NORM_R32) inv_sig_next = 1.0 / P.ctl->sig_next;

    double acc_r2 = 0.0, acc_b2 = 0.0;
    T racc[M / 2];
#pragma unroll
    for (int r = 0; r < M / 2; ++r) racc[r] = T(0);

    // prefetch registers: plane t+1 is loaded while plane t's stages run
    T nph[M], nbb[M];
    auto load_plane = [&](int t, T* dph, T* dbb) {
        const bool zin = (t >= 0) && (t < nz);
#pragma unroll
        for (int r = 0; r < M; ++r) {
            T v = T(0), bv = T(0);
            if (zin && vrow[r]) {
                const size_t idx = (size_t)t * plane + (size_t)(ybase + r) * nx + x;
                bv = P.b[idx];
                if constexpr (LOAD == LOAD_PHI) v = P.phi_in[idx];
                if constexpr (LOAD == LOAD_PROLONG)
                    v = P.phi_in[idx] + P.omega * P.ec[((size_t)(t >> 1) * cny + ((ybase + r) >> 1)) * cnx + (x >> 1)];
                if constexpr (LOAD == LOAD_CORR) v = P.phi_in[idx] + sig_cur * (T)P.corr[idx];
            }
            dph[r] = v;
            dbb[r] = bv;
        }
    };

    const int tbeg = z0 - S, tend = z1 + S;
    load_plane(tbeg, nph, nbb);

    for (int tb = tbeg; tb < tend; tb += R) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int t = tb + q;
            if (t < tend) {
                // ---- stage 0: the prefetched plane t enters the ring; prefetch t+1
#pragma unroll
                for (int r = 0; r < M; ++r) { ph[q][r] = nph[r]; bb[q][r] = nbb[r]; }
                if (t + 1 < tend) load_plane(t + 1, nph, nbb);
                if constexpr (S > 0) {
                    edge[0][t & 1][w][0][lane] = ph[q][0];
                    edge[0][t & 1][w][1][lane] = ph[q][M - 1];
                }
                // ---- stages 1..SPHI: colour half-sweeps, red first (Sec. 5.3)
#pragma unroll
                for (int s = 1; s <= SPHI; ++s) {
                    const int p = t - s;
                    constexpr int dummy = 0; (void)dummy;
                    const int sc = (q - s + 2 * R) % R;
                    const int sm = (q - s - 1 + 2 * R) % R;
                    const int sp = (q - s + 1 + 2 * R) % R;
                    const int colour = (s - 1) & 1;
                    const T* ein = &edge[s - 1][(t - 1) & 1][0][0][0];
                    const T yme = (w > 0) ? ein[((w - 1) * 2 + 1) * 64 + lane] : T(0);
                    const T ype = (w < WY - 1) ? ein[((w + 1) * 2 + 0) * 64 + lane] : T(0);
                    const bool pin = (p >= 0) && (p < nz);
                    int dz = 0;
                    if (p == 0) dz += P.sh[4];
                    if (p == nz - 1) dz += P.sh[5];
#pragma unroll
                    for (int r = 0; r < M; ++r) {
                        const T c = ph[sc][r];
                        const T xm = __shfl_up(c, 1);
                        const T xp = __shfl_down(c, 1);
                        const T ym = (r > 0) ? ph[sc][r - 1] : yme;
                        const T yp = (r < M - 1) ? ph[sc][r + 1] : ype;
                        const T sum = ((((xm + xp) + ym) + yp) + ph[sm][r]) + ph[sp][r];
                        const T inv = (dz == 0) ? invd[r] : T(1) / T(dxy[r] + dz);
                        const T nv = (bb[sc][r] + sum) * inv;
                        const bool upd = pin && vrow[r] && (((x + ybase + r + p) & 1) == colour);
                        ph[sc][r] = upd ? nv : c;
                    }
                    if (s < S) {
                        edge[s][t & 1][w][0][lane] = ph[sc][0];
                        edge[s][t & 1][w][1][lane] = ph[sc][M - 1];
                    }
                }
                // ---- output of the smoothed plane t - SPHI
                if (P.phi_out != nullptr) {
                    const int po = t - SPHI;
                    if (po >= z0 && po < z1 && xin) {
                        const int so = (q - SPHI + 2 * R) % R;
#pragma unroll
                        for (int r = 0; r < M; ++r)
                            if (vrow[r] && yin[r])
                                P.phi_out[(size_t)po * plane + (size_t)(ybase + r) * nx + x] = ph[so][r];
                    }
                }
                // ---- residual stage at plane t - S
                if constexpr (RES != RES_NONE) {
                    const int p = t - S;
                    const int sc = (q - S + 2 * R) % R;
                    const int sm = (q - S - 1 + 2 * R) % R;
                    const int sp = (q - S + 1 + 2 * R) % R;
                    const T* ein = &edge[S - 1][(t - 1) & 1][0][0][0];
                    const T yme = (w > 0) ? ein[((w - 1) * 2 + 1) * 64 + lane] : T(0);
                    const T ype = (w < WY - 1) ? ein[((w + 1) * 2 + 0) * 64 + lane] : T(0);
                    const bool pok = (p >= z0) && (p < z1);
                    int dz = 0;
                    if (p == 0) dz += P.sh[4];
                    if (p == nz - 1) dz += P.sh[5];
                    T res[M];
#pragma unroll
                    for (int r = 0; r < M; ++r) {
                        const T c = ph[sc][r];
                        const T xm = __shfl_up(c, 1);
                        const T xp = __shfl_down(c, 1);
                        const T ym = (r > 0) ? ph[sc][r - 1] : yme;
                        const T yp = (r < M - 1) ? ph[sc][r + 1] : ype;
                        const T sum = ((((xm + xp) + ym) + yp) + ph[sm][r]) + ph[sp][r];
                        res[r] = bb[sc][r] - (T(dxy[r] + dz) * c - sum);
                    }
                    if constexpr (RES == RES_RESTRICT) {
                        // children pairs: x (adjacent lanes), y (rows r, r+1), z (planes p, p+1)
                        T rx[M];
#pragma unroll
                        for (int r = 0; r < M; ++r) rx[r] = res[r] + __shfl_down(res[r], 1);
                        const bool writer = pok && xin && ((x & 1) == 0);
#pragma unroll
                        for (int r = 0; r < M; r += 2) {
                            const T s4 = rx[r] + rx[r + 1];
                            if ((p & 1) == 0) {
                                racc[r / 2] = s4;
                            } else if (writer && vrow[r] && yin[r]) {
                                P.bc_out[((size_t)(p >> 1) * cny + ((ybase + r) >> 1)) * cnx + (x >> 1)] =
                                    T(0.25) * (racc[r / 2] + s4);
                            }
                        }
                    } else {
                        if (pok && xin) {
#pragma unroll
                            for (int r = 0; r < M; ++r) {
                                if (vrow[r] && yin[r]) {
                                    const double rv = (double)res[r];
                                    acc_r2 += rv * rv;
                                    acc_b2 += (double)bb[sc][r] * (double)bb[sc][r];
                                    const size_t idx = (size_t)p * plane + (size_t)(ybase + r) * nx + x;
                                    if constexpr (RES == RES_NORM_R32) P.r32_out[idx] = (float)(rv * inv_sig_next);
                                    if constexpr (RES == RES_STORE) if (P.r_out) P.r_out[idx] = res[r] * P.rscale;
                                }
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }
    }

    if constexpr (RES == RES_NORM || RES == RES_NORM_R32 || RES == RES_STORE) {
        finish_norm<64 * WY>(acc_r2, acc_b2, P.partials, P.ctl, P.fin, P.cycle, nblk, blk);
    }
}

// ---------------------------------------------------------------------------
// Coarsest level: conjugate gradients in FP64 by one workgroup (Sec. 5.3),
// search direction resident in LDS.  Solves S x = b-tilde from x = 0 until
// ||r|| <= rtol ||b|| or maxit, and writes x (as T).
// ---------------------------------------------------------------------------
constexpr int kCgThreads = 256;

template <typename T, int NPT>
__global__ __launch_bounds__(kCgThreads) void k_coarse_cg(const T* b, T* x_out, int nx, int ny, int nz,
                                                          int sh0, int sh1, int sh2, int sh3, int sh4, int sh5,
                                                          double rtol, int maxit, Ctl* ctl)
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
                qv[k] = dg[k] ? (double)dg[k] * pc - s : 0.0;
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
// Elementwise kernels
// ---------------------------------------------------------------------------

// Finest right-hand side with the boundary terms folded in (Sec. 2.4, Sec. 5.3):
// b-tilde = h^2 (f + sum over the cell's boundary faces of term_f), where
// term_f = 2 g_d / h^2 (Dirichlet) or g_n / h (Neumann).
__global__ void k_fold(const double* f, double* bt, int nx, int ny, int nz, double h2,
                       double t0, double t1, double t2, double t3, double t4, double t5, Ctl* ctl)
{
    const size_t n = (size_t)nx * ny * nz;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx);
        const int j = (int)((c / nx) % ny);
        const int k = (int)(c / ((size_t)nx * ny));
        double v = f[c];
        if (i == 0) v += t0;
        if (i == nx - 1) v += t1;
        if (j == 0) v += t2;
        if (j == ny - 1) v += t3;
        if (k == 0) v += t4;
        if (k == nz - 1) v += t5;
        bt[c] = v * h2;
    }
}

template <typename T>
__global__ void k_fill(T* a, size_t n, T v)
{
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x)
        a[c] = v;
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
        ctl->counter = 0u;
        ctl->cg_iters = 0;
    }
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

}  // namespace ccmg
