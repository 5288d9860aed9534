// Nystrom approximation around the sketch (Sec. 5, Alg. 2): with B = A Omega and
// the core C = Omega^T B (both from the product kernels), the approximation is
// A~ = B C^+ B^T.  This file holds the rest of it on the device, in FP64:
//
//   * the pseudo-inverse of the symmetric r x r core by a parallel block Jacobi
//     eigensolver (two-sided, cyclic round-robin over 16-row blocks), with the
//     eigenvalue cut of Sec. 6.2: eigenvalues of modulus at most tol times the
//     largest are treated as zero;
//   * W = B C^+, then rows of A~ = W B^T or the squared Frobenius norms
//     ||A - A~||^2 and ||A||^2 (relative error of Table 2).
//
// Jacobi: S = (C + C^T)/2 is padded with zero rows and columns to Rp, a
// multiple of 32, and split into nb = Rp/16 blocks.  A step pairs the blocks by
// the circle method (nb/2 disjoint pairs; nb-1 steps meet every pair once).
// For each pair, one workgroup runs one cyclic sweep of 2x2 Jacobi rotations on
// the pair's 32 x 32 diagonal tile and keeps their product Q_P.  A second
// launch forms S <- Q^T S Q tile by tile (pair-tile (a, b) becomes
// Q_a^T S_ab Q_b; tiles a <= b are computed and mirrored, so S stays exactly
// symmetric) and V <- V Q.  After each sweep the off-diagonal norm decides
// convergence; the kernels of later sweeps return at once.  Padding rows and
// columns are zero and are never rotated (a rotation needs a non-zero
// off-diagonal entry), so they stay zero and carry the eigenvalue 0.
//
// Every sum runs in a fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "sk_internal.hpp"

namespace sk {
namespace {

constexpr int kJB = 16;            // rows of a Jacobi block
constexpr int kJT = 2 * kJB;       // rows of a pair tile
constexpr int kJP = kJT + 1;       // LDS row pitch of a tile (doubles)
constexpr int kJThreads = 256;
constexpr int kPerThread = kJT * kJT / kJThreads;   // tile elements per thread (4)

// Circle-method pairing of nb (even) players at round s in [0, nb - 1): player 0
// meets 1 + s; for i >= 1 the players 1 + (s + i) mod (nb - 1) and
// 1 + (s - i) mod (nb - 1) meet.
__device__ __forceinline__ void circle_pair(int nb, int s, int i, int& a, int& b) {
    const int m = nb - 1;
    if (i == 0) {
        a = 0;
        b = 1 + s % m;
    } else {
        a = 1 + (s + i) % m;
        b = 1 + (s - i + m) % m;
    }
}

// Global row of tile index t (0..31) of the pair of blocks (I, J).
__device__ __forceinline__ int64_t tile_row(int I, int J, int t) {
    return t < kJB ? (int64_t)I * kJB + t : (int64_t)J * kJB + (t - kJB);
}

struct JacState {
    int converged;      // set once the off-diagonal norm is small enough
    int sweeps;         // sweeps run before convergence
};

// S = (C + C^T)/2 padded to Rp x Rp, V = I, state cleared.
template <typename TC>
__global__ __launch_bounds__(256) void k_jac_init(const TC* __restrict__ C, int64_t r, int64_t ldc,
                                                  double* __restrict__ S, double* __restrict__ V,
                                                  int64_t Rp, JacState* st) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e == 0) {
        st->converged = 0;
        st->sweeps = 0;
    }
    if (e >= Rp * Rp) return;
    const int64_t i = e / Rp, j = e % Rp;
    double s = 0.0;
    if (i < r && j < r) s = 0.5 * ((double)C[i * ldc + j] + (double)C[j * ldc + i]);
    S[e] = s;
    V[e] = (i == j) ? 1.0 : 0.0;
}

// 1/sqrt(x) and 1/x for normal positive x: the hardware estimates refined by
// two Newton steps (each squares the relative error).
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    for (int i = 0; i < 2; ++i) {
        const double e = fma(-(x * y), y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// Rotation for the symmetric 2x2 [[app, apq], [apq, aqq]]: J = [[c, s], [-s, c]]
// with t = tan theta = sign(d) e / (|d| + sqrt(d^2 + e^2)), d = aqq - app,
// e = 2 apq, the smaller root of the equation that zeroes the off-diagonal
// entry.  t is evaluated in FP32 (d and e brought into [2^-64, 2^64] by a
// power of two when they lie outside; an angle within a few 2^-24 of the
// exact one leaves that fraction of apq), then c = (1 + t^2)^-1/2 and s = t c
// in FP64, so that J is orthogonal to FP64 rounding.  Identity when apq = 0.
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, double& c,
                                                double& s) {
    double d = aqq - app, e = 2.0 * apq;
    const double m = fmax(fabs(d), fabs(e));
    if (m > 0x1p64 || m < 0x1p-64) {
        int ex;
        (void)frexp(m, &ex);
        d = ldexp(d, -ex);
        e = ldexp(e, -ex);
    }
    const float df = (float)d, ef = (float)e;
    const float hf = __builtin_amdgcn_sqrtf(fmaf(df, df, ef * ef));
    const float tf = (df >= 0.f ? ef : -ef) * __builtin_amdgcn_rcpf(fabsf(df) + hf);
    const double t = (double)tf;
    const double cc = rsqrt_nr(fma(t, t, 1.0));
    c = apq == 0.0 ? 1.0 : cc;
    s = apq == 0.0 ? 0.0 : t * cc;
}

// Pairing of the blocks in a launch: kFull pairs blocks (2i, 2i + 1) and runs
// a full inner sweep (every pair of the tile's 32 indices); kCross pairs the
// blocks by the circle method at the given step and rotates only the 256
// pairs (one index of each block).  A sweep of the whole matrix is one kFull
// launch and nb - 1 kCross launches: every pair of indices is rotated at least
// once, in 31 + 16 (nb - 1) rounds.
enum { kFull = 0, kCross = 1 };

template <int MODE>
__device__ __forceinline__ void pair_blocks(int nb, int step, int i, int& I, int& J) {
    if (MODE == kFull) {
        I = 2 * i;
        J = 2 * i + 1;
    } else {
        circle_pair(nb, step, i, I, J);
    }
}

// Inner schedule on the 32 positions of a pair tile: the pairs of a round are
// always the positions (2i, 2i + 1); after each round the entry at position p
// moves to sigma(p).
//  kFull (31 rounds): position p starts with tile index p; sigma is the circle
//   method seen from the positions: position 0 stays, the others carry an
//   offset c in [0, 31) (position 1: c = 0, 2i: c = i, 2i + 1: c = 31 - i) that
//   drops by one each round, so every pair of indices meets once.
//  kCross (16 rounds): position 2k starts with index k of the first block and
//   2k + 1 with index k of the second; even positions stay and the second
//   block's indices step down one odd position per round, so each first-block
//   index meets every second-block index once.
// Both schedules return every index to its starting position.
template <int MODE>
__device__ __forceinline__ int tile_index(int p) {
    return MODE == kFull ? p : (p & 1) ? kJB + p / 2 : p / 2;
}
__device__ __forceinline__ int pos_offset(int p) { return p == 1 ? 0 : (p & 1) ? kJT - 1 - p / 2 : p / 2; }
__device__ __forceinline__ int offset_pos(int c) {
    return c == 0 ? 1 : c < kJT / 2 ? 2 * c : 2 * (kJT - 1 - c) + 1;
}
template <int MODE>
__device__ __forceinline__ int sigma(int p) {
    if (MODE == kCross) return (p & 1) ? 2 * ((p / 2 + kJB - 1) % kJB) + 1 : p;
    return p == 0 ? 0 : offset_pos((pos_offset(p) + kJT - 2) % (kJT - 1));
}
template <int MODE>
constexpr int rounds() { return MODE == kFull ? kJT - 1 : kJB; }

// One inner sweep on each pair's 32 x 32 diagonal tile; Q_P (32 x 32,
// row-major) = the product of its rotations.  512 threads: thread (X, Y) of the
// first 256 keeps the 2x2 block of rows 2X, 2X+1 and columns 2Y, 2Y+1 of the
// tile in registers, the same thread of the second 256 that block of Q.  A
// round computes the 16 rotations (on the diagonal blocks), applies them to
// every block, and moves the entries to their next positions through LDS.
constexpr int kSolveThreads = 2 * kJThreads;

template <int MODE>
__global__ __launch_bounds__(kSolveThreads) void k_jac_solve(const double* __restrict__ S,
                                                             int64_t Rp, double* __restrict__ Q,
                                                             int nb, int step, const JacState* st) {
    if (st->converged) return;
    __shared__ double al[kJT][kJP];
    __shared__ double ql[kJT][kJP];
    __shared__ double rc[kJT / 2], rs[kJT / 2];
    const bool qrole = threadIdx.x >= kJThreads;
    const int tid = threadIdx.x & (kJThreads - 1), X = tid / 16, Y = tid % 16;
    int I, J;
    pair_blocks<MODE>(nb, step, blockIdx.x, I, J);
    double a[2][2];
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v)
            a[u][v] = qrole ? ((2 * X + u == 2 * Y + v) ? 1.0 : 0.0)
                            : S[tile_row(I, J, tile_index<MODE>(2 * X + u)) * Rp +
                                tile_row(I, J, tile_index<MODE>(2 * Y + v))];
    int sx[2], sy[2];
    for (int u = 0; u < 2; ++u) {
        sx[u] = qrole ? 2 * X + u : sigma<MODE>(2 * X + u);    // Q's rows do not move
        sy[u] = sigma<MODE>(2 * Y + u);
    }
    double (*buf)[kJP] = qrole ? ql : al;
    for (int t = 0; t < rounds<MODE>(); ++t) {
        if (!qrole && X == Y) {
            double c, sn;
            jacobi_rotation(a[0][0], a[1][1], a[0][1], c, sn);
            rc[X] = c;
            rs[X] = sn;
        }
        __syncthreads();
        // J of a pair: [[c, s], [-s, c]] on its two positions
        const double cy = rc[Y], syn = rs[Y];
        const double jy[2][2] = {{cy, syn}, {-syn, cy}};
        double na[2][2];
        if (qrole) {
            for (int u = 0; u < 2; ++u)
                for (int v = 0; v < 2; ++v) na[u][v] = a[u][v] * jy[v][v] + a[u][v ^ 1] * jy[v ^ 1][v];
        } else {
            const double cx = rc[X], sxn = rs[X];
            const double jx[2][2] = {{cx, sxn}, {-sxn, cx}};
            for (int u = 0; u < 2; ++u)
                for (int v = 0; v < 2; ++v) {
                    // (J_X^T A J_Y)(u, v) as (T(u,v) + T(u',v')) + (T(u,v') + T(u',v)),
                    // T(i, j) = (J_X(i, u) J_Y(j, v)) A(i, j): block (Y, X) sums the same
                    // terms, so the tile stays exactly symmetric
                    const int ub = u ^ 1, vb = v ^ 1;
                    const double t1 = (jx[u][u] * jy[v][v]) * a[u][v];
                    const double t4 = (jx[ub][u] * jy[vb][v]) * a[ub][vb];
                    const double t2 = (jx[u][u] * jy[vb][v]) * a[u][vb];
                    const double t3 = (jx[ub][u] * jy[v][v]) * a[ub][v];
                    na[u][v] = (t1 + t4) + (t2 + t3);
                }
        }
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v) buf[sx[u]][sy[v]] = na[u][v];
        __syncthreads();
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v) a[u][v] = buf[2 * X + u][2 * Y + v];
    }
    if (qrole) {        // back at the starting positions: Q in tile-index order
        double* Qp = Q + (int64_t)blockIdx.x * kJT * kJT;
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v)
                Qp[tile_index<MODE>(2 * X + u) * kJT + tile_index<MODE>(2 * Y + v)] = a[u][v];
    }
}

// Fixed-order workgroup sum of two doubles per thread (256 threads).
__device__ __forceinline__ void block_sum2(double& x, double& y, double (*red)[kJThreads]) {
    const int tid = threadIdx.x;
    red[0][tid] = x;
    red[1][tid] = y;
    __syncthreads();
    for (int w = kJThreads / 2; w > 0; w >>= 1) {
        if (tid < w) {
            red[0][tid] += red[0][tid + w];
            red[1][tid] += red[1][tid + w];
        }
        __syncthreads();
    }
    x = red[0][0];
    y = red[1][0];
}

// S <- Q^T S Q over the upper pair-tiles (blocks [0, nT)) and V <- V Q over
// 32-row blocks of V (blocks [nT, nT + nV)).  Each S tile also writes its
// squared off-diagonal and total norms (mirror counted) to part[2 b], part[2 b + 1].
template <int MODE>
__global__ __launch_bounds__(kJThreads) void k_jac_apply(double* __restrict__ S,
                                                         double* __restrict__ V, int64_t Rp,
                                                         const double* __restrict__ Q, int nb,
                                                         int step, double* __restrict__ part,
                                                         const JacState* st) {
    if (st->converged) return;
    __shared__ double x[kJT][kJP];
    __shared__ double qa[kJT][kJP];
    __shared__ double qb[kJT][kJP];
    __shared__ double u[kJT][kJP];
    __shared__ double red[2][kJThreads];
    const int tid = threadIdx.x;
    const int np = nb / 2;
    const int nT = np * (np + 1) / 2;
    int b = blockIdx.x;
    if (b < nT) {
        int pa = 0;
        while (b >= np - pa) {
            b -= np - pa;
            ++pa;
        }
        const int pb = pa + b;
        int Ia, Ja, Ib, Jb;
        pair_blocks<MODE>(nb, step, pa, Ia, Ja);
        pair_blocks<MODE>(nb, step, pb, Ib, Jb);
        for (int v = 0; v < kPerThread; ++v) {
            const int e = tid + kJThreads * v, i = e / kJT, j = e % kJT;
            x[i][j] = S[tile_row(Ia, Ja, i) * Rp + tile_row(Ib, Jb, j)];
            qa[i][j] = Q[(int64_t)pa * kJT * kJT + e];
            qb[i][j] = Q[(int64_t)pb * kJT * kJT + e];
        }
        __syncthreads();
        const int ti = tid / 16, tj = tid % 16;           // rows ti, ti+16; columns tj, tj+16
        double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
        for (int z = 0; z < kJT; ++z) {                  // U = X Q_b
            const double x0 = x[ti][z], x1 = x[ti + 16][z], q0 = qb[z][tj], q1 = qb[z][tj + 16];
            acc[0][0] = fma(x0, q0, acc[0][0]);
            acc[0][1] = fma(x0, q1, acc[0][1]);
            acc[1][0] = fma(x1, q0, acc[1][0]);
            acc[1][1] = fma(x1, q1, acc[1][1]);
        }
        for (int a2 = 0; a2 < 2; ++a2)
            for (int b2 = 0; b2 < 2; ++b2) u[ti + 16 * a2][tj + 16 * b2] = acc[a2][b2];
        __syncthreads();
        double tacc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
        for (int z = 0; z < kJT; ++z) {                  // T = Q_a^T U
            const double q0 = qa[z][ti], q1 = qa[z][ti + 16], u0 = u[z][tj], u1 = u[z][tj + 16];
            tacc[0][0] = fma(q0, u0, tacc[0][0]);
            tacc[0][1] = fma(q0, u1, tacc[0][1]);
            tacc[1][0] = fma(q1, u0, tacc[1][0]);
            tacc[1][1] = fma(q1, u1, tacc[1][1]);
        }
        __syncthreads();
        for (int a2 = 0; a2 < 2; ++a2)
            for (int b2 = 0; b2 < 2; ++b2) x[ti + 16 * a2][tj + 16 * b2] = tacc[a2][b2];
        __syncthreads();
        double off = 0.0, tot = 0.0;
        for (int v = 0; v < kPerThread; ++v) {
            const int e = tid + kJThreads * v, i = e / kJT, j = e % kJT;
            const int64_t gi = tile_row(Ia, Ja, i), gj = tile_row(Ib, Jb, j);
            if (pa == pb) {
                const double t = i <= j ? x[i][j] : x[j][i];
                S[gi * Rp + gj] = t;
                tot += t * t;
                if (i != j) off += t * t;
            } else {
                const double t = x[i][j];
                S[gi * Rp + gj] = t;
                S[gj * Rp + gi] = t;
                tot += 2.0 * t * t;
                off += 2.0 * t * t;
            }
        }
        block_sum2(off, tot, red);
        if (tid == 0) {
            part[2 * blockIdx.x] = off;
            part[2 * blockIdx.x + 1] = tot;
        }
        return;
    }
    b -= nT;                                              // V role
    const int rb = b / np, pc = b % np;
    int Ic, Jc;
    pair_blocks<MODE>(nb, step, pc, Ic, Jc);
    for (int v = 0; v < kPerThread; ++v) {
        const int e = tid + kJThreads * v, i = e / kJT, j = e % kJT;
        x[i][j] = V[((int64_t)rb * kJT + i) * Rp + tile_row(Ic, Jc, j)];
        qa[i][j] = Q[(int64_t)pc * kJT * kJT + e];
    }
    __syncthreads();
    const int ti = tid / 16, tj = tid % 16;
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int z = 0; z < kJT; ++z) {
        const double x0 = x[ti][z], x1 = x[ti + 16][z], q0 = qa[z][tj], q1 = qa[z][tj + 16];
        acc[0][0] = fma(x0, q0, acc[0][0]);
        acc[0][1] = fma(x0, q1, acc[0][1]);
        acc[1][0] = fma(x1, q0, acc[1][0]);
        acc[1][1] = fma(x1, q1, acc[1][1]);
    }
    for (int a2 = 0; a2 < 2; ++a2)
        for (int b2 = 0; b2 < 2; ++b2)
            V[((int64_t)rb * kJT + ti + 16 * a2) * Rp + tile_row(Ic, Jc, tj + 16 * b2)] = acc[a2][b2];
}

// End of a sweep: sum the tiles' norms in tile order; converged when
// off <= tolc * total (Frobenius).
__global__ __launch_bounds__(kJThreads) void k_jac_flag(const double* __restrict__ part, int nT,
                                                        double tolc, JacState* st) {
    if (st->converged) return;
    __shared__ double red[2][kJThreads];
    double off = 0.0, tot = 0.0;
    for (int i = threadIdx.x; i < nT; i += kJThreads) {
        off += part[2 * i];
        tot += part[2 * i + 1];
    }
    block_sum2(off, tot, red);
    if (threadIdx.x == 0) {
        st->sweeps += 1;
        if (off <= tolc * tolc * tot) st->converged = 1;
    }
}

// Fixed-shape FP64 tile engine: out(i, j) = sum_l X(i, l) Y(j, l) (times mu_l
// when mu is given), l ascending, for a TM x TM tile per workgroup (256 threads,
// (TM/16) x (TM/16) outputs each, l in chunks of 16 staged in LDS).
constexpr int kGT = 64, kGK = 16;

template <int TM, typename TX, typename TY>
__device__ __forceinline__ void tile_accumulate(const TX* __restrict__ X, int64_t ldx, int64_t mx,
                                                const TY* __restrict__ Y, int64_t ldy, int64_t my,
                                                int64_t K, const double* mu, int64_t i0,
                                                int64_t j0, double acc[TM / 16][TM / 16],
                                                double (*xs)[TM], double (*ys)[TM]) {
    constexpr int R = TM / 16;                  // outputs per thread and dimension
    const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
    const int li = tid / (16 / R), lk = (tid % (16 / R)) * R;
    for (int a = 0; a < R; ++a)
        for (int c = 0; c < R; ++c) acc[a][c] = 0.0;
    for (int64_t l0 = 0; l0 < K; l0 += kGK) {
        for (int w = 0; w < R; ++w) {
            const int64_t l = l0 + lk + w;
            const int64_t gi = i0 + li, gj = j0 + li;
            xs[lk + w][li] = (gi < mx && l < K) ? (double)X[gi * ldx + l] : 0.0;
            ys[lk + w][li] = (gj < my && l < K) ? (double)Y[gj * ldy + l] : 0.0;
        }
        __syncthreads();
        const int kk_end = (int)((K - l0) < kGK ? (K - l0) : kGK);
        for (int kk = 0; kk < kk_end; ++kk) {
            double xv[R], yv[R];
            for (int a = 0; a < R; ++a) xv[a] = xs[kk][ty * R + a];
            for (int c = 0; c < R; ++c) yv[c] = ys[kk][tx * R + c];
            if (mu) {
                const double m = mu[l0 + kk];
                for (int a = 0; a < R; ++a)
                    for (int c = 0; c < R; ++c) acc[a][c] = fma(xv[a] * yv[c], m, acc[a][c]);
            } else {
                for (int a = 0; a < R; ++a)
                    for (int c = 0; c < R; ++c) acc[a][c] = fma(xv[a], yv[c], acc[a][c]);
            }
        }
        __syncthreads();
    }
}

// C^+ = V diag(mu) V^T on the first r rows / columns, mu_l = 1 / lambda_l for
// |lambda_l| > tol max|lambda|, else 0 (lambda_l = S(l, l) after convergence).
// (V_il V_jl) mu_l is the same product for (i, j) and (j, i): C^+ is exactly
// symmetric.
__global__ __launch_bounds__(256) void k_pinv_form(const double* __restrict__ S,
                                                   const double* __restrict__ V, int64_t Rp,
                                                   int64_t r, double tol, double* __restrict__ Cp,
                                                   int64_t ldcp, double* __restrict__ eig) {
    constexpr int TM = 32;
    __shared__ double xs[kGK][TM], ys[kGK][TM];
    __shared__ double mu[1024];
    __shared__ double red[256];
    const int tid = threadIdx.x;
    double mx = 0.0;
    for (int64_t l = tid; l < r; l += 256) mx = fmax(mx, fabs(S[l * Rp + l]));
    red[tid] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
        __syncthreads();
    }
    const double cut = tol * red[0];
    for (int64_t l = tid; l < r; l += 256) {
        const double lam = S[l * Rp + l];
        mu[l] = fabs(lam) > cut ? 1.0 / lam : 0.0;
        if (eig && blockIdx.x == 0 && blockIdx.y == 0) eig[l] = lam;
    }
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.y * TM, j0 = (int64_t)blockIdx.x * TM;
    double acc[2][2];
    tile_accumulate<TM>(V, Rp, r, V, Rp, r, r, mu, i0, j0, acc, xs, ys);
    const int ty = tid / 16, tx = tid % 16;
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) {
            const int64_t i = i0 + ty * 2 + a, j = j0 + tx * 2 + c;
            if (i < r && j < r) Cp[i * ldcp + j] = acc[a][c];
        }
}

// W = B C^+ (rows [row0, row0 + mw) of B; C^+ symmetric, so W(i, j) =
// sum_l B(i, l) C^+(j, l)).
__global__ __launch_bounds__(256) void k_bw(const float* __restrict__ B, int64_t ldb, int64_t mw,
                                            int64_t r, const double* __restrict__ Cp, int64_t ldcp,
                                            double* __restrict__ W) {
    __shared__ double xs[kGK][kGT], ys[kGK][kGT];
    const int64_t i0 = (int64_t)blockIdx.y * kGT, j0 = (int64_t)blockIdx.x * kGT;
    double acc[4][4];
    tile_accumulate<kGT>(B, ldb, mw, Cp, ldcp, r, r, (const double*)nullptr, i0, j0, acc, xs, ys);
    const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 4; ++c) {
            const int64_t i = i0 + ty * 4 + a, j = j0 + tx * 4 + c;
            if (i < mw && j < r) W[i * r + j] = acc[a][c];
        }
}

// Rows of A~ = W B^T (out, mr x n) or, with A given, per-tile sums of
// (A - A~)^2 and A^2 over the n x n matrix (part[2 t], part[2 t + 1]).
template <bool ERR>
__global__ __launch_bounds__(256) void k_nys_tile(const double* __restrict__ W, int64_t mw,
                                                  const float* __restrict__ B, int64_t ldb,
                                                  int64_t n, int64_t r,
                                                  const float* __restrict__ A, int64_t lda,
                                                  double* __restrict__ out, int64_t ldo,
                                                  double* __restrict__ part) {
    __shared__ double xs[kGK][kGT], ys[kGK][kGT];
    __shared__ double red[2][kJThreads];
    const int64_t i0 = (int64_t)blockIdx.y * kGT, j0 = (int64_t)blockIdx.x * kGT;
    double acc[4][4];
    tile_accumulate<kGT>(W, r, mw, B, ldb, n, r, (const double*)nullptr, i0, j0, acc, xs, ys);
    const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
    double se = 0.0, sa = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 4; ++c) {
            const int64_t i = i0 + ty * 4 + a, j = j0 + tx * 4 + c;
            if (i >= mw || j >= n) continue;
            if (ERR) {
                const double av = (double)A[i * lda + j];
                const double d = av - acc[a][c];
                se = fma(d, d, se);
                sa = fma(av, av, sa);
            } else {
                out[i * ldo + j] = acc[a][c];
            }
        }
    if (ERR) {
        block_sum2(se, sa, red);
        if (threadIdx.x == 0) {
            const int64_t t = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
            part[2 * t] = se;
            part[2 * t + 1] = sa;
        }
    }
}

// sums = (sum of part[2 t], sum of part[2 t + 1], sqrt(sums[0] / sums[1])), t in order.
__global__ __launch_bounds__(kJThreads) void k_err_sum(const double* __restrict__ part, int64_t T,
                                                       double* __restrict__ sums) {
    __shared__ double red[2][kJThreads];
    double se = 0.0, sa = 0.0;
    for (int64_t t = threadIdx.x; t < T; t += kJThreads) {
        se += part[2 * t];
        sa += part[2 * t + 1];
    }
    block_sum2(se, sa, red);
    if (threadIdx.x == 0) {
        sums[0] = se;
        sums[1] = sa;
        sums[2] = sa > 0.0 ? sqrt(se / sa) : 0.0;
    }
}

__global__ void k_jac_info(const JacState* st, int32_t* info) {
    if (threadIdx.x == 0) {
        info[0] = st->sweeps;
        info[1] = st->converged;
    }
}

inline int64_t jac_rp(int64_t r) { return (r + kJT - 1) / kJT * kJT; }
inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

size_t pinv_workspace_bytes(int64_t r) {
    if (r <= 0) return 0;
    const int64_t Rp = jac_rp(r), np = Rp / kJT;
    const int64_t nT = np * (np + 1) / 2;
    return align256(sizeof(JacState)) + 2 * align256((size_t)(Rp * Rp) * 8) +
           align256((size_t)(np * kJT * kJT) * 8) + align256((size_t)nT * 16);
}

hipError_t launch_core_pinv(const void* C, int c_f64, int64_t r, int64_t ldc, double tol,
                            int max_sweeps, double* Cp, int64_t ldcp, double* eig, int32_t* info,
                            void* ws, hipStream_t s) {
    const int64_t Rp = jac_rp(r), nb = Rp / kJB, np = nb / 2;
    const int64_t nT = np * (np + 1) / 2, nV = (Rp / kJT) * np;
    char* p = static_cast<char*>(ws);
    JacState* st = reinterpret_cast<JacState*>(p);
    p += align256(sizeof(JacState));
    double* S = reinterpret_cast<double*>(p);
    p += align256((size_t)(Rp * Rp) * 8);
    double* V = reinterpret_cast<double*>(p);
    p += align256((size_t)(Rp * Rp) * 8);
    double* Q = reinterpret_cast<double*>(p);
    p += align256((size_t)(np * kJT * kJT) * 8);
    double* part = reinterpret_cast<double*>(p);
    const unsigned gi = (unsigned)((Rp * Rp + 255) / 256);
    if (c_f64)
        k_jac_init<double><<<gi, 256, 0, s>>>(static_cast<const double*>(C), r, ldc, S, V, Rp, st);
    else
        k_jac_init<float><<<gi, 256, 0, s>>>(static_cast<const float*>(C), r, ldc, S, V, Rp, st);
    // off-diagonal Frobenius norm at most 8 Rp units of FP64 rounding of ||S||
    const double tolc = 8.0 * (double)Rp * 0x1p-53;
    const unsigned ga = (unsigned)(nT + nV);
    for (int sw = 0; sw < max_sweeps; ++sw) {
        k_jac_solve<kFull><<<(unsigned)np, kSolveThreads, 0, s>>>(S, Rp, Q, (int)nb, 0, st);
        k_jac_apply<kFull><<<ga, kJThreads, 0, s>>>(S, V, Rp, Q, (int)nb, 0, part, st);
        for (int step = 0; nb > 2 && step < nb - 1; ++step) {
            k_jac_solve<kCross><<<(unsigned)np, kSolveThreads, 0, s>>>(S, Rp, Q, (int)nb, step, st);
            k_jac_apply<kCross><<<ga, kJThreads, 0, s>>>(S, V, Rp, Q, (int)nb, step, part, st);
        }
        k_jac_flag<<<1, kJThreads, 0, s>>>(part, (int)nT, tolc, st);
    }
    const unsigned gt = (unsigned)((r + 31) / 32);
    k_pinv_form<<<dim3(gt, gt), 256, 0, s>>>(S, V, Rp, r, tol, Cp, ldcp, eig);
    if (info) k_jac_info<<<1, 64, 0, s>>>(st, info);
    return hipGetLastError();
}

size_t nystrom_workspace_bytes(int64_t n, int64_t r) {
    if (n <= 0 || r <= 0) return 0;
    const int64_t t = (n + kGT - 1) / kGT;
    return align256((size_t)(n * r) * 8) + align256((size_t)(t * t) * 16);
}

hipError_t launch_nystrom(const float* A, int64_t lda, const float* B, int64_t n, int64_t r,
                          int64_t ldb, const double* Cp, int64_t ldcp, int64_t row0, int64_t mr,
                          double* out, int64_t ldo, double* sums, void* ws, hipStream_t s) {
    double* W = static_cast<double*>(ws);
    double* part = reinterpret_cast<double*>(static_cast<char*>(ws) +
                                             align256((size_t)(n * r) * 8));
    const unsigned gr = (unsigned)((r + kGT - 1) / kGT);
    const int64_t mw = A ? n : mr;
    const float* Bw = A ? B : B + row0 * ldb;
    k_bw<<<dim3(gr, (unsigned)((mw + kGT - 1) / kGT)), 256, 0, s>>>(Bw, ldb, mw, r, Cp, ldcp, W);
    const unsigned gn = (unsigned)((n + kGT - 1) / kGT);
    const unsigned gm = (unsigned)((mw + kGT - 1) / kGT);
    if (A) {
        k_nys_tile<true><<<dim3(gn, gm), 256, 0, s>>>(W, mw, B, ldb, n, r, A, lda, nullptr, 0,
                                                      part);
        k_err_sum<<<1, kJThreads, 0, s>>>(part, (int64_t)gn * gm, sums);
    } else {
        k_nys_tile<false><<<dim3(gn, gm), 256, 0, s>>>(W, mw, B, ldb, n, r, nullptr, 0, out, ldo,
                                                       nullptr);
    }
    return hipGetLastError();
}

}  // namespace sk
