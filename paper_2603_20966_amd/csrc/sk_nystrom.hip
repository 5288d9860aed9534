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

// Rotation annihilating a_pq of the symmetric 2x2 [[app, apq], [apq, aqq]]:
// J = [[c, s], [-s, c]] with t = tan theta the smaller root of
// t^2 + 2 tau t - 1 = 0, tau = (aqq - app) / (2 apq).  Identity when apq is zero
// or negligible against sqrt(|app aqq|).
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, double& c,
                                                double& s) {
    c = 1.0;
    s = 0.0;
    if (apq == 0.0 || fabs(apq) <= 0x1p-60 * sqrt(fabs(app)) * sqrt(fabs(aqq))) return;
    const double tau = (aqq - app) / (2.0 * apq);
    double t;
    if (fabs(tau) > 1e150) {
        t = 0.5 / tau;
    } else {
        t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    }
    c = 1.0 / sqrt(1.0 + t * t);
    s = t * c;
}

// One cyclic sweep of parallel 2x2 rotations on each pair's 32 x 32 diagonal
// tile; Q_P (32 x 32, row-major) = the product of the sweep's rotations.
__global__ __launch_bounds__(kJThreads) void k_jac_solve(const double* __restrict__ S, int64_t Rp,
                                                         double* __restrict__ Q, int nb, int step,
                                                         const JacState* st) {
    if (st->converged) return;
    __shared__ double a[2][kJT][kJP];
    __shared__ double q[2][kJT][kJP];
    __shared__ double self_c[kJT], other_c[kJT];
    __shared__ int partner[kJT];
    const int tid = threadIdx.x;
    int I, J;
    circle_pair(nb, step, blockIdx.x, I, J);
    for (int u = 0; u < kPerThread; ++u) {
        const int e = tid + kJThreads * u, x = e / kJT, y = e % kJT;
        a[0][x][y] = S[tile_row(I, J, x) * Rp + tile_row(I, J, y)];
        q[0][x][y] = (x == y) ? 1.0 : 0.0;
    }
    __syncthreads();
    int cur = 0;
    for (int t = 0; t < kJT - 1; ++t) {
        if (tid < kJT / 2) {
            int p, r;
            circle_pair(kJT, t, tid, p, r);
            if (p > r) {
                const int w = p;
                p = r;
                r = w;
            }
            double c, s;
            jacobi_rotation(a[cur][p][p], a[cur][r][r], a[cur][p][r], c, s);
            // column p of J is (c, -s) on rows (p, r); column r is (s, c)
            self_c[p] = c;
            other_c[p] = -s;
            partner[p] = r;
            self_c[r] = c;
            other_c[r] = s;
            partner[r] = p;
        }
        __syncthreads();
        const int nxt = cur ^ 1;
        for (int u = 0; u < kPerThread; ++u) {
            const int e = tid + kJThreads * u, x = e / kJT, y = e % kJT;
            const int xb = partner[x], yb = partner[y];
            const double sx = self_c[x], ox = other_c[x], sy = self_c[y], oy = other_c[y];
            // (J^T A J)(x, y) as (P1 + P4) + (P2 + P3): the same terms for (y, x), so the
            // tile stays exactly symmetric
            const double p1 = (sx * sy) * a[cur][x][y];
            const double p4 = (ox * oy) * a[cur][xb][yb];
            const double p2 = (sx * oy) * a[cur][x][yb];
            const double p3 = (ox * sy) * a[cur][xb][y];
            double v = (p1 + p4) + (p2 + p3);
            if (y == xb && ox != 0.0) v = 0.0;     // the entry the rotation annihilates
            a[nxt][x][y] = v;
            q[nxt][x][y] = sy * q[cur][x][y] + oy * q[cur][x][yb];
        }
        __syncthreads();
        cur = nxt;
    }
    double* Qp = Q + (int64_t)blockIdx.x * kJT * kJT;
    for (int u = 0; u < kPerThread; ++u) {
        const int e = tid + kJThreads * u;
        Qp[e] = q[cur][e / kJT][e % kJT];
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
        circle_pair(nb, step, pa, Ia, Ja);
        circle_pair(nb, step, pb, Ib, Jb);
        for (int v = 0; v < kPerThread; ++v) {
            const int e = tid + kJThreads * v, i = e / kJT, j = e % kJT;
            x[i][j] = S[tile_row(Ia, Ja, i) * Rp + tile_row(Ib, Jb, j)];
            qa[i][j] = Q[(int64_t)pa * kJT * kJT + e];
            qb[i][j] = Q[(int64_t)pb * kJT * kJT + e];
        }
        __syncthreads();
        for (int v = 0; v < kPerThread; ++v) {            // U = X Q_b
            const int e = tid + kJThreads * v, i = e / kJT, j = e % kJT;
            double acc = 0.0;
            for (int z = 0; z < kJT; ++z) acc = fma(x[i][z], qb[z][j], acc);
            u[i][j] = acc;
        }
        __syncthreads();
        double tv[kPerThread];
        for (int v = 0; v < kPerThread; ++v) {            // T = Q_a^T U
            const int e = tid + kJThreads * v, i = e / kJT, j = e % kJT;
            double acc = 0.0;
            for (int z = 0; z < kJT; ++z) acc = fma(qa[z][i], u[z][j], acc);
            tv[v] = acc;
        }
        __syncthreads();
        for (int v = 0; v < kPerThread; ++v) {
            const int e = tid + kJThreads * v;
            x[e / kJT][e % kJT] = tv[v];
        }
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
    circle_pair(nb, step, pc, Ic, Jc);
    for (int v = 0; v < kPerThread; ++v) {
        const int e = tid + kJThreads * v, i = e / kJT, j = e % kJT;
        x[i][j] = V[((int64_t)rb * kJT + i) * Rp + tile_row(Ic, Jc, j)];
        qa[i][j] = Q[(int64_t)pc * kJT * kJT + e];
    }
    __syncthreads();
    for (int v = 0; v < kPerThread; ++v) {
        const int e = tid + kJThreads * v, i = e / kJT, j = e % kJT;
        double acc = 0.0;
        for (int z = 0; z < kJT; ++z) acc = fma(x[i][z], qa[z][j], acc);
        V[((int64_t)rb * kJT + i) * Rp + tile_row(Ic, Jc, j)] = acc;
    }
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
// when mu is given), l ascending, for a 64 x 64 tile per workgroup (256
// threads, 4 x 4 outputs each, l in chunks of 16 staged in LDS).
constexpr int kGT = 64, kGK = 16;

template <typename TX, typename TY>
__device__ __forceinline__ void tile_accumulate(const TX* __restrict__ X, int64_t ldx, int64_t mx,
                                                const TY* __restrict__ Y, int64_t ldy, int64_t my,
                                                int64_t K, const double* mu, int64_t i0,
                                                int64_t j0, double acc[4][4],
                                                double (*xs)[kGT], double (*ys)[kGT]) {
    const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
    const int li = tid / 4, lk = (tid % 4) * 4;
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
    for (int64_t l0 = 0; l0 < K; l0 += kGK) {
        for (int w = 0; w < 4; ++w) {
            const int64_t l = l0 + lk + w;
            const int64_t gi = i0 + li, gj = j0 + li;
            xs[lk + w][li] = (gi < mx && l < K) ? (double)X[gi * ldx + l] : 0.0;
            double yv = (gj < my && l < K) ? (double)Y[gj * ldy + l] : 0.0;
            ys[lk + w][li] = yv;
        }
        __syncthreads();
        const int kk_end = (int)((K - l0) < kGK ? (K - l0) : kGK);
        for (int kk = 0; kk < kk_end; ++kk) {
            double xv[4], yv[4];
            for (int a = 0; a < 4; ++a) xv[a] = xs[kk][ty * 4 + a];
            for (int c = 0; c < 4; ++c) yv[c] = ys[kk][tx * 4 + c];
            if (mu) {
                const double m = mu[l0 + kk];
                for (int a = 0; a < 4; ++a)
                    for (int c = 0; c < 4; ++c) acc[a][c] = fma(xv[a] * yv[c], m, acc[a][c]);
            } else {
                for (int a = 0; a < 4; ++a)
                    for (int c = 0; c < 4; ++c) acc[a][c] = fma(xv[a], yv[c], acc[a][c]);
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
    __shared__ double xs[kGK][kGT], ys[kGK][kGT];
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
    const int64_t i0 = (int64_t)blockIdx.y * kGT, j0 = (int64_t)blockIdx.x * kGT;
    double acc[4][4];
    tile_accumulate(V, Rp, r, V, Rp, r, r, mu, i0, j0, acc, xs, ys);
    const int ty = tid / 16, tx = tid % 16;
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 4; ++c) {
            const int64_t i = i0 + ty * 4 + a, j = j0 + tx * 4 + c;
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
    tile_accumulate(B, ldb, mw, Cp, ldcp, r, r, (const double*)nullptr, i0, j0, acc, xs, ys);
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
    tile_accumulate(W, r, mw, B, ldb, n, r, (const double*)nullptr, i0, j0, acc, xs, ys);
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
    for (int sw = 0; sw < max_sweeps; ++sw) {
        for (int step = 0; step < nb - 1; ++step) {
            k_jac_solve<<<(unsigned)np, kJThreads, 0, s>>>(S, Rp, Q, (int)nb, step, st);
            k_jac_apply<<<(unsigned)(nT + nV), kJThreads, 0, s>>>(S, V, Rp, Q, (int)nb, step, part,
                                                                   st);
        }
        k_jac_flag<<<1, kJThreads, 0, s>>>(part, (int)nT, tolc, st);
    }
    const unsigned gt = (unsigned)((r + kGT - 1) / kGT);
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
