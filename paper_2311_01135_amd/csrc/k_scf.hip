// SCF steps around the Fock build, all FP64, one work group per molecule:
// Fock assembly and energy terms (compensated sums), Loewdin S^-1/2, DIIS
// extrapolation, the generalised eigenproblem through X = S^-1/2 and a
// parallel-order cyclic Jacobi solver held in LDS, the new density
// rho = C D C^T (paper section 3.1, equation "roothaan" and the iteration
// description under it), and the convergence / retire bookkeeping.
#include "kernels.h"

namespace ks {

constexpr int kScfThreads = 256;
// Work groups whose matrices sit in LDS (one molecule per group, which fills
// most of a CU's LDS: the eigensolver, and the DIIS, Loewdin, density and
// guess products) run 16 wavefronts: their steps are latency-bound loops
// between barriers, and more waves shorten each loop.
constexpr int kEighThreads = 1024;
constexpr int kScfThreadsFull = 1024;

__device__ __forceinline__ void two_sum_add(double& s, double& c, double x)
{
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x; else c += (x - t) + s;
    s = t;
}

// compensated work-group sum (every thread gets the result)
__device__ double block_sum(double s, double c, double* red)
{
    // fold the pair into one value per lane, then tree-sum with compensation
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double so = __shfl_xor(s, o, 64), co = __shfl_xor(c, o, 64);
        two_sum_add(s, c, so);
        c += co;
    }
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        red[2 * wave] = s;
        red[2 * wave + 1] = c;
    }
    __syncthreads();
    double ts = 0.0, tc = 0.0;
    for (int w = 0; w < nw; w++) {
        two_sum_add(ts, tc, red[2 * w]);
        tc += red[2 * w + 1];
    }
    __syncthreads();
    return ts + tc;
}

__device__ double block_max(double v, double* red)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < nw; w++) r = fmax(r, red[w]);
    __syncthreads();
    return r;
}

// C = op(A) op(B) for N x N row-major matrices: both operands are staged in
// LDS (sm: 2 N^2 + 4 doubles), each thread forms four adjacent outputs of a
// row; every output sums over k in ascending order.  C must not alias A or B.
__device__ void wg_matmul_full(int N, const double* __restrict__ A, bool ta, const double* __restrict__ B, bool tb,
                               double* C, double* sm)
{
    double* As = sm;             // op(A), row-major
    double* Bs = sm + N * N;     // op(B), row-major (+4 doubles of slack for the last column block)
    for (int t = threadIdx.x; t < N * N; t += blockDim.x) {
        const int r = t / N, c = t % N;
        As[t] = ta ? A[c * N + r] : A[t];
        Bs[t] = tb ? B[c * N + r] : B[t];
    }
    if (threadIdx.x < 4) Bs[N * N + threadIdx.x] = 0.0;
    __syncthreads();
    const int nb = (N + 3) / 4;
    for (int t = threadIdx.x; t < N * nb; t += blockDim.x) {
        const int i = t / nb, j0 = (t % nb) * 4;
        const double* ar = As + i * N;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int k = 0; k < N; k++) {
            const double a = ar[k];
            const double* br = Bs + k * N + j0;
            s0 += a * br[0];
            s1 += a * br[1];
            s2 += a * br[2];
            s3 += a * br[3];
        }
        double* cr = C + i * N + j0;
        cr[0] = s0;
        if (j0 + 1 < N) cr[1] = s1;
        if (j0 + 2 < N) cr[2] = s2;
        if (j0 + 3 < N) cr[3] = s3;
    }
    __syncthreads();
}

// Panel product for molecules whose operands do not fit in LDS:
// C (N x N) = alpha op(A) op(B), op(A) N x K, op(B) K x N, leading dimension N
// for all three.  C is formed in row blocks of kPanR rows; for each block K is
// walked in panels of kPanK: the op(A) panel [kPanR][kPanK + 1] and the op(B)
// panel [kPanK][4 ceil(N/4) + 4] are staged in LDS (global reads coalesced
// for either transpose) and each thread keeps up to kPanT 4 x 4 output tiles
// in registers.  Every output sums over k in ascending order.  C must not
// alias A or B.  Needs blockDim.x * kPanT >= (kPanR / 4) ceil(N / 4).
constexpr int kPanR = 64, kPanK = 32, kPanT = 4;
__host__ __device__ constexpr int panel_ldb(int n) { return ((n + 3) / 4) * 4 + 4; }
__host__ __device__ constexpr size_t panel_lds_doubles(int n) { return kPanR * (kPanK + 1) + kPanK * panel_ldb(n); }

__device__ void wg_matmul_panel(int N, int K, const double* __restrict__ A, bool ta, const double* __restrict__ B,
                                bool tb, double* C, double* sm, double alpha)
{
    const int n4 = (N + 3) / 4, ldb = panel_ldb(N), lda = kPanK + 1;
    double* As = sm;
    double* Bs = sm + kPanR * lda;
    const int ntile = (kPanR / 4) * n4;
    for (int i0 = 0; i0 < N; i0 += kPanR) {
        double acc[kPanT][16];
#pragma unroll
        for (int s = 0; s < kPanT; s++)
#pragma unroll
            for (int e = 0; e < 16; e++) acc[s][e] = 0.0;
        for (int k0 = 0; k0 < K; k0 += kPanK) {
            const int kb = min(kPanK, K - k0);
            for (int t = threadIdx.x; t < kPanR * kPanK; t += blockDim.x) {
                int r, kk;
                if (ta) { kk = t / kPanR; r = t % kPanR; }
                else { r = t / kPanK; kk = t % kPanK; }
                const int i = i0 + r, k = k0 + kk;
                double v = 0.0;
                if (i < N && kk < kb) v = ta ? A[(long)k * N + i] : A[(long)i * N + k];
                As[r * lda + kk] = v;
            }
            for (int t = threadIdx.x; t < kPanK * 4 * n4; t += blockDim.x) {
                int kk, j;
                if (tb) { j = t / kPanK; kk = t % kPanK; }
                else { kk = t / (4 * n4); j = t % (4 * n4); }
                const int k = k0 + kk;
                double v = 0.0;
                if (j < N && kk < kb) v = tb ? B[(long)j * N + k] : B[(long)k * N + j];
                Bs[kk * ldb + j] = v;
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < kPanT; s++) {
                const int tile = threadIdx.x + s * blockDim.x;
                if (tile < ntile) {
                    const double* ar = As + 4 * (tile / n4) * lda;
                    const double* br = Bs + 4 * (tile % n4);
                    for (int kk = 0; kk < kb; kk++) {
                        const double a0 = ar[kk], a1 = ar[lda + kk], a2 = ar[2 * lda + kk], a3 = ar[3 * lda + kk];
                        const double2 b01 = *(const double2*)(br + kk * ldb);
                        const double2 b23 = *(const double2*)(br + kk * ldb + 2);
                        const double av[4] = {a0, a1, a2, a3}, bv[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
                        for (int r = 0; r < 4; r++)
#pragma unroll
                            for (int c = 0; c < 4; c++) acc[s][4 * r + c] += av[r] * bv[c];
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int s = 0; s < kPanT; s++) {
            const int tile = threadIdx.x + s * blockDim.x;
            if (tile < ntile) {
                const int ib = i0 + 4 * (tile / n4), jb = 4 * (tile % n4);
#pragma unroll
                for (int r = 0; r < 4; r++)
#pragma unroll
                    for (int c = 0; c < 4; c++)
                        if (ib + r < N && jb + c < N) C[(long)(ib + r) * N + jb + c] = alpha * acc[s][4 * r + c];
            }
        }
    }
    __syncthreads();
}

// C = op(A) op(B) (N x N): operands fully staged in LDS when full, else panels.
__device__ __forceinline__ void wg_matmul(int N, const double* __restrict__ A, bool ta, const double* __restrict__ B,
                                          bool tb, double* C, double* sm, int full)
{
    if (full) wg_matmul_full(N, A, ta, B, tb, C, sm);
    else wg_matmul_panel(N, N, A, ta, B, tb, C, sm, 1.0);
}

extern __shared__ __align__(16) double smem_scf[];   // wg_matmul staging (full or panel)

struct ScfArgs {
    const MolDesc* mol;
    MolState* state;
    const double *S, *H, *X;
    double *F, *P, *J, *K, *Vxc;
    double *Fp, *C, *eps;
    double *work;           // 3 * nmat
    double *Fh, *Eh;        // diis_space * nmat
    const double* exc;
    long nmat;
    double a0;
    double e_tol, comm_tol;
    int max_iter, diis_space;
    int only_active;
};

// F = H + J - (a0/2) K + V_xc and the energy terms
// {tr PH, 1/2 tr PJ, -a0/4 tr PK, E_xc, E_nn, E}.
__global__ __launch_bounds__(kScfThreads) void fock_kernel(ScfArgs g, const double* __restrict__ Pin,
                                                           double* __restrict__ Fout, double* __restrict__ Eterms)
{
    __shared__ double red[2 * kScfThreads / 64];
    const int m = blockIdx.x;
    MolState& st = g.state[m];
    if (g.only_active && st.status != KS_MOL_ACTIVE) return;
    const MolDesc md = g.mol[m];
    const long o = md.mat0;
    const int NN = md.nbf * md.nbf;
    double s1 = 0, c1 = 0, s2 = 0, c2 = 0, s3 = 0, c3 = 0;
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        const double p = Pin[o + i], h = g.H[o + i], j = g.J[o + i], k = g.K[o + i];
        Fout[o + i] = h + j - 0.5 * g.a0 * k + g.Vxc[o + i];
        two_sum_add(s1, c1, p * h);
        two_sum_add(s2, c2, p * j);
        two_sum_add(s3, c3, p * k);
    }
    const double e1 = block_sum(s1, c1, red);
    const double e2 = 0.5 * block_sum(s2, c2, red);
    const double e3 = -0.25 * g.a0 * block_sum(s3, c3, red);
    if (threadIdx.x == 0) {
        const double exc = g.exc[m];
        double s = 0.0, c = 0.0;
        two_sum_add(s, c, e1);
        two_sum_add(s, c, e2);
        two_sum_add(s, c, e3);
        two_sum_add(s, c, exc);
        two_sum_add(s, c, md.enuc);
        const double E = s + c;
        double* et = Eterms ? Eterms + 6 * m : st.Eterms;
        et[0] = e1; et[1] = e2; et[2] = e3; et[3] = exc; et[4] = md.enuc; et[5] = E;
        if (!Eterms) {
            st.E = E;
            if (!isfinite(E)) st.status = KS_MOL_DIVERGED;
        }
    }
}

// Bordered DIIS system [B -1; -1^T 0][c; l] = [0; -1] by Gaussian elimination
// with partial pivoting; 0 if a pivot falls below 1e-12 max|B|.
__device__ int diis_solve_dev(int n, const double* B, double* c)
{
    double a[(kMaxDiis + 1) * (kMaxDiis + 2)];
    const int M = n + 1, W = M + 1;
    double bmax = 0.0;
    for (int i = 0; i < n * n; i++) bmax = fmax(bmax, fabs(B[i]));
    for (int i = 0; i < M; i++) {
        for (int j = 0; j < M; j++)
            a[i * W + j] = (i < n && j < n) ? B[i * n + j] : ((i == n && j == n) ? 0.0 : -1.0);
        a[i * W + M] = (i == n) ? -1.0 : 0.0;
    }
    for (int k = 0; k < M; k++) {
        int piv = k;
        for (int i = k + 1; i < M; i++)
            if (fabs(a[i * W + k]) > fabs(a[piv * W + k])) piv = i;
        if (fabs(a[piv * W + k]) < 1e-12 * bmax) return 0;
        if (piv != k)
            for (int j = 0; j <= M; j++) {
                const double t = a[k * W + j];
                a[k * W + j] = a[piv * W + j];
                a[piv * W + j] = t;
            }
        for (int i = k + 1; i < M; i++) {
            const double f = a[i * W + k] / a[k * W + k];
            for (int j = k; j <= M; j++) a[i * W + j] -= f * a[k * W + j];
        }
    }
    for (int i = M - 1; i >= 0; i--) {
        double s = a[i * W + M];
        for (int j = i + 1; j < M; j++) s -= a[i * W + j] * c[j];
        c[i] = s / a[i * W + i];
    }
    return 1;
}

// error vector e = X^T (F P S - S P F) X, convergence test, DIIS push and
// extrapolation, and F' = X^T Fbar X.
template <bool FULL>
__global__ __launch_bounds__(FULL ? kScfThreadsFull : kScfThreads) void diis_kernel(ScfArgs g)
{
    __shared__ double red[2 * kScfThreadsFull / 64];
    __shared__ double coef[kMaxDiis + 1];
    __shared__ int sl[kMaxDiis];
    __shared__ int nkeep;
    const int m = blockIdx.x;
    MolState& st = g.state[m];
    if (st.status != KS_MOL_ACTIVE) return;
    const MolDesc md = g.mol[m];
    const int N = md.nbf, NN = N * N;
    const long o = md.mat0;
    const double *F = g.F + o, *P = g.P + o, *S = g.S + o, *X = g.X + o;
    double *W0 = g.work + o, *W1 = g.work + g.nmat + o, *W2 = g.work + 2 * g.nmat + o;
    const int it = st.iter + 1;
    wg_matmul(N, F, false, P, false, W0, smem_scf, FULL);
    wg_matmul(N, W0, false, S, false, W1, smem_scf, FULL);     // FPS
    for (int t = threadIdx.x; t < NN; t += blockDim.x) {
        const int i = t / N, j = t % N;
        W0[t] = W1[i * N + j] - W1[j * N + i];
    }
    __syncthreads();
    wg_matmul(N, X, true, W0, false, W2, smem_scf, FULL);
    wg_matmul(N, W2, false, X, false, W0, smem_scf, FULL);     // e
    double mx = 0.0;
    for (int t = threadIdx.x; t < NN; t += blockDim.x) mx = fmax(mx, fabs(W0[t]));
    const double err = block_max(mx, red);
    const double E = st.E;
    const double dE = fabs(E - st.Eprev);
    // convergence is tested on the main grid only, from its second iteration;
    // on the coarse start grid the looser test moves the molecule on
    const bool coarse = st.stage != 0;
    const bool conv = !coarse && it > st.it_full && dE < g.e_tol && err < g.comm_tol;
    const bool to_main = coarse && ((it > 1 && dE < kCoarseETol && err < kCoarseCommTol) || it >= kCoarseMaxIter);
    const bool last = it >= g.max_iter;
    const double* Fsrc = F;
    if (conv || last) {
        if (threadIdx.x == 0) st.final_ = conv ? 1 : 2;
    } else {
        const int D = g.diis_space;
        const int slot = st.head;
        double* fh = g.Fh + (size_t)slot * g.nmat + o;
        double* eh = g.Eh + (size_t)slot * g.nmat + o;
        for (int t = threadIdx.x; t < NN; t += blockDim.x) {
            fh[t] = F[t];
            eh[t] = W0[t];
        }
        __syncthreads();
        const int head = (slot + 1) % D;
        const int nh = min(st.nhist + 1, D);
        // overlaps of the new error vector with every held one
        for (int i = 0; i < nh; i++) {
            const int s = ((head - nh + i) % D + D) % D;
            const double* ei = g.Eh + (size_t)s * g.nmat + o;
            double a = 0.0, c = 0.0;
            for (int t = threadIdx.x; t < NN; t += blockDim.x) two_sum_add(a, c, eh[t] * ei[t]);
            const double d = block_sum(a, c, red);
            if (threadIdx.x == 0) {
                st.B[slot * kMaxDiis + s] = d;
                st.B[s * kMaxDiis + slot] = d;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int n = nh, ok = 0;
            double Bm[kMaxDiis * kMaxDiis], cv[kMaxDiis + 1];
            while (!ok && n > 0) {
                for (int i = 0; i < n; i++) sl[i] = ((head - n + i) % D + D) % D;
                for (int i = 0; i < n; i++)
                    for (int j = 0; j < n; j++) Bm[i * n + j] = st.B[sl[i] * kMaxDiis + sl[j]];
                ok = diis_solve_dev(n, Bm, cv);
                if (!ok) n--;
            }
            for (int i = 0; i < n; i++) coef[i] = cv[i];
            nkeep = n;
            st.nhist = n;
            st.head = head;
        }
        __syncthreads();
        const int n = nkeep;
        for (int t = threadIdx.x; t < NN; t += blockDim.x) {
            double s = 0.0;
            for (int i = 0; i < n; i++) s += coef[i] * g.Fh[(size_t)sl[i] * g.nmat + o + t];
            W1[t] = s;
        }
        __syncthreads();
        Fsrc = W1;
    }
    wg_matmul(N, X, true, Fsrc, false, W2, smem_scf, FULL);
    wg_matmul(N, W2, false, X, false, g.Fp + o, smem_scf, FULL);
    if (threadIdx.x == 0) {
        st.iter = it;
        st.err = err;
        st.dE = E - st.Eprev;
        if (!(conv || last)) st.Eprev = E;
        if (to_main && !last) {
            // the next F comes from the main grid; the DIIS history of the
            // coarse-grid iterations stays (restarting it cost 0.4 more
            // main-grid iterations per molecule on 9-11-heavy-atom trees)
            st.stage = 0;
            st.it_full = it + 1;
        }
    }
}

// Diagonal atomic-occupation density from the shells' neutral-atom
// occupations (STO-3G: H 1s 1; C/N/O/F 1s 2, 2s 2, 2p (Z-4)/3 per component;
// 6-31G: the valence split evenly over the inner and outer shells), scaled
// so that tr(P S) = tr(P) = N_e.
__global__ __launch_bounds__(kScfThreads) void atom_guess_kernel(const MolDesc* __restrict__ mols,
                                                                 const Shell* __restrict__ shells,
                                                                 const double* __restrict__ Zat, double* __restrict__ P)
{
    __shared__ double red[2 * kScfThreads / 64];
    const int m = blockIdx.x;
    const MolDesc md = mols[m];
    const int N = md.nbf;
    double* Pm = P + md.mat0;
    for (int t = threadIdx.x; t < N * N; t += blockDim.x) Pm[t] = 0.0;
    __syncthreads();
    double s = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < md.nshell; i += blockDim.x) {
        const Shell& sh = shells[md.shell0 + i];
        const double occ = sh.occ;      // neutral-atom occupation per function (set with the basis)
        for (int k = 0; k < (sh.L ? 3 : 1); k++) {
            Pm[(sh.ao + k) * N + sh.ao + k] = occ;
            two_sum_add(s, c, occ);
        }
    }
    const double tot = block_sum(s, c, red);
    const double scale = 2.0 * md.nocc / tot;
    for (int i = threadIdx.x; i < N; i += blockDim.x) Pm[i * N + i] *= scale;
}

// W = X^T A X (guess from the core Hamiltonian)
template <bool FULL>
__global__ __launch_bounds__(FULL ? kScfThreadsFull : kScfThreads) void xtax_kernel(ScfArgs g, const double* __restrict__ A)
{
    const int m = blockIdx.x;
    const MolDesc md = g.mol[m];
    const long o = md.mat0;
    wg_matmul(md.nbf, g.X + o, true, A + o, false, g.work + o, smem_scf, FULL);
    wg_matmul(md.nbf, g.work + o, false, g.X + o, false, g.Fp + o, smem_scf, FULL);
}

// Symmetric eigenproblem, parallel-order cyclic Jacobi (round-robin pairing:
// every step rotates N/2 disjoint (p, q) planes at once), matrix and vectors in
// LDS.  Rotation: theta = (a_qq - a_pp)/(2 a_pq), t = sgn(theta)/(|theta| +
// sqrt(theta^2 + 1)), c = 1/sqrt(1 + t^2), s = t c; rows then columns.
// Output: ascending eigenvalues vals[N], eigenvectors as columns of vecs.
// Warm start (SCF iterations): with the previous iteration's eigenvectors W
// (warm), the rotations start from V = W on A = W^T F' W, which is nearly
// diagonal close to self-consistency, so few sweeps remain; the sorted
// vectors are kept in `keep` for the next iteration.  tmp: N^2 scratch.
template <bool GLOBAL>
__global__ __launch_bounds__(GLOBAL ? kScfThreads : kEighThreads) void eigh_kernel(const MolDesc* __restrict__ mols,
                                                           const MolState* __restrict__ state, int only_active,
                                                           const double* __restrict__ src, double* __restrict__ vecs,
                                                           double* __restrict__ vals, const double* __restrict__ warm,
                                                           double* __restrict__ keep, double* __restrict__ tmp,
                                                           int* __restrict__ have_warm, double* __restrict__ gws,
                                                           long nmat)
{
    const int m = blockIdx.x;
    if (only_active && state[m].status != KS_MOL_ACTIVE) return;
    const MolDesc md = mols[m];
    const int N = md.nbf, NN = N * N;
    extern __shared__ __align__(16) unsigned char smem_eig[];
    // matrix and vectors in LDS, or (GLOBAL: molecules too large for LDS) in
    // global memory after the warm-start scratch region of gws
    double* A = GLOBAL ? gws + nmat + md.mat0 : (double*)smem_eig;
    double* Vv = GLOBAL ? gws + 2 * nmat + md.mat0 : A + NN;
    __shared__ int rp[kMaxNbf / 2 + 1], rq[kMaxNbf / 2 + 1];
    __shared__ double rc[kMaxNbf / 2 + 1], rs[kMaxNbf / 2 + 1];
    __shared__ double red[2 * kEighThreads / 64];
    __shared__ int rank_of[kMaxNbf];
    const double* a0 = src + md.mat0;
    const bool use_warm = warm && have_warm[m];
    for (int t = threadIdx.x; t < NN; t += blockDim.x) {
        A[t] = a0[t];
        Vv[t] = use_warm ? warm[md.mat0 + t] : ((t / N == t % N) ? 1.0 : 0.0);
    }
    __syncthreads();
    if (use_warm && GLOBAL) {
        double* T = tmp + md.mat0;
        wg_matmul_panel(N, N, A, false, Vv, false, T, (double*)smem_eig, 1.0);   // T = F' W
        wg_matmul_panel(N, N, Vv, true, T, false, A, (double*)smem_eig, 1.0);    // A = W^T T
        for (int t = threadIdx.x; t < NN; t += blockDim.x) {      // symmetrise
            const int i = t / N, j = t % N;
            if (i < j) {
                const double s = 0.5 * (A[i * N + j] + A[j * N + i]);
                A[i * N + j] = s;
                A[j * N + i] = s;
            }
        }
        __syncthreads();
    } else if (use_warm) {
        double* T = tmp + md.mat0;
        for (int t = threadIdx.x; t < NN; t += blockDim.x) {      // T = F' W
            const int i = t / N, j = t % N;
            double s = 0.0;
            for (int k = 0; k < N; k++) s += A[i * N + k] * Vv[k * N + j];
            T[t] = s;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < NN; t += blockDim.x) {      // A = W^T T
            const int i = t / N, j = t % N;
            double s = 0.0;
            for (int k = 0; k < N; k++) s += Vv[k * N + i] * T[k * N + j];
            A[t] = s;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < NN; t += blockDim.x) {      // symmetrise
            const int i = t / N, j = t % N;
            if (i < j) {
                const double s = 0.5 * (A[i * N + j] + A[j * N + i]);
                A[i * N + j] = s;
                A[j * N + i] = s;
            }
        }
        __syncthreads();
    }
    const int nn = N + (N & 1), half = nn / 2;
    for (int sweep = 0; sweep < 60; sweep++) {
        double off = 0.0, oc = 0.0, tot = 0.0, tc = 0.0;
        for (int t = threadIdx.x; t < NN; t += blockDim.x) {
            const double v = A[t] * A[t];
            two_sum_add(tot, tc, v);
            if (t / N != t % N) two_sum_add(off, oc, v);
        }
        const double offs = block_sum(off, oc, red);
        const double tots = block_sum(tot, tc, red);
        if (offs <= 1e-30 * tots || offs == 0.0) break;
        for (int step = 0; step < nn - 1; step++) {
            if (threadIdx.x < half) {
                const int k = threadIdx.x;
                int p, q;
                if (k == 0) { p = nn - 1; q = step; }
                else { p = (step + k) % (nn - 1); q = (step - k + nn - 1) % (nn - 1); }
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < N) {
                    const double apq = A[p * N + q];
                    if (apq != 0.0) {
                        const double th = (A[q * N + q] - A[p * N + p]) / (2.0 * apq);
                        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                    }
                }
                rp[k] = p; rq[k] = q; rc[k] = c; rs[k] = s;
            }
            __syncthreads();
            for (int idx = threadIdx.x; idx < half * N; idx += blockDim.x) {
                const int k = idx / N, j = idx % N;
                if (rq[k] >= N || rs[k] == 0.0) continue;
                const int p = rp[k], q = rq[k];
                const double c = rc[k], s = rs[k];
                const double apj = A[p * N + j], aqj = A[q * N + j];
                A[p * N + j] = c * apj - s * aqj;
                A[q * N + j] = s * apj + c * aqj;
            }
            __syncthreads();
            // columns: lanes take the planes of one row (contiguous columns)
            for (int idx = threadIdx.x; idx < half * N; idx += blockDim.x) {
                const int i = idx / half, k = idx % half;
                if (rq[k] >= N || rs[k] == 0.0) continue;
                const int p = rp[k], q = rq[k];
                const double c = rc[k], s = rs[k];
                const double aip = A[i * N + p], aiq = A[i * N + q];
                A[i * N + p] = c * aip - s * aiq;
                A[i * N + q] = s * aip + c * aiq;
                const double vip = Vv[i * N + p], viq = Vv[i * N + q];
                Vv[i * N + p] = c * vip - s * viq;
                Vv[i * N + q] = s * vip + c * viq;
            }
            __syncthreads();
        }
    }
    // ascending order (ties by index)
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double wi = A[i * N + i];
        int r = 0;
        for (int j = 0; j < N; j++) {
            const double wj = A[j * N + j];
            if (wj < wi || (wj == wi && j < i)) r++;
        }
        rank_of[i] = r;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < NN; t += blockDim.x) {
        const int i = t / N, k = t % N;   // component i of eigenvector k
        vecs[md.mat0 + i * N + rank_of[k]] = Vv[i * N + k];
        if (keep) keep[md.mat0 + i * N + rank_of[k]] = Vv[i * N + k];
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x) vals[md.ao0 + rank_of[i]] = A[i * N + i];
    if (keep && threadIdx.x == 0) have_warm[m] = 1;
}

// X = U s^-1/2 U^T from eigh(S) (vectors in C, values in eps); flags near-singular S.
// The scaled vectors W = U s^-1/2 go to work, then X = W U^T.
template <bool FULL>
__global__ __launch_bounds__(FULL ? kScfThreadsFull : kScfThreads) void lowdin_kernel(ScfArgs g)
{
    const int m = blockIdx.x;
    const MolDesc md = g.mol[m];
    const int N = md.nbf;
    const long o = md.mat0;
    const double* u = g.C + o;
    const double* w = g.eps + md.ao0;
    if (threadIdx.x == 0 && w[0] < 1e-8) g.state[m].status = -1;
    for (int t = threadIdx.x; t < N * N; t += blockDim.x) g.work[o + t] = u[t] / sqrt(fmax(w[t % N], 1e-300));
    __syncthreads();
    wg_matmul(N, g.work + o, false, u, true, (double*)g.X + o, smem_scf, FULL);
}

// C = X C'; unless this was the final iteration, P = 2 C_occ C_occ^T.
// Final iterations keep P (the density that produced the last F) and retire.
template <bool FULL>
__global__ __launch_bounds__(FULL ? kScfThreadsFull : kScfThreads) void density_kernel(ScfArgs g, int guess)
{
    const int m = blockIdx.x;
    MolState& st = g.state[m];
    if (!guess && st.status != KS_MOL_ACTIVE) return;
    const MolDesc md = g.mol[m];
    const int N = md.nbf, no = md.nocc;
    const long o = md.mat0;
    const int fin = guess ? 0 : st.final_;
    wg_matmul(N, g.X + o, false, g.Fp + o, false, g.C + o, smem_scf, FULL);   // Fp holds C' here
    if (!fin && !FULL) {
        wg_matmul_panel(N, no, g.C + o, false, g.C + o, true, g.P + o, smem_scf, 2.0);
    } else if (!fin) {
        for (int t = threadIdx.x; t < N * N; t += blockDim.x) smem_scf[t] = g.C[o + t];
        __syncthreads();
        for (int t = threadIdx.x; t < N * N; t += blockDim.x) {
            const int i = t / N, j = t % N;
            double s = 0.0;
            for (int k = 0; k < no; k++) s += smem_scf[i * N + k] * smem_scf[j * N + k];
            g.P[o + t] = 2.0 * s;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && fin) {
        st.status = fin == 1 ? KS_MOL_CONVERGED : KS_MOL_MAXITER;
        st.final_ = 0;
    }
}

__global__ void count_active_kernel(const MolState* __restrict__ state, int n, int* out)
{
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int c = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) c += state[i].status == KS_MOL_ACTIVE;
    atomicAdd(&cnt, c);
    __syncthreads();
    if (threadIdx.x == 0) *out = cnt;
}

// ---------------------------------------------------------------------------
static size_t max_nbf(const ks_batch* b)
{
    int maxn = 0;
    for (auto& m : b->mol) maxn = std::max(maxn, m.nbf);
    return (size_t)maxn;
}

// LDS available to dynamic allocations of the SCF kernels (their static
// arrays take a few KB)
constexpr size_t kScfLds = 152 * 1024;

static bool matmul_fits(const ks_batch* b)
{
    const size_t n = max_nbf(b);
    return sizeof(double) * (2 * n * n + 4) <= kScfLds;
}

static ScfArgs scf_args(ks_batch* b, bool only_active)
{
    ScfArgs g;
    g.mol = b->d_mol;
    g.state = b->d_state;
    g.S = b->d_S; g.H = b->d_H; g.X = b->d_X;
    g.F = b->d_F; g.P = b->d_P; g.J = b->d_J; g.K = b->d_K; g.Vxc = b->d_Vxc;
    g.Fp = b->d_Fp; g.C = b->d_C; g.eps = b->d_eps;
    g.work = b->d_work;
    g.Fh = b->d_Fh; g.Eh = b->d_Eh;
    g.exc = b->d_exc;
    g.nmat = b->nmat;
    g.a0 = b->a0;
    g.e_tol = b->opt.e_tol;
    g.comm_tol = b->opt.comm_tol;
    g.max_iter = b->opt.max_iter;
    g.diis_space = b->opt.diis_space;
    g.only_active = only_active;
    return g;
}

// dynamic LDS of the kernels that call wg_matmul
static size_t matmul_lds(const ks_batch* b)
{
    const size_t n = max_nbf(b);
    return matmul_fits(b) ? sizeof(double) * (2 * n * n + 4) : sizeof(double) * panel_lds_doubles((int)n);
}

static bool eigh_fits(const ks_batch* b)
{
    const size_t n = max_nbf(b);
    return 2 * sizeof(double) * n * n <= kScfLds;
}

// matrix and vectors in LDS, or (global mode) the panel staging of the
// warm-start products
static size_t eigh_lds(const ks_batch* b)
{
    const size_t n = max_nbf(b);
    return eigh_fits(b) ? 2 * sizeof(double) * n * n : sizeof(double) * panel_lds_doubles((int)n);
}

// One work group per molecule: kern<true> when wg_matmul's operands fit in
// LDS whole, else kern<false> (panel staging).
template <typename K1, typename K0, typename... Args>
static ks_status launch_mm(ks_batch* b, K1 kfull, K0 kpanel, Args... args)
{
    const bool full = matmul_fits(b);
    const size_t lds = matmul_lds(b);
    KS_HIP(hipFuncSetAttribute(full ? (const void*)kfull : (const void*)kpanel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (full) hipLaunchKernelGGL(kfull, dim3(b->n_mol), dim3(kScfThreadsFull), lds, b->stream, args...);
    else hipLaunchKernelGGL(kpanel, dim3(b->n_mol), dim3(kScfThreads), lds, b->stream, args...);
    KS_HIP(hipGetLastError());
    return KS_OK;
}

// warm == nullptr: cold start from the identity.  Otherwise warm/keep hold the
// previous eigenvectors (read when have_warm[m], then overwritten).
static ks_status run_eigh(ks_batch* b, bool only_active, const double* src, double* vecs, double* vals,
                          double* warm = nullptr)
{
    const size_t lds = eigh_lds(b);
    const void* fn = eigh_fits(b) ? (const void*)eigh_kernel<false> : (const void*)eigh_kernel<true>;
    KS_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (eigh_fits(b))
        hipLaunchKernelGGL(eigh_kernel<false>, dim3(b->n_mol), dim3(kEighThreads), lds, b->stream, b->d_mol,
                           b->d_state, (int)only_active, src, vecs, vals, (const double*)warm, warm,
                           warm ? b->d_work : nullptr, warm ? b->d_have_warm : nullptr, nullptr, b->nmat);
    else
        hipLaunchKernelGGL(eigh_kernel<true>, dim3(b->n_mol), dim3(kScfThreads), lds, b->stream, b->d_mol,
                           b->d_state, (int)only_active, src, vecs, vals, (const double*)warm, warm,
                           warm ? b->d_work : nullptr, warm ? b->d_have_warm : nullptr, b->d_work, b->nmat);
    KS_HIP(hipGetLastError());
    return KS_OK;
}

ks_status launch_fock(ks_batch* b, const double* P, const double* J, const double* K, const double* Vxc, double* F,
                      bool only_active, double* d_eterms)
{
    KTimer tm(b, "fock");
    ScfArgs g = scf_args(b, only_active);
    g.J = (double*)J;
    g.K = (double*)K;
    g.Vxc = (double*)Vxc;
    hipLaunchKernelGGL(fock_kernel, dim3(b->n_mol), dim3(kScfThreads), 0, b->stream, g, P, F, d_eterms);
    KS_HIP(hipGetLastError());
    return KS_OK;
}

ks_status launch_lowdin(ks_batch* b)
{
    KTimer tm(b, "lowdin");
    ks_status st = run_eigh(b, false, b->d_S, b->d_C, b->d_eps);
    if (st) return st;
    return launch_mm(b, lowdin_kernel<true>, lowdin_kernel<false>, scf_args(b, false));
}

ks_status launch_guess(ks_batch* b)
{
    KTimer tm(b, "guess");
    if (b->opt.guess == KS_GUESS_ATOM) {
        hipLaunchKernelGGL(atom_guess_kernel, dim3(b->n_mol), dim3(kScfThreads), 0, b->stream, b->d_mol, b->d_shells,
                           b->d_Zc, b->d_P);
        KS_HIP(hipGetLastError());
        return KS_OK;
    }
    ScfArgs g = scf_args(b, false);
    ks_status st = launch_mm(b, xtax_kernel<true>, xtax_kernel<false>, g, (const double*)b->d_H);
    if (st) return st;
    st = run_eigh(b, false, b->d_Fp, b->d_Fp, b->d_eps);
    if (st) return st;
    return launch_mm(b, density_kernel<true>, density_kernel<false>, g, 1);
}

ks_status launch_iteration_tail(ks_batch* b)
{
    ScfArgs g = scf_args(b, true);
    {
        KTimer tm(b, "diis");
        ks_status st = launch_mm(b, diis_kernel<true>, diis_kernel<false>, g);
        if (st) return st;
    }
    {
        KTimer tm(b, "eigh");
        ks_status st = run_eigh(b, true, b->d_Fp, b->d_Fp, b->d_eps, b->d_Cp);
        if (st) return st;
    }
    {
        KTimer tm(b, "density");
        ks_status st = launch_mm(b, density_kernel<true>, density_kernel<false>, g, 0);
        if (st) return st;
    }
    return KS_OK;
}

ks_status launch_count_active(ks_batch* b)
{
    hipLaunchKernelGGL(count_active_kernel, dim3(1), dim3(256), 0, b->stream, b->d_state, b->n_mol, b->d_nactive);
    KS_HIP(hipGetLastError());
    return KS_OK;
}

}  // namespace ks
