// J/K digestion of the packed unique ERIs against the density (paper
// section 3.1: J_kl = sum_ij I_ijkl rho_ij, K_il = sum_jk I_ijkl rho_jk up to
// the -1/2; section 3.2: the 8-fold symmetry cuts the digestion FLOPs 8x;
// section 5 "Bottleneck": the ERIs act as a matrix M on x = flatten(rho)).
//
// Design for gfx950: one work group per (molecule, chunk of its quartets).
// The density, J and K of that molecule sit in LDS (3 N^2 values, <= 160 KB),
// the group streams its share of each class's ERIs from HBM (component-major,
// so a wavefront reads contiguous 256 B rows), and each lane scatters the six
// shell blocks J_ab, J_cd, K_ac, K_bc, K_ad, K_bd of its quartet with LDS
// atomics.  For a unique shell quartet Q with stabiliser size s (a = b,
// c = d and {ab} = {cd} each double it) summing all 8 permutations and
// dividing by s gives the orbit sum, so per component
//   AJ[ab] += 2/s I P_cd,  AJ[cd] += 2/s I P_ab,
//   AK[ac] += 1/s I P_bd,  AK[bc] += 1/s I P_ad,  AK[ad] += 1/s I P_bc,  AK[bd] += 1/s I P_ac,
// and J = AJ + AJ^T, K = AK + AK^T after the chunks are summed.  The
// contraction is a matrix-vector product with no reuse dimension, so it runs
// on VALU FMAs, bounded by the HBM stream of the integrals.
#include "kernels.h"
#include "jk_scatter.h"

#include <type_traits>

namespace ks {

__device__ __forceinline__ void decode_quartet_jk(int c, long q, int nket, int& i, int& j)
{
    if (class_tri(c)) {
        long ii = (long)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
        while (ii * (ii + 1) / 2 > q) ii--;
        while ((ii + 1) * (ii + 2) / 2 <= q) ii++;
        i = (int)ii;
        j = (int)(q - ii * (ii + 1) / 2);
    } else {
        i = (int)(q / nket);
        j = (int)(q % nket);
    }
}

struct JkArgs {
    const MolDesc* mol;
    const MolState* state;
    const JkItem* items;
    const int2* pao[3];     // per pair of each pair class: (AO of sa | same shell << 16, AO of sb)
    const void* eri[kNClass];
    long nq[kNClass];
    const double* P;
    const double* Pref;     // incremental build: digest P - Pref (NULL: P itself)
    const double* dP;       // global mode: the digested density, materialised by delta_kernel
    void* part;             // [items][2][np_max^2]
    long part_stride;       // np_max^2
    int only_active;
};

// 8 wavefronts per group: the LDS holds one molecule's P, J, K, so one group
// fills a CU, and the waves hide the latency of the integral stream.
constexpr int kJkThreads = 512;


// Ps, AJ, AK: N x N matrices in LDS with row stride ld.
template <int LA, int LB, int LC, int LD, typename S, typename A>
__device__ __forceinline__ void digest_class(const JkArgs& g, const MolDesc& md, int chunk, int nchunk,
                                             const A* __restrict__ Ps, A* AJ, A* AK, int ld)
{
    constexpr int C = (LA + LB == 0) ? 0 : (LA + LB == 1 ? (LC + LD == 0 ? 1 : 2) : (LC + LD == 0 ? 3 : (LC + LD == 1 ? 4 : 5)));
    constexpr int NA = LA ? 3 : 1, NB = LB ? 3 : 1, NC = LC ? 3 : 1, ND = LD ? 3 : 1;
    constexpr int NCOMP = NA * NB * NC * ND;
    const long nq = md.nq[C];
    const long lo = nq * chunk / nchunk, hi = nq * (chunk + 1) / nchunk;
    const S* __restrict__ eri = (const S*)g.eri[C];
    const long NQ = g.nq[C];
    const int2* __restrict__ pb = g.pao[class_bra(C)] + md.pair0[class_bra(C)];
    const int2* __restrict__ pk = g.pao[class_ket(C)] + md.pair0[class_ket(C)];
    const int nket = md.npair[class_ket(C)];
    const int step = blockDim.x;
    // Each lane takes U of its quartets (q, q + step, ...) per batch: their
    // integrals and pair-table entries are loaded before the first scatter
    // (a pair-table load per quartet in front of its scatter left its
    // latency exposed), and in classes of up to 27 components the next
    // batch's integrals are loaded before this batch's scatter.  The
    // integrals stay in the storage type until use.
    constexpr int U = sizeof(S) == 4 ? (NCOMP <= 3 ? 4 : 1)
                                     : (NCOMP == 1 ? 4 : NCOMP <= 3 ? 2 : 1);
    constexpr bool kAhead = NCOMP <= 27;
    // segmented J_ab sums for the classes with at most three bra functions
    // (the pp-bra classes keep the uniform-bra sum and per-lane adds, whose
    // registers the segmented form would spill)
    constexpr bool kFull = NA * NB <= 3;
    const long ustep = (long)U * step;
    const size_t qoff = md.q0[C];
    // (i, j) of the lane's quartet advanced by step in row-major order over
    // the triangle (j <= i) or the rectangle (j < nket)
    auto advance = [&](int& i2, int& j2) {
        j2 += step;
        if (class_tri(C)) {
            while (j2 > i2) { j2 -= i2 + 1; i2++; }
        } else {
            while (j2 >= nket) { j2 -= nket; i2++; }
        }
    };
    auto load = [&](long qb, S (&dst)[U][NCOMP]) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const long qu = qb + (long)u * step;
            if (qu < hi) {
#pragma unroll
                for (int k = 0; k < NCOMP; k++) dst[u][k] = eri[(size_t)k * NQ + qoff + qu];
            }
        }
    };
    // kFull: the loop runs while the wavefront's first lane (its smallest q)
    // has quartets left, so that all 64 lanes reach every scatter together
    long q = lo + threadIdx.x;
    const long lane0 = kFull ? (long)(threadIdx.x & 63) : 0;
    if (q - lane0 >= hi) return;
    int ci, cj;
    decode_quartet_jk(C, q, nket, ci, cj);
    S cur[U][NCOMP];
    if constexpr (kAhead) load(q, cur);
    for (; q - lane0 < hi; q += ustep) {
        S I[U][NCOMP];
        if constexpr (kAhead) {
#pragma unroll
            for (int u = 0; u < U; u++)
#pragma unroll
                for (int k = 0; k < NCOMP; k++) I[u][k] = cur[u][k];
            load(q + ustep, cur);
        } else {
            load(q, I);
        }
        // the batch's pair-table entries, all loaded before the first scatter
        int bi[U], bj[U];
        int2 P1[U], P2[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            bi[u] = ci;
            bj[u] = cj;
            P1[u] = P2[u] = make_int2(0, 0);
            if (q + (long)u * step < hi) {
                P1[u] = pb[ci];
                P2[u] = pk[cj];
            }
            advance(ci, cj);
        }
        // kFull: every lane of the wavefront scatters (lanes past the range
        // with zero integrals), so that J_ab is summed per bra pair across it
#pragma unroll
        for (int u = 0; u < U; u++) {
            const bool ok = q + (long)u * step < hi;
            if (kFull || ok) {
                if (!ok) {
#pragma unroll
                    for (int k = 0; k < NCOMP; k++) I[u][k] = S(0);
                }
                A f = A(1);
                if (P1[u].x >> 16) f *= A(0.5);
                if (P2[u].x >> 16) f *= A(0.5);
                if (class_tri(C) && bi[u] == bj[u]) f *= A(0.5);
                jk_scatter<NA, NB, NC, ND, A, S, kFull>(I[u], P1[u].x & 0xffff, P1[u].y, P2[u].x & 0xffff, P2[u].y,
                                                        f, ok ? bi[u] : -1, ld, Ps, AJ, AK, ok);
            }
        }
    }
}

// Large molecules (partials in global memory): the work group walks its
// quartet range one bra pair at a time, the kets of a bra being consecutive
// quartets (coalesced integral reads).  Per bra the density rows of its two
// shells are staged in LDS (Prow), the K rows of those shells (K_ac, K_ad,
// K_bc, K_bd) accumulate in LDS (Krow) and J_ab in registers; both are added
// to the partials once per bra, so only J_cd reaches global memory per
// quartet.
template <int LA, int LB, int LC, int LD, typename S>
__device__ __forceinline__ void digest_class_rows(const JkArgs& g, const MolDesc& md, int chunk, int nchunk,
                                                  const double* __restrict__ Pg, double* AJ, double* AK,
                                                  double* Prow, double* Krow)
{
    constexpr int C = (LA + LB == 0) ? 0 : (LA + LB == 1 ? (LC + LD == 0 ? 1 : 2) : (LC + LD == 0 ? 3 : (LC + LD == 1 ? 4 : 5)));
    constexpr int NA = LA ? 3 : 1, NB = LB ? 3 : 1, NC = LC ? 3 : 1, ND = LD ? 3 : 1;
    constexpr int NCOMP = NA * NB * NC * ND;
    const int N = md.nbf;
    const long nq = md.nq[C];
    const long lo = nq * chunk / nchunk, hi = nq * (chunk + 1) / nchunk;
    if (lo >= hi) return;
    const S* __restrict__ eri = (const S*)g.eri[C];
    const long NQ = g.nq[C];
    const int2* __restrict__ pb = g.pao[class_bra(C)] + md.pair0[class_bra(C)];
    const int2* __restrict__ pk = g.pao[class_ket(C)] + md.pair0[class_ket(C)];
    const int nket = md.npair[class_ket(C)];
    int i, j0;
    decode_quartet_jk(C, lo, nket, i, j0);
    for (long q = lo; q < hi; i++, j0 = 0) {
        const int nk = class_tri(C) ? i + 1 : nket;
        const int seg = (int)min((long)(nk - j0), hi - q);
        const long qbase = md.q0[C] + q;      // batch-global index of ket j0
        q += seg;
        const int2 A1 = pb[i];
        const int oa = A1.x & 0xffff, ob = A1.y;
        const bool same = (A1.x >> 16) != 0;
        for (int t = threadIdx.x; t < (NA + NB) * N; t += blockDim.x) {
            const int r = t / N, col = t % N;
            Prow[t] = Pg[(r < NA ? oa + r : ob + r - NA) * N + col];
            Krow[t] = 0.0;
        }
        __syncthreads();
        double pab[NA][NB], jab[NA][NB];
#pragma unroll
        for (int a = 0; a < NA; a++)
#pragma unroll
            for (int b = 0; b < NB; b++) {
                pab[a][b] = Prow[a * N + ob + b];
                jab[a][b] = 0.0;
            }
        for (int t = threadIdx.x; t < seg; t += blockDim.x) {
            const int j = j0 + t;
            const int2 A2 = pk[j];
            double I[NCOMP];
#pragma unroll
            for (int k = 0; k < NCOMP; k++) I[k] = double(eri[(size_t)k * NQ + qbase + t]);
            double f = same ? 0.5 : 1.0;
            if (A2.x >> 16) f *= 0.5;
            if (class_tri(C) && i == j) f *= 0.5;
            jk_scatter_rows<NA, NB, NC, ND, double>(I, A2.x & 0xffff, A2.y, f, N, Prow, Prow + NA * N, Pg, pab, jab,
                                                    AJ, Krow, Krow + NA * N);
        }
#pragma unroll
        for (int a = 0; a < NA; a++)
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const double v = wave_sum(jab[a][b]);
                if ((threadIdx.x & 63) == 0 && v != 0.0) lds_add(&AJ[(oa + a) * N + ob + b], v);
            }
        __syncthreads();
        // a same-shell pair's b rows are its a rows
        for (int t = threadIdx.x; t < (same ? NA : NA + NB) * N; t += blockDim.x) {
            const int r = t / N, col = t % N;
            const double v = same ? Krow[t] + Krow[t + NA * N] : Krow[t];
            if (v != 0.0) lds_add(&AK[(r < NA ? oa + r : ob + r - NA) * N + col], v);
        }
        __syncthreads();
    }
}

// GLOBAL (molecules whose 3 N^2 accumulators exceed the LDS): the density
// is read from dP and the partials of this item are in global memory
// (A = double), digested bra by bra (digest_class_rows).  Molecules whose
// accumulators fit the LDS use jk_class_kernel below.
template <typename S, typename A, bool GLOBAL>
__global__ __launch_bounds__(kJkThreads) void jk_kernel(JkArgs g)
{
    static_assert(GLOBAL, "LDS-resident digestion runs in jk_class_kernel");
    static_assert(std::is_same<A, double>::value, "global partials are FP64");
    const JkItem it = g.items[blockIdx.x];
    if (g.only_active && g.state[it.mol].status != KS_MOL_ACTIVE) return;
    const MolDesc md = g.mol[it.mol];
    const int N = md.nbf, NN = N * N;
    extern __shared__ __align__(16) unsigned char smem_jk[];
    const double* Ps = g.dP + md.mat0;
    double* AJ = (double*)g.part + (size_t)blockIdx.x * 2 * g.part_stride;
    double* AK = AJ + g.part_stride;
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        AJ[i] = 0.0;
        AK[i] = 0.0;
    }
    __syncthreads();
    double* Prow = (double*)smem_jk;          // [6][N]
    double* Krow = Prow + 6 * N;              // [6][N]
    digest_class_rows<0, 0, 0, 0, S>(g, md, it.chunk, it.nchunk, Ps, AJ, AK, Prow, Krow);
    digest_class_rows<1, 0, 0, 0, S>(g, md, it.chunk, it.nchunk, Ps, AJ, AK, Prow, Krow);
    digest_class_rows<1, 0, 1, 0, S>(g, md, it.chunk, it.nchunk, Ps, AJ, AK, Prow, Krow);
    digest_class_rows<1, 1, 0, 0, S>(g, md, it.chunk, it.nchunk, Ps, AJ, AK, Prow, Krow);
    digest_class_rows<1, 1, 1, 0, S>(g, md, it.chunk, it.nchunk, Ps, AJ, AK, Prow, Krow);
    digest_class_rows<1, 1, 1, 1, S>(g, md, it.chunk, it.nchunk, Ps, AJ, AK, Prow, Krow);
}

// LDS-resident digestion of a subset of the quartet classes (bit c of CMASK
// set: class c), with NTH threads per group: each class group gets its own
// register allocation, so the classes of few components run with twice the
// wavefronts of the (pp|pp)-bearing group.  The first group of a build
// starts its partial J/K from zero, the later ones from the partial the
// earlier groups wrote for the same work item.
// LDS row stride of the N x N matrices: even, so that lanes whose ket pairs
// step along an anti-diagonal (c + 1, d - 1) address rows ld - 1 (odd)
// elements apart and fall in distinct banks (with ld = N odd, the stride N - 1
// is even and up to 32 lanes share a bank in the P_cd reads and J_cd atomics).
__host__ __device__ constexpr int jk_ld(int n) { return n + (n & 1); }

template <typename S, typename A, int CMASK, int NTH, bool FIRST>
__global__ __launch_bounds__(NTH) void jk_class_kernel(JkArgs g)
{
    const JkItem it = g.items[blockIdx.x];
    if (g.only_active && g.state[it.mol].status != KS_MOL_ACTIVE) return;
    const MolDesc md = g.mol[it.mol];
    const int N = md.nbf, NN = N * N, ld = jk_ld(N), NL = N * ld;
    extern __shared__ __align__(16) unsigned char smem_jk[];
    A* Pl = (A*)smem_jk;
    A* AJ = Pl + NL;
    A* AK = AJ + NL;
    const double* P = g.P + md.mat0;
    const double* Pr = g.Pref ? g.Pref + md.mat0 : nullptr;
    A* out = (A*)g.part + (size_t)blockIdx.x * 2 * g.part_stride;
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        const int l = (i / N) * ld + i % N;
        Pl[l] = A(Pr ? P[i] - Pr[i] : P[i]);
        AJ[l] = FIRST ? A(0) : out[i];
        AK[l] = FIRST ? A(0) : out[g.part_stride + i];
    }
    __syncthreads();
    if constexpr ((CMASK & 1) != 0) digest_class<0, 0, 0, 0, S, A>(g, md, it.chunk, it.nchunk, Pl, AJ, AK, ld);
    if constexpr ((CMASK & 2) != 0) digest_class<1, 0, 0, 0, S, A>(g, md, it.chunk, it.nchunk, Pl, AJ, AK, ld);
    if constexpr ((CMASK & 4) != 0) digest_class<1, 0, 1, 0, S, A>(g, md, it.chunk, it.nchunk, Pl, AJ, AK, ld);
    if constexpr ((CMASK & 8) != 0) digest_class<1, 1, 0, 0, S, A>(g, md, it.chunk, it.nchunk, Pl, AJ, AK, ld);
    if constexpr ((CMASK & 16) != 0) digest_class<1, 1, 1, 0, S, A>(g, md, it.chunk, it.nchunk, Pl, AJ, AK, ld);
    if constexpr ((CMASK & 32) != 0) digest_class<1, 1, 1, 1, S, A>(g, md, it.chunk, it.nchunk, Pl, AJ, AK, ld);
    __syncthreads();
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        const int l = (i / N) * ld + i % N;
        out[i] = AJ[l];
        out[g.part_stride + i] = AK[l];
    }
}

// Class groups: (ss|ss), (ps|ss), (ps|ps) need at most ~120 registers and
// run 16 wavefronts per group; the classes with a pp pair run 8.
constexpr int kJkLightMask = 1 | 2 | 4, kJkHeavyMask = 8 | 16 | 32;
constexpr int kJkLightThreads = 1024, kJkHeavyThreads = 512;

// dP = P - Pref (or P) for the global-mode digestion, active molecules only.
__global__ void delta_kernel(const MolDesc* __restrict__ mols, const MolState* __restrict__ state, int only_active,
                             const double* __restrict__ P, const double* __restrict__ Pref, double* __restrict__ dP)
{
    const int m = blockIdx.y;
    if (only_active && state[m].status != KS_MOL_ACTIVE) return;
    const MolDesc md = mols[m];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= md.nbf * md.nbf) return;
    dP[md.mat0 + t] = Pref ? P[md.mat0 + t] - Pref[md.mat0 + t] : P[md.mat0 + t];
}

// J = sum_chunks (AJ + AJ^T), K = sum_chunks (AK + AK^T), in FP64; added to
// J, K when accumulate is set (incremental build).  Pnext, when given, is
// copied to Pref: the density the accumulated J, K now correspond to.
template <typename A>
__global__ void jk_reduce_kernel(const MolDesc* __restrict__ mols, const MolState* __restrict__ state, int nchunk,
                                 const A* __restrict__ part, long stride, int only_active, int accumulate,
                                 const double* __restrict__ Pnext, double* __restrict__ Pref,
                                 double* __restrict__ J, double* __restrict__ K)
{
    const int m = blockIdx.y;
    if (only_active && state[m].status != KS_MOL_ACTIVE) return;
    const MolDesc md = mols[m];
    const int N = md.nbf;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int mu = t / N, nu = t % N;
    double sj = 0.0, sk = 0.0;
    for (int c = 0; c < nchunk; c++) {
        const A* pj = part + (size_t)(m * nchunk + c) * 2 * stride;
        const A* pk = pj + stride;
        sj += (double)pj[mu * N + nu] + (double)pj[nu * N + mu];
        sk += (double)pk[mu * N + nu] + (double)pk[nu * N + mu];
    }
    if (accumulate) {
        J[md.mat0 + t] += sj;
        K[md.mat0 + t] += sk;
    } else {
        J[md.mat0 + t] = sj;
        K[md.mat0 + t] = sk;
    }
    if (Pnext) Pref[md.mat0 + t] = Pnext[md.mat0 + t];
}

// LDS accumulation type: FP64 whenever 3 N^2 doubles (rows padded to an even
// stride) fit the 160 KB LDS.
// The digest is bound by its LDS atomics, and on gfx950 ds_add_f64 runs at
// twice the rate of ds_add_f32 here, so the mixed path stores its ERIs in
// FP32 (half the HBM stream) but accumulates J/K in FP64; molecules above 82
// functions fall back to FP32 accumulation.
// 0: LDS, FP64 accumulators; 1: LDS, FP32 (only the mixed path uses it);
// 2: global partial matrices, FP64.
int jk_mode(const ks_batch* b)
{
    int maxn = 0;
    for (auto& m : b->mol) maxn = std::max(maxn, m.nbf);
    const size_t nn3 = 3 * (size_t)maxn * jk_ld(maxn);
    if (nn3 * sizeof(double) <= 163840) return 0;
    if (b->opt.prec == KS_MIXED && nn3 * sizeof(float) <= 163840) return 1;
    return 2;
}

bool jk_acc_fp64(const ks_batch* b) { return jk_mode(b) != 1; }

size_t jk_lds_bytes(const ks_batch* b)
{
    const int mode = jk_mode(b);
    int maxn = 0;
    for (auto& m : b->mol) maxn = std::max(maxn, m.nbf);
    if (mode == 2) return 12 * (size_t)maxn * sizeof(double);   // density and K rows of one bra
    return 3 * (size_t)maxn * jk_ld(maxn) * (mode == 0 ? sizeof(double) : sizeof(float));
}

ks_status launch_delta(ks_batch* b, const double* P, const double* Pref, bool only_active)
{
    int maxnn = 0;
    for (auto& m : b->mol) maxnn = std::max(maxnn, m.nbf * m.nbf);
    hipLaunchKernelGGL(delta_kernel, dim3((maxnn + 255) / 256, b->n_mol), dim3(256), 0, b->stream, b->d_mol,
                       b->d_state, (int)only_active, P, Pref, b->d_work);
    KS_HIP(hipGetLastError());
    return KS_OK;
}

template <typename S, typename A, bool GLOBAL>
static ks_status run_jk(ks_batch* b, const double* P, double* J, double* K, bool only_active, bool incremental,
                        bool track)
{
    JkArgs g;
    g.mol = b->d_mol;
    g.state = b->d_state;
    g.items = b->d_jk_items;
    for (int c = 0; c < 3; c++) g.pao[c] = b->d_pair_ao[c];
    for (int c = 0; c < kNClass; c++) {
        g.eri[c] = b->d_eri[c];
        g.nq[c] = b->nq[c];
    }
    g.P = P;
    g.Pref = incremental ? b->d_Pprev : nullptr;
    g.dP = b->d_work;
    if (GLOBAL) {
        ks_status st = launch_delta(b, P, g.Pref, only_active);
        if (st) return st;
    }
    g.part = b->d_jk_part;
    g.part_stride = (long)b->max_np * b->max_np;
    g.only_active = only_active;
    const size_t lds = jk_lds_bytes(b);
    const dim3 grid((unsigned)b->jk_items.size());
    if constexpr (GLOBAL) {
        KS_HIP(hipFuncSetAttribute((const void*)jk_kernel<S, A, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
        KTimer tm(b, "jk");
        hipLaunchKernelGGL((jk_kernel<S, A, true>), grid, dim3(kJkThreads), lds, b->stream, g);
    } else {
        auto light = jk_class_kernel<S, A, kJkLightMask, kJkLightThreads, true>;
        auto heavy = jk_class_kernel<S, A, kJkHeavyMask, kJkHeavyThreads, false>;
        KS_HIP(hipFuncSetAttribute((const void*)light, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        KS_HIP(hipFuncSetAttribute((const void*)heavy, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        KTimer tm(b, "jk");
        hipLaunchKernelGGL(light, grid, dim3(kJkLightThreads), lds, b->stream, g);
        hipLaunchKernelGGL(heavy, grid, dim3(kJkHeavyThreads), lds, b->stream, g);
    }
    KS_HIP(hipGetLastError());
    return launch_jk_reduce(b, std::is_same<A, double>::value, P, J, K, only_active, incremental, track);
}

template <typename A>
static ks_status run_jk_reduce(ks_batch* b, const double* P, double* J, double* K, bool only_active,
                               bool incremental, bool track)
{
    KTimer tr(b, "jk_reduce");
    const int nchunk = b->jk_items.empty() ? 1 : b->jk_items[0].nchunk;
    int maxnn = 0;
    for (auto& m : b->mol) maxnn = std::max(maxnn, m.nbf * m.nbf);
    hipLaunchKernelGGL(jk_reduce_kernel<A>, dim3((maxnn + 255) / 256, b->n_mol), dim3(256), 0, b->stream, b->d_mol,
                       b->d_state, nchunk, (const A*)b->d_jk_part, (long)b->max_np * b->max_np, (int)only_active,
                       (int)incremental, track ? P : nullptr, b->d_Pprev, J, K);
    KS_HIP(hipGetLastError());
    return KS_OK;
}

ks_status launch_jk_reduce(ks_batch* b, bool acc_fp64, const double* P, double* J, double* K, bool only_active,
                           bool incremental, bool track)
{
    if (acc_fp64) return run_jk_reduce<double>(b, P, J, K, only_active, incremental, track);
    return run_jk_reduce<float>(b, P, J, K, only_active, incremental, track);
}

ks_status launch_jk(ks_batch* b, const double* P, double* J, double* K, bool only_active, bool incremental,
                    bool track)
{
    if (b->opt.direct) return launch_direct_jk(b, P, J, K, only_active, incremental, track);
    const int mode = jk_mode(b);
    if (b->opt.prec == KS_MIXED) {
        if (mode == 0) return run_jk<float, double, false>(b, P, J, K, only_active, incremental, track);
        if (mode == 1) return run_jk<float, float, false>(b, P, J, K, only_active, incremental, track);
        return run_jk<float, double, true>(b, P, J, K, only_active, incremental, track);
    }
    if (mode == 0) return run_jk<double, double, false>(b, P, J, K, only_active, incremental, track);
    return run_jk<double, double, true>(b, P, J, K, only_active, incremental, track);
}

}  // namespace ks
