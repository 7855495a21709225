// Scatter of one unique shell quartet's integrals into the J/K accumulators
// of a work group (LDS), shared by the stored-integral digestion and the
// integral-direct build.  For a unique shell quartet Q with stabiliser size s
// (f = 1/s), per component
//   AJ[ab] += 2 f I P_cd,  AJ[cd] += 2 f I P_ab,
//   AK[ac] += f I P_bd,  AK[bc] += f I P_ad,  AK[ad] += f I P_bc,  AK[bd] += f I P_ac,
// and J = AJ + AJ^T, K = AK + AK^T once the work groups are summed.
#pragma once

#include "ks_internal.h"
#include "wave.h"

namespace ks {

template <typename A>
__device__ __forceinline__ void lds_add(A* p, A v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// I: the quartet's NA NB NC ND components (a slowest); oa..od: first AO of
// each shell; bra_key: identifies the bra pair (lanes of a wavefront that
// all share it sum their J_ab contributions before a single LDS atomic).
// FULL: every lane of the wavefront calls (lanes without a quartet pass
// valid = false, zero integrals and in-range AO offsets); lanes that share a
// bra pair then sum their J_ab contributions over the wavefront whatever
// the number of bra pairs in it.  Otherwise (callers in divergent code)
// only a wavefront whose lanes all share one bra pair sums them, and the
// rest add per lane.  FP64 LDS atomics to one address from many lanes of
// an instruction serialise (about 0.3 lane-updates per cycle per CU
// against about 7 at distinct banks).
template <int NA, int NB, int NC, int ND, typename A, typename SI = A, bool FULL = false>
__device__ __forceinline__ void jk_scatter(const SI (&I)[NA * NB * NC * ND], int oa, int ob, int oc, int od, A f,
                                           int bra_key, int N, const A* __restrict__ Ps, A* AJ, A* AK,
                                           bool valid = true)
{
    const A f2 = A(2) * f;
    const unsigned long long act = __ballot(valid);
    const unsigned long long same = __ballot(valid && __builtin_amdgcn_readfirstlane(bra_key) == bra_key);
    const bool wave_bra = FULL ? same == ~0ull : (act == ~0ull && same == act);
    // density blocks and accumulators that involve no bra function a, kept
    // over the loop on a; the a-dependent ones are formed and flushed per a,
    // which bounds the live registers of the large classes
    A pcd[NC][ND], pbd[NB][ND], pbc[NB][NC];
#pragma unroll
    for (int c = 0; c < NC; c++)
#pragma unroll
        for (int d = 0; d < ND; d++) pcd[c][d] = Ps[(oc + c) * N + od + d];
#pragma unroll
    for (int b = 0; b < NB; b++) {
#pragma unroll
        for (int d = 0; d < ND; d++) pbd[b][d] = Ps[(ob + b) * N + od + d];
#pragma unroll
        for (int c = 0; c < NC; c++) pbc[b][c] = Ps[(ob + b) * N + oc + c];
    }
    A jcd[NC][ND] = {}, kbc[NB][NC] = {}, kbd[NB][ND] = {};
#pragma unroll
    for (int a = 0; a < NA; a++) {
        A pab[NB], pad[ND], pac[NC];
#pragma unroll
        for (int b = 0; b < NB; b++) pab[b] = Ps[(oa + a) * N + ob + b];
#pragma unroll
        for (int d = 0; d < ND; d++) pad[d] = Ps[(oa + a) * N + od + d];
#pragma unroll
        for (int c = 0; c < NC; c++) pac[c] = Ps[(oa + a) * N + oc + c];
        A jab[NB] = {}, kac[NC] = {}, kad[ND] = {};
#pragma unroll
        for (int b = 0; b < NB; b++)
#pragma unroll
            for (int c = 0; c < NC; c++)
#pragma unroll
                for (int d = 0; d < ND; d++) {
                    const A v = A(I[((a * NB + b) * NC + c) * ND + d]);
                    jab[b] += v * pcd[c][d];
                    jcd[c][d] += v * pab[b];
                    kac[c] += v * pbd[b][d];
                    kbc[b][c] += v * pad[d];
                    kad[d] += v * pbc[b][c];
                    kbd[b][d] += v * pac[c];
                }
        if (wave_bra) {
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const A v = wave_sum(f2 * jab[b]);
                if ((threadIdx.x & 63) == 0) lds_add(&AJ[(oa + a) * N + ob + b], v);
            }
        } else if (FULL) {
            // one wavefront sum per bra pair present (the lanes' bra pairs
            // are few and contiguous); the loop bound is wavefront-uniform
            unsigned long long rem = act;
            while (rem) {
                const int leader = __builtin_ctzll(rem);
                const int key = __builtin_amdgcn_readlane(bra_key, leader);
                const bool mine = valid && bra_key == key;
                rem &= ~__ballot(mine);
                const int ra = __builtin_amdgcn_readlane(oa, leader) + a, cb = __builtin_amdgcn_readlane(ob, leader);
#pragma unroll
                for (int b = 0; b < NB; b++) {
                    const A v = wave_sum(mine ? f2 * jab[b] : A(0));
                    if ((int)(threadIdx.x & 63) == leader) lds_add(&AJ[ra * N + cb + b], v);
                }
            }
        } else {
#pragma unroll
            for (int b = 0; b < NB; b++) lds_add(&AJ[(oa + a) * N + ob + b], f2 * jab[b]);
        }
        if (valid) {
#pragma unroll
            for (int c = 0; c < NC; c++) lds_add(&AK[(oa + a) * N + oc + c], f * kac[c]);
#pragma unroll
            for (int d = 0; d < ND; d++) lds_add(&AK[(oa + a) * N + od + d], f * kad[d]);
        }
    }
    if (valid) {
#pragma unroll
        for (int c = 0; c < NC; c++)
#pragma unroll
            for (int d = 0; d < ND; d++) lds_add(&AJ[(oc + c) * N + od + d], f2 * jcd[c][d]);
#pragma unroll
        for (int b = 0; b < NB; b++) {
#pragma unroll
            for (int c = 0; c < NC; c++) lds_add(&AK[(ob + b) * N + oc + c], f * kbc[b][c]);
#pragma unroll
            for (int d = 0; d < ND; d++) lds_add(&AK[(ob + b) * N + od + d], f * kbd[b][d]);
        }
    }
}

}  // namespace ks

namespace ks {

// Bra-major scatter for work groups whose J/K partials live in global
// memory: every lane holds a quartet of the same bra pair (ab).  Pa, Pb: LDS
// copies of the density rows of the bra's shells ([NA][N], [NB][N]); Pg: the
// density in global memory (for P_cd); pab: P_ab of the bra.  J_ab
// accumulates in the caller's registers (jab, with the factor 2 f), J_cd
// goes to the global partial AJ, and K_ac, K_ad (K_bc, K_bd) to the LDS rows
// Ka (Kb) of the bra's shells, which the caller adds to the partial K once
// per bra.  Same per-component terms as jk_scatter.
template <int NA, int NB, int NC, int ND, typename A>
__device__ __forceinline__ void jk_scatter_rows(const A (&I)[NA * NB * NC * ND], int oc, int od, A f, int N,
                                                const A* Pa, const A* Pb, const A* __restrict__ Pg,
                                                const A (&pab)[NA][NB], A (&jab)[NA][NB], A* AJ, A* Ka, A* Kb)
{
    A pcd[NC][ND], pbd[NB][ND], pbc[NB][NC], pad[NA][ND], pac[NA][NC];
#pragma unroll
    for (int c = 0; c < NC; c++)
#pragma unroll
        for (int d = 0; d < ND; d++) pcd[c][d] = Pg[(oc + c) * N + od + d];
#pragma unroll
    for (int b = 0; b < NB; b++) {
#pragma unroll
        for (int d = 0; d < ND; d++) pbd[b][d] = Pb[b * N + od + d];
#pragma unroll
        for (int c = 0; c < NC; c++) pbc[b][c] = Pb[b * N + oc + c];
    }
#pragma unroll
    for (int a = 0; a < NA; a++) {
#pragma unroll
        for (int d = 0; d < ND; d++) pad[a][d] = Pa[a * N + od + d];
#pragma unroll
        for (int c = 0; c < NC; c++) pac[a][c] = Pa[a * N + oc + c];
    }
    A jb[NA][NB] = {}, jcd[NC][ND] = {}, kac[NA][NC] = {}, kbc[NB][NC] = {}, kad[NA][ND] = {}, kbd[NB][ND] = {};
#pragma unroll
    for (int a = 0; a < NA; a++)
#pragma unroll
        for (int b = 0; b < NB; b++)
#pragma unroll
            for (int c = 0; c < NC; c++)
#pragma unroll
                for (int d = 0; d < ND; d++) {
                    const A v = I[((a * NB + b) * NC + c) * ND + d];
                    jb[a][b] += v * pcd[c][d];
                    jcd[c][d] += v * pab[a][b];
                    kac[a][c] += v * pbd[b][d];
                    kbc[b][c] += v * pad[a][d];
                    kad[a][d] += v * pbc[b][c];
                    kbd[b][d] += v * pac[a][c];
                }
    const A f2 = A(2) * f;
#pragma unroll
    for (int a = 0; a < NA; a++)
#pragma unroll
        for (int b = 0; b < NB; b++) jab[a][b] += f2 * jb[a][b];
#pragma unroll
    for (int c = 0; c < NC; c++)
#pragma unroll
        for (int d = 0; d < ND; d++) lds_add(&AJ[(oc + c) * N + od + d], f2 * jcd[c][d]);
#pragma unroll
    for (int a = 0; a < NA; a++) {
#pragma unroll
        for (int c = 0; c < NC; c++) lds_add(&Ka[a * N + oc + c], f * kac[a][c]);
#pragma unroll
        for (int d = 0; d < ND; d++) lds_add(&Ka[a * N + od + d], f * kad[a][d]);
    }
#pragma unroll
    for (int b = 0; b < NB; b++) {
#pragma unroll
        for (int c = 0; c < NC; c++) lds_add(&Kb[b * N + oc + c], f * kbc[b][c]);
#pragma unroll
        for (int d = 0; d < ND; d++) lds_add(&Kb[b * N + od + d], f * kbd[b][d]);
    }
}

}  // namespace ks
