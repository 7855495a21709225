// One- and two-electron integrals over contracted s/p Gaussians by the
// McMurchie-Davidson scheme (Hermite expansion of Gaussian products and the
// Hermite Coulomb integrals R_tuv), for gfx950.
//
// Paper section 3.2 ("Libcint"): the ERIs are computed once per molecule,
// each call independent, and stored with their 8-fold symmetry.  Here one
// lane computes one contracted unique shell quartet; the quartets of a class
// (ss|ss), (ps|ss), (ps|ps), (pp|ss), (pp|ps), (pp|pp) run in their own
// fully unrolled kernel so that every lane of a wavefront executes the same
// instruction stream (the SIMD answer to the paper's MIMD-per-thread port).
#include <cmath>

#include "kernels.h"
#include "jk_scatter.h"

namespace ks {

// ---------------------------------------------------------------------------
// Boys function
// ---------------------------------------------------------------------------
// Table F_m(T_i), T_i = i * DT, from the power series
// F_m(T) = exp(-T) sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1))   (all terms > 0).
void build_boys_table(std::vector<double>& tab)
{
    tab.assign((size_t)kBoysNT * kBoysM, 0.0);
    for (int i = 0; i < kBoysNT; i++) {
        long double T = (long double)i * kBoysDT;
        for (int m = 0; m < kBoysM; m++) {
            long double term = 1.0L / (2 * m + 1), sum = term;
            for (int k = 1; k < 2000; k++) {
                term *= 2.0L * T / (2 * m + 2 * k + 1);
                sum += term;
                if (term < 1e-22L * sum) break;
            }
            tab[(size_t)i * kBoysM + m] = (double)(expl(-T) * sum);
        }
    }
}

// The same series at the row-table nodes: rows[L][i][k] = F_{L+k}(i DTR).
static long double boys_series(int m, long double T)
{
    long double term = 1.0L / (2 * m + 1), sum = term;
    for (int k = 1; k < 2000; k++) {
        term *= 2.0L * T / (2 * m + 2 * k + 1);
        sum += term;
        if (term < 1e-22L * sum) break;
    }
    return expl(-T) * sum;
}

void build_boys_rows(std::vector<double>& rows)
{
    static_assert(kBoysLR - 1 + kBoysKR <= kBoysM, "row table orders");
    rows.assign((size_t)kBoysLR * kBoysNTR * kBoysKR, 0.0);
    for (int i = 0; i < kBoysNTR; i++) {
        const long double T = (long double)i * kBoysDTR;
        long double F[kBoysM];
        for (int m = 0; m < kBoysM; m++) F[m] = boys_series(m, T);
        for (int L = 0; L < kBoysLR; L++)
            for (int k = 0; k < kBoysKR; k++) rows[((size_t)L * kBoysNTR + i) * kBoysKR + k] = (double)F[L + k];
    }
}

// Reciprocal square root for x > 0: the hardware estimate refined by
// Newton-Raphson steps y <- y (3 - x y^2) / 2, each of which roughly doubles
// the number of correct bits (two for FP64; the FP32 estimate is ~1 ulp).
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}
__device__ __forceinline__ float rsqrt_nr(float x) { return __builtin_amdgcn_rsqf(x); }

template <typename R> struct BoysOrder;
template <> struct BoysOrder<double> { static constexpr int K = 7; };
template <> struct BoysOrder<float> { static constexpr int K = 4; };

// F_0..F_L at T: Taylor expansion about the nearest table node for the top
// order (dF_m/dT = -F_{m+1}), downward recursion F_m = (2T F_{m+1} + e^-T)/(2m+1);
// above the table, F_0 = sqrt(pi/T)/2 and upward recursion.
template <int L, typename R, int KT = 0>
__device__ __forceinline__ void boys(R T, R (&F)[L + 1], const R* __restrict__ tab)
{
    if (T < R(kBoysTMax)) {
        constexpr int K = KT > 0 ? KT : BoysOrder<R>::K;
        int i = (int)(T * R(1.0 / kBoysDT) + R(0.5));
        R dt = R(i) * R(kBoysDT) - T;
        const R* row = tab + (size_t)i * kBoysM + L;
        R s = row[K - 1];
#pragma unroll
        for (int k = K - 1; k >= 1; --k) s = row[k - 1] + dt * s * R(1.0 / k);
        F[L] = s;
        if (L > 0) {
            R e = exp(-T);
#pragma unroll
            for (int m = L - 1; m >= 0; --m) F[m] = (R(2) * T * F[m + 1] + e) * R(1.0 / (2 * m + 1));
        }
    } else {
        const R rt = rsqrt_nr(T);
        R e = exp(-T), inv = rt * rt;
        // sqrt(pi) / 2 / sqrt(T), the constant applied in FP64 (an FP32 copy
        // would bias every far-apart integral by its rounding)
        F[0] = R((0.5 * 1.7724538509055160273) * (double)rt);
#pragma unroll
        for (int m = 0; m < L; ++m) F[m + 1] = (R(2 * m + 1) * F[m] - e) * R(0.5) * inv;
    }
}

// Hermite Coulomb integrals R_tuv for t+u+v <= L:
// R^(n)_000 = (-2 alpha)^n F_n(T),
// R^(n)_{t+1,u,v} = t R^(n+1)_{t-1,u,v} + X R^(n+1)_{t,u,v}  (same for u with Y, v with Z).
// F_0..F_L at T from the row table of this L (rows: F_L..F_{L+7} at
// T_i = i DTR, typically in LDS): eight Taylor terms about the nearest node
// (|T - T_i| <= DTR/2, truncation below 0.05^8/8! ~ 1e-15 relative), then the
// same downward recursion; above the table as in boys().
template <int L>
__device__ __forceinline__ void boys_rows(double T, double (&F)[L + 1], const double* rows)
{
    if (T < kBoysTMax) {
        const int i = (int)(T * (1.0 / kBoysDTR) + 0.5);
        const double dt = (double)i * kBoysDTR - T;
        const double2* row = (const double2*)(rows + (size_t)i * kBoysKR);
        const double2 r01 = row[0], r23 = row[1], r45 = row[2], r67 = row[3];
        double s = r67.y;
        s = r67.x + dt * s * (1.0 / 7);
        s = r45.y + dt * s * (1.0 / 6);
        s = r45.x + dt * s * (1.0 / 5);
        s = r23.y + dt * s * (1.0 / 4);
        s = r23.x + dt * s * (1.0 / 3);
        s = r01.y + dt * s * (1.0 / 2);
        s = r01.x + dt * s;
        F[L] = s;
        if (L > 0) {
            const double e = exp(-T);
#pragma unroll
            for (int m = L - 1; m >= 0; --m) F[m] = (2.0 * T * F[m + 1] + e) * (1.0 / (2 * m + 1));
        }
    } else {
        const double rt = rsqrt_nr(T);
        const double e = exp(-T), inv = rt * rt;
        F[0] = (0.5 * 1.7724538509055160273) * rt;
#pragma unroll
        for (int m = 0; m < L; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) * 0.5 * inv;
    }
}

template <int L, typename R>
__device__ __forceinline__ void hermite_R(R m2a, R X, R Y, R Z, const R (&F)[L + 1], R (&out)[L + 1][L + 1][L + 1])
{
    R pw[L + 1];
    pw[0] = R(1);
#pragma unroll
    for (int n = 1; n <= L; n++) pw[n] = pw[n - 1] * m2a;
    R cur[L + 1][L + 1][L + 1];
    cur[0][0][0] = pw[L] * F[L];
#pragma unroll
    for (int n = L - 1; n >= 0; --n) {
        R nxt[L + 1][L + 1][L + 1];
#pragma unroll
        for (int t = 0; t <= L; t++)
#pragma unroll
            for (int u = 0; u <= L; u++)
#pragma unroll
                for (int v = 0; v <= L; v++) {
                    if (t + u + v > L - n) continue;
                    R val;
                    if (t + u + v == 0) val = pw[n] * F[n];
                    else if (t > 0) val = (t > 1 ? R(t - 1) * cur[t > 1 ? t - 2 : 0][u][v] : R(0)) + X * cur[t - 1][u][v];
                    else if (u > 0) val = (u > 1 ? R(u - 1) * cur[t][u > 1 ? u - 2 : 0][v] : R(0)) + Y * cur[t][u - 1][v];
                    else val = (v > 1 ? R(v - 1) * cur[t][u][v > 1 ? v - 2 : 0] : R(0)) + Z * cur[t][u][v - 1];
                    nxt[t][u][v] = val;
                }
#pragma unroll
        for (int t = 0; t <= L; t++)
#pragma unroll
            for (int u = 0; u <= L; u++)
#pragma unroll
                for (int v = 0; v <= L; v++)
                    if (t + u + v <= L - n) cur[t][u][v] = nxt[t][u][v];
    }
#pragma unroll
    for (int t = 0; t <= L; t++)
#pragma unroll
        for (int u = 0; u <= L; u++)
#pragma unroll
            for (int v = 0; v <= L; v++)
                if (t + u + v <= L) out[t][u][v] = cur[t][u][v];
}

// Hermite expansion coefficients of a 1D product x_A^i x_B^j (i, j <= 1):
// e[combo][t], combo = i + 2 j:  E^00 = 1; E^10 = (XPA, 1/2p); E^01 = (XPB, 1/2p);
// E^11 = (XPA XPB + 1/2p, (XPA + XPB)/2p, 1/4p^2).
template <typename R>
__device__ __forceinline__ void hermite_E(R XPA, R XPB, R i2p, R (&e)[4][3])
{
    e[0][0] = R(1); e[0][1] = R(0); e[0][2] = R(0);
    e[1][0] = XPA; e[1][1] = i2p; e[1][2] = R(0);
    e[2][0] = XPB; e[2][1] = i2p; e[2][2] = R(0);
    e[3][0] = XPA * XPB + i2p; e[3][1] = (XPA + XPB) * i2p; e[3][2] = i2p * i2p;
}

// Cartesian exponent of component c (0..2 for p, s has 0) along direction d.
__host__ __device__ constexpr int lexp(int L, int c, int d) { return (L == 1 && c == d) ? 1 : 0; }

// Read-only view of one pair in a field-major primitive-pair table with PP
// primitive pairs per shell pair (9 for STO-3G; 36 for 6-31G, padded with
// zero-weight pairs where a shell has fewer than six primitives).
template <int PP = kNPrimPair>
struct PairView {
    const double* t;
    long n;
    int i;
    __device__ __forceinline__ double get(int f, int k) const { return t[((size_t)f * PP + k) * n + i]; }
};

// ---------------------------------------------------------------------------
// contracted shell quartet (ab|cd), McMurchie-Davidson:
// (ab|cd) = 2 pi^(5/2) / (p q sqrt(p+q)) K_ab K_cd
//           sum_tuv E^ab_tuv sum_tau,nu,phi (-1)^(tau+nu+phi) E^cd_tau,nu,phi R_{t+tau,u+nu,v+phi}
// ---------------------------------------------------------------------------
// ROWS: tab is the Boys row table of L = LA + LB + LC + LD (boys_rows), else
// the full table (boys) with BK Taylor terms (0: the type's default).
// Acc: the accumulator type of the contracted integrals (FP64 for FP32
// evaluation of the classes of few components, where it costs little).  The
// prefactor 2 pi^(5/2) K_ab / p and K_cd / q are formed in FP64 per primitive
// pair and rounded once each: an FP32 2 pi^(5/2) would scale every integral
// by the same relative error (3e-8), a bias of ~1e-5 Ha in the energy.
template <int LA, int LB, int LC, int LD, typename R, bool ROWS = false, int PP = kNPrimPair, int BK = 0,
          typename Acc = R, int UNR = 3>
__device__ __forceinline__ void eri_quartet(const Shell& sa, const Shell& sb, const Shell& sc, const Shell& sd,
                                            const PairView<PP>& vb, const PairView<PP>& vk, const R* __restrict__ tab,
                                            R cut, Acc* acc)
{
    constexpr int NA = LA ? 3 : 1, NB = LB ? 3 : 1, NC = LC ? 3 : 1, ND = LD ? 3 : 1;
    constexpr int L = LA + LB + LC + LD, LAB = LA + LB;
    constexpr double pi25 = 2.0 * 17.493418327624862;   // 2 pi^(5/2)
    // FP32 evaluation with an ss ket (the (ss|ss), (ps|ss), (pp|ss) classes):
    // the nine ket primitive pairs' centres, exponents and scaled weights are
    // read once into registers instead of once per bra primitive pair
    constexpr bool kKetReg = (LC + LD == 0) && PP == kNPrimPair;
    double kPr[kKetReg ? PP : 1][3];
    R kqr[kKetReg ? PP : 1], kKr[kKetReg ? PP : 1];
    if constexpr (kKetReg) {
#pragma unroll
        for (int jp = 0; jp < PP; jp++) {
#pragma unroll
            for (int d = 0; d < 3; d++) kPr[jp][d] = vk.get(1 + d, jp);
            kqr[jp] = R(vk.get(0, jp));
            kKr[jp] = R(vk.get(4, jp) * vk.get(5, jp));
        }
    }
#pragma unroll
    for (int i = 0; i < NA * NB * NC * ND; i++) acc[i] = Acc(0);
    auto bra = [&](int ip) {
        const double bP[3] = {vb.get(1, ip), vb.get(2, ip), vb.get(3, ip)};
        const double ipd = vb.get(5, ip);
        const R p = R(vb.get(0, ip)), Kbp = R(pi25 * vb.get(4, ip) * ipd), ipv = R(ipd);
        // negligible for every ket: q >= kQMin and |K_cd| <= kKMax bound the prefactor
        if (fabs(Kbp) * R(kKMax / kQMin) * rsqrt_nr(p + R(kQMin)) < cut) return;
        R eb[3][4][3];
        const R i2p = R(0.5) * ipv;
#pragma unroll
        for (int d = 0; d < 3; d++) hermite_E<R>(R(bP[d] - sa.A[d]), R(bP[d] - sb.A[d]), i2p, eb[d]);
        auto ket = [&](int jp) {
            double kP[3];
            R q, Kkq, iqv;
            if constexpr (kKetReg) {
                kP[0] = kPr[jp][0]; kP[1] = kPr[jp][1]; kP[2] = kPr[jp][2];
                q = kqr[jp];
                Kkq = kKr[jp];
                iqv = R(1);                                // unused: an ss ket's Hermite expansion is 1
            } else {
                kP[0] = vk.get(1, jp); kP[1] = vk.get(2, jp); kP[2] = vk.get(3, jp);
                const double iqd = vk.get(5, jp);
                q = R(vk.get(0, jp));
                Kkq = R(vk.get(4, jp) * iqd);
                iqv = R(iqd);
            }
            const R rs = rsqrt_nr(p + q);                 // 1/sqrt(p + q)
            const R pref = Kbp * Kkq * rs;
            if (fabs(pref) < cut) return;
            R ek[3][4][3];
            const R i2q = R(0.5) * iqv;
#pragma unroll
            for (int d = 0; d < 3; d++) hermite_E<R>(R(kP[d] - sc.A[d]), R(kP[d] - sd.A[d]), i2q, ek[d]);
            const R PQx = R(bP[0] - kP[0]), PQy = R(bP[1] - kP[1]), PQz = R(bP[2] - kP[2]);
            const R alpha = p * q * (rs * rs);            // p q / (p + q)
            const R T = alpha * (PQx * PQx + PQy * PQy + PQz * PQz);
            R F[L + 1];
            if constexpr (ROWS) boys_rows<L>(T, F, tab);
            else boys<L, R, BK>(T, F, tab);
            R Rt[L + 1][L + 1][L + 1];
            hermite_R<L, R>(R(-2) * alpha, PQx, PQy, PQz, F, Rt);
#pragma unroll
            for (int kc = 0; kc < NC; kc++)
#pragma unroll
                for (int ld = 0; ld < ND; ld++) {
                    const int cx = lexp(LC, kc, 0) + 2 * lexp(LD, ld, 0);
                    const int cy = lexp(LC, kc, 1) + 2 * lexp(LD, ld, 1);
                    const int cz = lexp(LC, kc, 2) + 2 * lexp(LD, ld, 2);
                    const int tx = lexp(LC, kc, 0) + lexp(LD, ld, 0);
                    const int ty = lexp(LC, kc, 1) + lexp(LD, ld, 1);
                    const int tz = lexp(LC, kc, 2) + lexp(LD, ld, 2);
                    // H_tuv = sum (-1)^(tau+nu+phi) E^cd R_{t+tau,...} for t+u+v <= LAB
                    R H[LAB + 1][LAB + 1][LAB + 1];
#pragma unroll
                    for (int t = 0; t <= LAB; t++)
#pragma unroll
                        for (int u = 0; u <= LAB; u++)
#pragma unroll
                            for (int v = 0; v <= LAB; v++) {
                                if (t + u + v > LAB) continue;
                                R h = R(0);
#pragma unroll
                                for (int ta = 0; ta <= 2; ta++)
#pragma unroll
                                    for (int nu = 0; nu <= 2; nu++)
#pragma unroll
                                        for (int ph = 0; ph <= 2; ph++) {
                                            if (ta > tx || nu > ty || ph > tz) continue;
                                            if (t + ta > L || u + nu > L || v + ph > L) continue;
                                            if (t + ta + u + nu + v + ph > L) continue;
                                            const R ee = ek[0][cx][ta] * ek[1][cy][nu] * ek[2][cz][ph];
                                            const R rr = Rt[t + ta][u + nu][v + ph];
                                            if ((ta + nu + ph) & 1) h -= ee * rr;
                                            else h += ee * rr;
                                        }
                                H[t][u][v] = h;
                            }
#pragma unroll
                    for (int ia = 0; ia < NA; ia++)
#pragma unroll
                        for (int jb = 0; jb < NB; jb++) {
                            const int bx = lexp(LA, ia, 0) + 2 * lexp(LB, jb, 0);
                            const int by = lexp(LA, ia, 1) + 2 * lexp(LB, jb, 1);
                            const int bz = lexp(LA, ia, 2) + 2 * lexp(LB, jb, 2);
                            const int sx = lexp(LA, ia, 0) + lexp(LB, jb, 0);
                            const int sy = lexp(LA, ia, 1) + lexp(LB, jb, 1);
                            const int sz = lexp(LA, ia, 2) + lexp(LB, jb, 2);
                            R val = R(0);
#pragma unroll
                            for (int t = 0; t <= 2; t++)
#pragma unroll
                                for (int u = 0; u <= 2; u++)
#pragma unroll
                                    for (int v = 0; v <= 2; v++) {
                                        if (t > sx || u > sy || v > sz || t + u + v > LAB) continue;
                                        val += eb[0][bx][t] * eb[1][by][u] * eb[2][bz][v] * H[t][u][v];
                                    }
                            acc[((ia * NB + jb) * NC + kc) * ND + ld] += Acc(pref * val);
                        }
                }
        };
        // STO-3G: nine ket primitive pairs in groups of UNR, each group
        // unrolled (by default three: fully unrolled FP64 kernels keep all
        // nine pairs' data in registers and drop to two or three waves per
        // SIMD, 467 -> 385 ms for the ERIs of 2048 molecules; the autotuner
        // picks per class); 6-31G: the real pairs in a plain loop
        if constexpr (kKetReg) {
#pragma unroll
            for (int jp = 0; jp < PP; jp++) ket(jp);
        } else if constexpr (PP <= kNPrimPair) {
            static_assert(PP % UNR == 0, "ket groups");
#pragma unroll 1
            for (int j0 = 0; j0 < PP; j0 += UNR) {
#pragma unroll
                for (int u = 0; u < UNR; u++) ket(j0 + u);
            }
        } else {
            const int nk = sc.np * sd.np;       // the ket's real primitive pairs
#pragma unroll 1
            for (int jp = 0; jp < nk; jp++) ket(jp);
        }
    };
    if constexpr (PP <= kNPrimPair) {
        for (int ip = 0; ip < PP; ip++) bra(ip);
    } else {
        const int nb = sa.np * sb.np;
#pragma unroll 1
        for (int ip = 0; ip < nb; ip++) bra(ip);
    }
}

// ---------------------------------------------------------------------------
// quartet decoding shared by the ERI, J/K and unpack kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_mol(const long* __restrict__ off, int n, long q)
{
    int lo = 0, hi = n;  // off[lo] <= q < off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= q) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void decode_quartet(int c, long q, int nket, int& i, int& j)
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

struct EriArgs {
    const MolDesc* mol;
    const long* qoff;       // [n_mol + 1]
    int n_mol;
    long nq;                // quartets of this class in the batch
    const Shell* shells;
    const Pair* pb;         // bra pair class list
    const Pair* pk;
    const double* ppb;      // primitive-pair tables [5][9][npair] of the bra / ket class
    const double* ppk;
    long npb, npk;
    const void* tab;
    const double* rows;     // Boys row tables [kBoysLR][kBoysNTR][kBoysKR]
    void* out;              // [ncomp][nq]
    double cut;             // primitive quartets with |prefactor| below this are skipped
    const double* Qb;       // Schwarz factors of the bra / ket pair class (when schwarz > 0)
    const double* Qk;
    double schwarz;         // quartets with Q_ab Q_cd below this are stored as 0 (0 = off)
};

// One thread per contracted quartet; the Boys interpolation reads the full
// table from global memory (L1/L2).  (A copy of the row table in LDS per
// group made the class kernels 15% faster alone, but beside the grid kernel
// on the other stream the two compete for LDS and the pair finished no
// earlier.)
// Work-group size per class: the options' (64, 128 or 256; autotuned), else 128.
constexpr int kEriThreads = 128, kEriThreadsMax = 256;

template <int LA, int LB, int LC, int LD, typename R, typename S, int PP, int UNR = 3>
__global__ __launch_bounds__(kEriThreadsMax) void eri_class_kernel(EriArgs g)
{
    constexpr int C = (LA + LB == 0) ? 0 : (LA + LB == 1 ? (LC + LD == 0 ? 1 : 2) : (LC + LD == 0 ? 3 : (LC + LD == 1 ? 4 : 5)));
    constexpr int NCOMP = class_ncomp(C);
    const long qg = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (qg >= g.nq) return;
    S* out = (S*)g.out;
    const int m = find_mol(g.qoff, g.n_mol, qg);
    const MolDesc& md = g.mol[m];
    const long q = qg - g.qoff[m];
    int i, j;
    decode_quartet(C, q, md.npair[class_ket(C)], i, j);
    const int ib = md.pair0[class_bra(C)] + i, ik = md.pair0[class_ket(C)] + j;
    if (g.schwarz > 0.0 && g.Qb[ib] * g.Qk[ik] < g.schwarz) {
#pragma unroll
        for (int k = 0; k < NCOMP; k++) out[(size_t)k * g.nq + qg] = S(0);
        return;
    }
    const Pair P1 = g.pb[ib], P2 = g.pk[ik];
    const Shell sa = g.shells[P1.sa], sb = g.shells[P1.sb], sc = g.shells[P2.sa], sd = g.shells[P2.sb];
    typedef typename std::conditional<(sizeof(R) == 4 && NCOMP <= 9), double, R>::type Acc;
    Acc acc[NCOMP];
    const PairView<PP> vb{g.ppb, g.npb, ib}, vk{g.ppk, g.npk, ik};
    // integrals stored in FP32: five Taylor terms of the Boys function
    // (truncation below 0.025^5/5! ~ 1e-10 relative, far under the FP32
    // rounding of the stored value) instead of seven
    eri_quartet<LA, LB, LC, LD, R, false, PP, sizeof(S) == 4 ? 5 : 0, Acc, UNR>(sa, sb, sc, sd, vb, vk,
                                                                                 (const R*)g.tab, R(g.cut), acc);
#pragma unroll
    for (int k = 0; k < NCOMP; k++) out[(size_t)k * g.nq + qg] = (S)acc[k];
}

// Primitive-pair tables of every shell pair of one pair class, stored
// field-major [f][k][pair] (f = p, Px, Py, Pz, K; k = primitive pair) so that
// lanes working on consecutive pairs load consecutive addresses.
// pp primitive pairs per shell pair: entry k = ka nb + kb for the na x nb
// primitive pairs of the two shells (pp = 9: always 3 x 3); with pp = 36
// (6-31G) the entries from na nb on are padding (K = 0, p = 1, P = A), which
// the integral loops do not visit.
__global__ void pair_kernel(const Shell* __restrict__ shells, const Pair* __restrict__ pairs, long npair, int pp,
                            double* __restrict__ out)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npair * pp) return;
    const long ip = t / pp;
    const int k = (int)(t % pp);
    const Pair pr = pairs[ip];
    const Shell& A = shells[pr.sa];
    const Shell& B = shells[pr.sb];
    const int ka = k / B.np, kb = k % B.np;
    if (k >= A.np * B.np) {
        for (int d = 0; d < 3; d++) out[((size_t)(1 + d) * pp + k) * npair + ip] = A.A[d];
        out[(size_t)k * npair + ip] = 1.0;
        out[((size_t)4 * pp + k) * npair + ip] = 0.0;
        out[((size_t)5 * pp + k) * npair + ip] = 1.0;
        return;
    }
    const double a = A.a[ka], b = B.a[kb], p = a + b;
    double r2 = 0.0;
    for (int d = 0; d < 3; d++) {
        out[((size_t)(1 + d) * pp + k) * npair + ip] = (a * A.A[d] + b * B.A[d]) / p;
        r2 += (A.A[d] - B.A[d]) * (A.A[d] - B.A[d]);
    }
    out[(size_t)k * npair + ip] = p;
    out[((size_t)4 * pp + k) * npair + ip] = A.c[ka] * B.c[kb] * exp(-a * b / p * r2);
    out[((size_t)5 * pp + k) * npair + ip] = 1.0 / p;
}

// ---------------------------------------------------------------------------
// one-electron integrals (McMurchie-Davidson): one thread per AO pair
// ---------------------------------------------------------------------------
// 1D Hermite coefficients E^{ij}_t for i <= 1, j <= 3 by
// E^{i,j+1}_t = E^{ij}_{t-1}/2p + XPB E^{ij}_t + (t+1) E^{ij}_{t+1} (same in i with XPA).
__device__ inline void hermite_E_1e(double XPA, double XPB, double i2p, double (&E)[2][4][5])
{
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 4; j++)
            for (int t = 0; t < 5; t++) E[i][j][t] = 0.0;
    E[0][0][0] = 1.0;
    for (int j = 0; j < 3; j++)
        for (int t = 0; t <= j + 1; t++)
            E[0][j + 1][t] = (t > 0 ? i2p * E[0][j][t - 1] : 0.0) + XPB * E[0][j][t] + (t + 1 < 5 ? (t + 1) * E[0][j][t + 1] : 0.0);
    for (int j = 0; j < 4; j++)
        for (int t = 0; t <= j + 1 && t < 5; t++)
            E[1][j][t] = (t > 0 ? i2p * E[0][j][t - 1] : 0.0) + XPA * E[0][j][t] + (t + 1 < 5 ? (t + 1) * E[0][j][t + 1] : 0.0);
}

__global__ void int1e_kernel(const MolDesc* __restrict__ mols, const Shell* __restrict__ shells,
                             const int2* __restrict__ aoinfo, const double* __restrict__ Rat,
                             const double* __restrict__ Zat, const double* __restrict__ tab,
                             double* __restrict__ S, double* __restrict__ T, double* __restrict__ V,
                             double* __restrict__ H)
{
    const int m = blockIdx.y;
    const MolDesc md = mols[m];
    const int N = md.nbf;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * (N + 1) / 2) return;
    int mu = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (mu * (mu + 1) / 2 > t) mu--;
    while ((mu + 1) * (mu + 2) / 2 <= t) mu++;
    const int nu = t - mu * (mu + 1) / 2;
    const int2 ia = aoinfo[md.ao0 + mu], ib = aoinfo[md.ao0 + nu];
    const Shell& A = shells[ia.x];
    const Shell& B = shells[ib.x];
    int la[3], lb[3];
    for (int d = 0; d < 3; d++) {
        la[d] = lexp(A.L, ia.y, d);
        lb[d] = lexp(B.L, ib.y, d);
    }
    double s = 0.0, kin = 0.0, v = 0.0;
    for (int ka = 0; ka < A.np; ka++)
        for (int kb = 0; kb < B.np; kb++) {
            const double a = A.a[ka], b = B.a[kb], p = a + b, i2p = 0.5 / p;
            double P[3], r2 = 0.0, E[3][2][4][5];
            for (int d = 0; d < 3; d++) {
                P[d] = (a * A.A[d] + b * B.A[d]) / p;
                r2 += (A.A[d] - B.A[d]) * (A.A[d] - B.A[d]);
                hermite_E_1e(P[d] - A.A[d], P[d] - B.A[d], i2p, E[d]);
            }
            const double K = A.c[ka] * B.c[kb] * exp(-a * b / p * r2);
            const double sp = sqrt(kPi / p);
            double Sd[3], Td[3];
            for (int d = 0; d < 3; d++) {
                const int i = la[d], j = lb[d];
                Sd[d] = E[d][i][j][0] * sp;
                // -1/2 d^2/dx^2 acting on x_B^j exp(-b x_B^2)
                double t2 = 4.0 * b * b * E[d][i][j + 2][0] * sp - 2.0 * b * (2 * j + 1) * Sd[d];
                if (j >= 2) t2 += j * (j - 1) * E[d][i][j - 2][0] * sp;
                Td[d] = -0.5 * t2;
            }
            s += K * Sd[0] * Sd[1] * Sd[2];
            kin += K * (Td[0] * Sd[1] * Sd[2] + Sd[0] * Td[1] * Sd[2] + Sd[0] * Sd[1] * Td[2]);
            for (int c = 0; c < md.natom; c++) {
                const double* Rc = Rat + 3 * (md.atom0 + c);
                const double X = P[0] - Rc[0], Y = P[1] - Rc[1], Z = P[2] - Rc[2];
                double F[3], Rt[3][3][3];
                boys<2, double>(p * (X * X + Y * Y + Z * Z), F, tab);
                hermite_R<2, double>(-2.0 * p, X, Y, Z, F, Rt);
                double sum = 0.0;
                for (int tt = 0; tt <= la[0] + lb[0]; tt++)
                    for (int u = 0; u <= la[1] + lb[1]; u++)
                        for (int w = 0; w <= la[2] + lb[2]; w++)
                            sum += E[0][la[0]][lb[0]][tt] * E[1][la[1]][lb[1]][u] * E[2][la[2]][lb[2]][w] * Rt[tt][u][w];
                v -= Zat[md.atom0 + c] * 2.0 * kPi / p * K * sum;
            }
        }
    const long o = md.mat0;
    S[o + mu * N + nu] = S[o + nu * N + mu] = s;
    T[o + mu * N + nu] = T[o + nu * N + mu] = kin;
    V[o + mu * N + nu] = V[o + nu * N + mu] = v;
    H[o + mu * N + nu] = H[o + nu * N + mu] = kin + v;
}

// ---------------------------------------------------------------------------
// packed unique-ERI copy-out of one molecule (canonical index of each component)
// ---------------------------------------------------------------------------
__device__ __forceinline__ long pidx(int i, int j) { return i >= j ? (long)i * (i + 1) / 2 + j : (long)j * (j + 1) / 2 + i; }

template <typename S>
__global__ void eri_unpack_kernel(const MolDesc* __restrict__ mols, int m, int c, long nqc,
                                  const Shell* __restrict__ shells, const Pair* __restrict__ pb,
                                  const Pair* __restrict__ pk, const S* __restrict__ eri, double* __restrict__ out)
{
    const MolDesc md = mols[m];
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= md.nq[c]) return;
    int i, j;
    decode_quartet(c, q, md.npair[class_ket(c)], i, j);
    const Pair P1 = pb[md.pair0[class_bra(c)] + i], P2 = pk[md.pair0[class_ket(c)] + j];
    const Shell &A = shells[P1.sa], &B = shells[P1.sb], &Cc = shells[P2.sa], &D = shells[P2.sb];
    const int na = A.L ? 3 : 1, nb = B.L ? 3 : 1, nc = Cc.L ? 3 : 1, nd = D.L ? 3 : 1;
    const long qg = md.q0[c] + q;
    int k = 0;
    for (int ia = 0; ia < na; ia++)
        for (int jb = 0; jb < nb; jb++)
            for (int kc = 0; kc < nc; kc++)
                for (int ld = 0; ld < nd; ld++, k++) {
                    const long ij = pidx(A.ao + ia, B.ao + jb), kl = pidx(Cc.ao + kc, D.ao + ld);
                    out[ij >= kl ? ij * (ij + 1) / 2 + kl : kl * (kl + 1) / 2 + ij] = (double)eri[(size_t)k * nqc + qg];
                }
}

// The same copy-out restricted to the packed indices lo .. hi-1, written to
// out[index - lo]: a window of the packed list in a caller-sized buffer.
// Every index of the window is written (each packed index is the image of at
// least one component of one unique quartet).
template <typename S>
__global__ void eri_unpack_window_kernel(const MolDesc* __restrict__ mols, int m, int c, long nqc,
                                         const Shell* __restrict__ shells, const Pair* __restrict__ pb,
                                         const Pair* __restrict__ pk, const S* __restrict__ eri, long lo, long hi,
                                         double* __restrict__ out)
{
    const MolDesc md = mols[m];
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= md.nq[c]) return;
    int i, j;
    decode_quartet(c, q, md.npair[class_ket(c)], i, j);
    const Pair P1 = pb[md.pair0[class_bra(c)] + i], P2 = pk[md.pair0[class_ket(c)] + j];
    const Shell &A = shells[P1.sa], &B = shells[P1.sb], &Cc = shells[P2.sa], &D = shells[P2.sb];
    const int na = A.L ? 3 : 1, nb = B.L ? 3 : 1, nc = Cc.L ? 3 : 1, nd = D.L ? 3 : 1;
    const long qg = md.q0[c] + q;
    int k = 0;
    for (int ia = 0; ia < na; ia++)
        for (int jb = 0; jb < nb; jb++)
            for (int kc = 0; kc < nc; kc++)
                for (int ld = 0; ld < nd; ld++, k++) {
                    const long ij = pidx(A.ao + ia, B.ao + jb), kl = pidx(Cc.ao + kc, D.ao + ld);
                    const long x = ij >= kl ? ij * (ij + 1) / 2 + kl : kl * (kl + 1) / 2 + ij;
                    if (x >= lo && x < hi) out[x - lo] = (double)eri[(size_t)k * nqc + qg];
                }
}

// ---------------------------------------------------------------------------
// Schwarz factors: Q_ab = max over the components (a_i b_j) of
// sqrt|(a_i b_j | a_i b_j)|, so |(ab|cd)| <= Q_ab Q_cd for every component.
// One thread per shell pair of the class; L: angular momenta of the pair.
// ---------------------------------------------------------------------------
template <int LA, int LB, int PP>
__global__ void schwarz_kernel(const Shell* __restrict__ shells, const Pair* __restrict__ pairs,
                               const double* __restrict__ pp, long npair, const double* __restrict__ tab,
                               double* __restrict__ Q)
{
    constexpr int NA = LA ? 3 : 1, NB = LB ? 3 : 1, NAB = NA * NB;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npair) return;
    const Pair pr = pairs[i];
    const Shell sa = shells[pr.sa], sb = shells[pr.sb];
    const PairView<PP> v{pp, npair, (int)i};
    double I[NAB * NAB];
    eri_quartet<LA, LB, LA, LB, double, false, PP>(sa, sb, sa, sb, v, v, tab, 0.0, I);
    double m = 0.0;
#pragma unroll
    for (int u = 0; u < NAB; u++) m = fmax(m, fabs(I[u * NAB + u]));
    Q[i] = sqrt(m);
}

// ---------------------------------------------------------------------------
// Integral-direct J/K (the paper's recomputation remedy for the memory of
// stored integrals, section 5): one work group per (molecule, chunk of its
// quartets), the density (or its change since the last build) and the J/K
// accumulators in LDS.  A quartet is skipped when Q_ab Q_cd max|P| < tol;
// the others are evaluated in FP64 (McMurchie-Davidson, as eri_class_kernel)
// and scattered with jk_scatter.  Partials go to the J/K partial buffer and
// are summed by jk_reduce.
// ---------------------------------------------------------------------------
struct DirectArgs {
    const MolDesc* mol;
    const MolState* state;
    const JkItem* items;
    const Shell* shells;
    const Pair* pairs[3];
    const int2* pao[3];
    const double* pp[3];
    long npp[3];
    const double* Q[3];
    const double* tab;      // Boys table, FP64
    const float* tabf;      // Boys table, FP32
    const double* rows;     // Boys row tables (large-molecule kernels stage theirs in LDS)
    const double* P;
    const double* Pref;     // incremental build: digest P - Pref
    const double* dP;       // global mode: the digested density (materialised)
    void* part;
    long part_stride;
    double tol;             // density-weighted Schwarz threshold
    double cut;             // primitive prefactor cut
    int only_active;
};

constexpr int kDirectThreads = 256;

template <typename R> __device__ __forceinline__ const R* direct_tab(const DirectArgs& g);
template <> __device__ __forceinline__ const double* direct_tab<double>(const DirectArgs& g) { return g.tab; }
template <> __device__ __forceinline__ const float* direct_tab<float>(const DirectArgs& g) { return g.tabf; }

// work-group maximum (every thread gets it); ends with a barrier
__device__ __forceinline__ double block_max_direct(double mx, double* red)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) r = fmax(r, red[w]);
    return r;
}

template <int LA, int LB, int LC, int LD, typename A, typename R, int PP>
__device__ __forceinline__ void direct_class(const DirectArgs& g, const MolDesc& md, int chunk, int nchunk, double pmax,
                                             const A* __restrict__ Ps, A* AJ, A* AK)
{
    constexpr int C = (LA + LB == 0) ? 0 : (LA + LB == 1 ? (LC + LD == 0 ? 1 : 2) : (LC + LD == 0 ? 3 : (LC + LD == 1 ? 4 : 5)));
    constexpr int NA = LA ? 3 : 1, NB = LB ? 3 : 1, NC = LC ? 3 : 1, ND = LD ? 3 : 1;
    constexpr int NCOMP = NA * NB * NC * ND;
    const int N = md.nbf;
    const long nq = md.nq[C];
    const long lo = nq * chunk / nchunk, hi = nq * (chunk + 1) / nchunk;
    const int cb = class_bra(C), ck = class_ket(C);
    const int nket = md.npair[ck];
    const double* __restrict__ Qb = g.Q[cb] + md.pair0[cb];
    const double* __restrict__ Qk = g.Q[ck] + md.pair0[ck];
    const double qtol = pmax > 0.0 ? g.tol / pmax : 1e300;
    for (long q = lo + threadIdx.x; q < hi; q += blockDim.x) {
        int i, j;
        decode_quartet(C, q, nket, i, j);
        if (Qb[i] * Qk[j] < qtol) continue;
        const int ib = md.pair0[cb] + i, ik = md.pair0[ck] + j;
        const Pair P1 = g.pairs[cb][ib], P2 = g.pairs[ck][ik];
        const Shell sa = g.shells[P1.sa], sb = g.shells[P1.sb], sc = g.shells[P2.sa], sd = g.shells[P2.sb];
        const PairView<PP> vb{g.pp[cb], g.npp[cb], ib}, vk{g.pp[ck], g.npp[ck], ik};
        R I[NCOMP];
        eri_quartet<LA, LB, LC, LD, R, false, PP>(sa, sb, sc, sd, vb, vk, direct_tab<R>(g), R(g.cut), I);
        A Ia[NCOMP];
#pragma unroll
        for (int k = 0; k < NCOMP; k++) Ia[k] = A(I[k]);
        const int2 A1 = g.pao[cb][ib], A2 = g.pao[ck][ik];
        A f = A(1);
        if (A1.x >> 16) f *= A(0.5);
        if (A2.x >> 16) f *= A(0.5);
        if (class_tri(C) && i == j) f *= A(0.5);
        jk_scatter<NA, NB, NC, ND, A>(Ia, A1.x & 0xffff, A1.y, A2.x & 0xffff, A2.y, f, i, N, Ps, AJ, AK);
    }
}

// Large molecules (partials in global memory): the work group walks its
// quartet range one bra pair at a time.  Per bra the density rows of its two
// shells are staged in LDS (Prow) and their K rows accumulate in LDS (Krow,
// K_ac, K_ad, K_bc, K_bd), J_ab in registers; both are added to the partials
// once per bra, so only J_cd reaches global memory per quartet.
template <int LA, int LB, int LC, int LD, typename R, int PP>
__device__ __forceinline__ void direct_class_rows(const DirectArgs& g, const MolDesc& md, int chunk, int nchunk,
                                                  double pmax, const double* __restrict__ Pg, double* AJ, double* AK,
                                                  double* Prow, double* Krow, const double* boys_rows_l)
{
    constexpr int C = (LA + LB == 0) ? 0 : (LA + LB == 1 ? (LC + LD == 0 ? 1 : 2) : (LC + LD == 0 ? 3 : (LC + LD == 1 ? 4 : 5)));
    constexpr int NA = LA ? 3 : 1, NB = LB ? 3 : 1, NC = LC ? 3 : 1, ND = LD ? 3 : 1;
    constexpr int NCOMP = NA * NB * NC * ND;
    const int N = md.nbf;
    const long nq = md.nq[C];
    const long lo = nq * chunk / nchunk, hi = nq * (chunk + 1) / nchunk;
    if (lo >= hi) return;
    const int cb = class_bra(C), ck = class_ket(C);
    const int nket = md.npair[ck];
    const double* __restrict__ Qb = g.Q[cb] + md.pair0[cb];
    const double* __restrict__ Qk = g.Q[ck] + md.pair0[ck];
    const double qtol = pmax > 0.0 ? g.tol / pmax : 1e300;
    int i, j0;
    decode_quartet(C, lo, nket, i, j0);
    for (long q = lo; q < hi; i++, j0 = 0) {
        const int nk = class_tri(C) ? i + 1 : nket;
        int seg = (int)min((long)(nk - j0), hi - q);
        q += seg;
        // pairs are ordered by decreasing Schwarz factor, so the kets that
        // pass the test form a prefix of [j0, j0 + seg)
        const double qb = Qb[i];
        if (qb * Qk[j0] < qtol) continue;
        {
            int a = j0, z = j0 + seg;       // Qk[a] passes; find the first failing ket in (a, z)
            while (z - a > 1) {
                const int mid = (a + z) >> 1;
                if (qb * Qk[mid] < qtol) z = mid; else a = mid;
            }
            seg = z - j0;
        }
        const int ib = md.pair0[cb] + i;
        const int2 A1 = g.pao[cb][ib];
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
        const Pair P1 = g.pairs[cb][ib];
        const Shell sa = g.shells[P1.sa], sb = g.shells[P1.sb];
        const PairView<PP> vb{g.pp[cb], g.npp[cb], ib};
        for (int t = threadIdx.x; t < seg; t += blockDim.x) {
            const int j = j0 + t;
            const int ik = md.pair0[ck] + j;
            const Pair P2 = g.pairs[ck][ik];
            const Shell sc = g.shells[P2.sa], sd = g.shells[P2.sb];
            const PairView<PP> vk{g.pp[ck], g.npp[ck], ik};
            R Ir[NCOMP];
            if constexpr (std::is_same<R, double>::value)
                eri_quartet<LA, LB, LC, LD, R, true, PP>(sa, sb, sc, sd, vb, vk, boys_rows_l, R(g.cut), Ir);
            else
                eri_quartet<LA, LB, LC, LD, R, false, PP>(sa, sb, sc, sd, vb, vk, direct_tab<R>(g), R(g.cut), Ir);
            double I[NCOMP];
#pragma unroll
            for (int k = 0; k < NCOMP; k++) I[k] = double(Ir[k]);
            const int2 A2 = g.pao[ck][ik];
            double f = same ? 0.5 : 1.0;
            if (A2.x >> 16) f *= 0.5;
            if (class_tri(C) && i == j) f *= 0.5;
            jk_scatter_rows<NA, NB, NC, ND, double>(I, A2.x & 0xffff, A2.y, f, N, Prow, Prow + NA * N, Pg, pab,
                                                    jab, AJ, Krow, Krow + NA * N);
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

// Molecules whose J/K accumulators fit in LDS: ΔP, J and K in LDS, all six
// classes in one work group per item, the accumulators written out once.
template <typename A, typename R, int PP>
__global__ __launch_bounds__(kDirectThreads) void direct_jk_kernel(DirectArgs g)
{
    const JkItem it = g.items[blockIdx.x];
    if (g.only_active && g.state[it.mol].status != KS_MOL_ACTIVE) return;
    const MolDesc md = g.mol[it.mol];
    const int N = md.nbf, NN = N * N;
    extern __shared__ __align__(16) unsigned char smem_direct[];
    A* Pl = (A*)smem_direct;
    A* AJ = Pl + NN;
    A* AK = AJ + NN;
    __shared__ double red[kDirectThreads / 64];
    const double* P = g.P + md.mat0;
    const double* Pr = g.Pref ? g.Pref + md.mat0 : nullptr;
    double mx = 0.0;
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        const double v = Pr ? P[i] - Pr[i] : P[i];
        mx = fmax(mx, fabs(v));
        Pl[i] = A(v);
        AJ[i] = A(0);
        AK[i] = A(0);
    }
    const double pmax = block_max_direct(mx, red);
    direct_class<0, 0, 0, 0, A, R, PP>(g, md, it.chunk, it.nchunk, pmax, Pl, AJ, AK);
    direct_class<1, 0, 0, 0, A, R, PP>(g, md, it.chunk, it.nchunk, pmax, Pl, AJ, AK);
    direct_class<1, 0, 1, 0, A, R, PP>(g, md, it.chunk, it.nchunk, pmax, Pl, AJ, AK);
    direct_class<1, 1, 0, 0, A, R, PP>(g, md, it.chunk, it.nchunk, pmax, Pl, AJ, AK);
    direct_class<1, 1, 1, 0, A, R, PP>(g, md, it.chunk, it.nchunk, pmax, Pl, AJ, AK);
    direct_class<1, 1, 1, 1, A, R, PP>(g, md, it.chunk, it.nchunk, pmax, Pl, AJ, AK);
    __syncthreads();
    A* out = (A*)g.part + (size_t)blockIdx.x * 2 * g.part_stride;
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        out[i] = AJ[i];
        out[g.part_stride + i] = AK[i];
    }
}

// Larger molecules: one launch per class (each class gets its own register
// allocation), ΔP materialised in global memory (dP), J/K partials per item
// in global memory, zeroed by the first launch.
template <int LA, int LB, int LC, int LD, typename R, int PP>
__global__ __launch_bounds__(kDirectThreads) void direct_rows_kernel(DirectArgs g, int zero)
{
    const JkItem it = g.items[blockIdx.x];
    if (g.only_active && g.state[it.mol].status != KS_MOL_ACTIVE) return;
    const MolDesc md = g.mol[it.mol];
    const int N = md.nbf, NN = N * N;
    extern __shared__ __align__(16) unsigned char smem_direct[];
    double* AJ = (double*)g.part + (size_t)blockIdx.x * 2 * g.part_stride;
    double* AK = AJ + g.part_stride;
    const double* dP = g.dP + md.mat0;
    __shared__ double red[kDirectThreads / 64];
    double mx = 0.0;
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        mx = fmax(mx, fabs(dP[i]));
        if (zero) {
            AJ[i] = 0.0;
            AK[i] = 0.0;
        }
    }
    const double pmax = block_max_direct(mx, red);   // also orders the zeroing before the scatter
    double* rows = (double*)smem_direct;             // Boys row table of this class's L
    double* Prow = rows + kBoysNTR * kBoysKR;        // [6][N]
    double* Krow = Prow + 6 * N;                     // [6][N]
    {
        constexpr int L = LA + LB + LC + LD;
        const double2* src = (const double2*)(g.rows + (size_t)L * kBoysNTR * kBoysKR);
        for (int t = threadIdx.x; t < kBoysNTR * kBoysKR / 2; t += blockDim.x) ((double2*)rows)[t] = src[t];
        __syncthreads();
    }
    direct_class_rows<LA, LB, LC, LD, R, PP>(g, md, it.chunk, it.nchunk, pmax, dP, AJ, AK, Prow, Krow, rows);
}

// out[k] = in[perm[k]] for the per-pair arrays of one pair class (pairs,
// AO offsets, Schwarz factors and the field-major primitive-pair table).
__global__ void permute_pairs_kernel(const int* __restrict__ perm, long n, int pp, const Pair* __restrict__ pairs_in,
                                     const int2* __restrict__ pao_in, const double* __restrict__ pp_in,
                                     const double* __restrict__ Q_in, Pair* __restrict__ pairs_out,
                                     int2* __restrict__ pao_out, double* __restrict__ pp_out, double* __restrict__ Q_out)
{
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const long src = perm[k];
    pairs_out[k] = pairs_in[src];
    pao_out[k] = pao_in[src];
    Q_out[k] = Q_in[src];
    for (int f = 0; f < kPairFields * pp; f++) pp_out[(size_t)f * n + k] = pp_in[(size_t)f * n + src];
}

ks_status launch_permute_pairs(ks_batch* b, int c, const int* perm, Pair* pairs_out, int2* pao_out, double* pp_out,
                               double* Q_out)
{
    const long n = b->npairs[c];
    if (!n) return KS_OK;
    hipLaunchKernelGGL(permute_pairs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, b->stream, perm, n,
                       b->pp, b->d_pairs[c], b->d_pair_ao[c], b->d_pp[c], b->d_Q[c], pairs_out, pao_out, pp_out, Q_out);
    KS_HIP(hipGetLastError());
    return KS_OK;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
ks_status launch_int1e(ks_batch* b)
{
    KTimer tm(b, "int1e");
    int maxp = 0;
    for (auto& m : b->mol) maxp = std::max(maxp, m.nbf * (m.nbf + 1) / 2);
    dim3 grid((maxp + 127) / 128, b->n_mol);
    hipLaunchKernelGGL(int1e_kernel, grid, dim3(128), 0, b->stream, b->d_mol, b->d_shells, b->d_aoinfo, b->d_R,
                       b->d_Zc, b->d_boys, b->d_S, b->d_T, b->d_V, b->d_H);
    KS_HIP(hipGetLastError());
    return KS_OK;
}

ks_status launch_pairs(ks_batch* b)
{
    for (int c = 0; c < 3; c++) {
        long n = b->npairs[c] * b->pp;
        if (!n) continue;
        hipLaunchKernelGGL(pair_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, b->stream, b->d_shells,
                           b->d_pairs[c], b->npairs[c], b->pp, b->d_pp[c]);
        KS_HIP(hipGetLastError());
    }
    return KS_OK;
}

template <int LA, int LB, int LC, int LD, typename R, typename S, int PP>
static ks_status launch_class(ks_batch* b, int c)
{
    if (!b->nq[c]) return KS_OK;
    EriArgs g;
    g.mol = b->d_mol;
    g.qoff = b->d_qoff[c];
    g.n_mol = b->n_mol;
    g.nq = b->nq[c];
    g.shells = b->d_shells;
    g.pb = b->d_pairs[class_bra(c)];
    g.pk = b->d_pairs[class_ket(c)];
    g.ppb = b->d_pp[class_bra(c)];
    g.ppk = b->d_pp[class_ket(c)];
    g.npb = b->npairs[class_bra(c)];
    g.npk = b->npairs[class_ket(c)];
    g.tab = std::is_same<R, double>::value ? (const void*)b->d_boys : (const void*)b->d_boys_f;
    g.cut = b->opt.prec == KS_MIXED ? kEriCutMixed : kEriCutFp64;
    g.out = b->d_eri[c];
    g.Qb = b->d_Q[class_bra(c)];
    g.Qk = b->d_Q[class_ket(c)];
    g.schwarz = b->schwarz_done ? b->opt.schwarz_tol : 0.0;
    const int nt = b->opt.eri_threads[c] > 0 ? b->opt.eri_threads[c] : kEriThreads;
    const long nb = (g.nq + nt - 1) / nt;
    static const char* const kClassTimer[kNClass] = {"eri_ssss", "eri_psss", "eri_psps", "eri_ppss", "eri_ppps",
                                                      "eri_pppp"};
    KTimer tc(b, kClassTimer[c]);
    // the ket-loop unroll of the options (autotuned; 9 = fully unrolled) for
    // the STO-3G table, else by three
    if (PP == kNPrimPair && b->opt.eri_unroll[c] == 9)
        hipLaunchKernelGGL((eri_class_kernel<LA, LB, LC, LD, R, S, PP, (PP == kNPrimPair ? 9 : 3)>),
                           dim3((unsigned)nb), dim3(nt), 0, b->stream, g);
    else
        hipLaunchKernelGGL((eri_class_kernel<LA, LB, LC, LD, R, S, PP, 3>), dim3((unsigned)nb), dim3(nt), 0,
                           b->stream, g);
    KS_HIP(hipGetLastError());
    return KS_OK;
}

template <typename R, typename S, int PP>
static ks_status launch_all_classes(ks_batch* b)
{
    ks_status st;
    if ((st = launch_class<0, 0, 0, 0, R, S, PP>(b, 0))) return st;
    if ((st = launch_class<1, 0, 0, 0, R, S, PP>(b, 1))) return st;
    if ((st = launch_class<1, 0, 1, 0, R, S, PP>(b, 2))) return st;
    if ((st = launch_class<1, 1, 0, 0, R, S, PP>(b, 3))) return st;
    if ((st = launch_class<1, 1, 1, 0, R, S, PP>(b, 4))) return st;
    if ((st = launch_class<1, 1, 1, 1, R, S, PP>(b, 5))) return st;
    return KS_OK;
}

ks_status launch_eri(ks_batch* b)
{
    KTimer tm(b, "eri");
    // FP64 evaluation in both paths: evaluated in FP32, a 130-function
    // molecule's SCF energy moved by 1.2e-4 Ha against the oracle
    if (b->pp == kPrimPairMax)
        return b->opt.prec == KS_MIXED ? launch_all_classes<double, float, kPrimPairMax>(b)
                                       : launch_all_classes<double, double, kPrimPairMax>(b);
    if (b->opt.prec == KS_MIXED && b->max_np <= 96) return launch_all_classes<float, float, kNPrimPair>(b);
    if (b->opt.prec == KS_MIXED) return launch_all_classes<double, float, kNPrimPair>(b);
    return launch_all_classes<double, double, kNPrimPair>(b);
}

ks_status launch_eri_unpack(const ks_batch* b, int mol, double* d_out)
{
    const MolDesc& md = b->mol[mol];
    for (int c = 0; c < kNClass; c++) {
        if (!md.nq[c]) continue;
        const unsigned nb = (unsigned)((md.nq[c] + 127) / 128);
        if (b->opt.prec == KS_MIXED)
            hipLaunchKernelGGL(eri_unpack_kernel<float>, dim3(nb), dim3(128), 0, b->stream, b->d_mol, mol, c, b->nq[c],
                               b->d_shells, b->d_pairs[class_bra(c)], b->d_pairs[class_ket(c)],
                               (const float*)b->d_eri[c], d_out);
        else
            hipLaunchKernelGGL(eri_unpack_kernel<double>, dim3(nb), dim3(128), 0, b->stream, b->d_mol, mol, c, b->nq[c],
                               b->d_shells, b->d_pairs[class_bra(c)], b->d_pairs[class_ket(c)],
                               (const double*)b->d_eri[c], d_out);
        KS_HIP(hipGetLastError());
    }
    return KS_OK;
}

ks_status launch_eri_unpack_window(const ks_batch* b, int mol, long lo, long hi, double* d_out)
{
    const MolDesc& md = b->mol[mol];
    for (int c = 0; c < kNClass; c++) {
        if (!md.nq[c]) continue;
        const unsigned nb = (unsigned)((md.nq[c] + 127) / 128);
        if (b->opt.prec == KS_MIXED)
            hipLaunchKernelGGL(eri_unpack_window_kernel<float>, dim3(nb), dim3(128), 0, b->stream, b->d_mol, mol, c,
                               b->nq[c], b->d_shells, b->d_pairs[class_bra(c)], b->d_pairs[class_ket(c)],
                               (const float*)b->d_eri[c], lo, hi, d_out);
        else
            hipLaunchKernelGGL(eri_unpack_window_kernel<double>, dim3(nb), dim3(128), 0, b->stream, b->d_mol, mol, c,
                               b->nq[c], b->d_shells, b->d_pairs[class_bra(c)], b->d_pairs[class_ket(c)],
                               (const double*)b->d_eri[c], lo, hi, d_out);
        KS_HIP(hipGetLastError());
    }
    return KS_OK;
}

template <int LA, int LB, int PP>
static ks_status launch_schwarz_class(ks_batch* b, int c)
{
    const long n = b->npairs[c];
    if (!n) return KS_OK;
    hipLaunchKernelGGL((schwarz_kernel<LA, LB, PP>), dim3((unsigned)((n + 127) / 128)), dim3(128), 0, b->stream,
                       b->d_shells, b->d_pairs[c], b->d_pp[c], n, b->d_boys, b->d_Q[c]);
    KS_HIP(hipGetLastError());
    return KS_OK;
}

ks_status launch_schwarz(ks_batch* b)
{
    KTimer tm(b, "schwarz");
    ks_status st;
    if (b->pp == kPrimPairMax) {
        if ((st = launch_schwarz_class<0, 0, kPrimPairMax>(b, 0))) return st;
        if ((st = launch_schwarz_class<1, 0, kPrimPairMax>(b, 1))) return st;
        if ((st = launch_schwarz_class<1, 1, kPrimPairMax>(b, 2))) return st;
    } else {
        if ((st = launch_schwarz_class<0, 0, kNPrimPair>(b, 0))) return st;
        if ((st = launch_schwarz_class<1, 0, kNPrimPair>(b, 1))) return st;
        if ((st = launch_schwarz_class<1, 1, kNPrimPair>(b, 2))) return st;
    }
    b->schwarz_done = true;
    return KS_OK;
}

template <int LA, int LB, int LC, int LD, typename R, int PP>
static ks_status launch_direct_rows(ks_batch* b, const DirectArgs& g, size_t lds, int zero)
{
    KS_HIP(hipFuncSetAttribute((const void*)direct_rows_kernel<LA, LB, LC, LD, R, PP>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((direct_rows_kernel<LA, LB, LC, LD, R, PP>), dim3((unsigned)b->jk_items.size()),
                       dim3(kDirectThreads), lds, b->stream, g, zero);
    KS_HIP(hipGetLastError());
    return KS_OK;
}

// Integrals evaluated in R (the Boys table of that type), accumulated in A.
template <typename A, typename R, bool GLOBAL, int PP>
static ks_status run_direct_jk(ks_batch* b, const double* P, bool only_active, bool incremental)
{
    DirectArgs g;
    g.mol = b->d_mol;
    g.state = b->d_state;
    g.items = b->d_jk_items;
    g.shells = b->d_shells;
    for (int c = 0; c < 3; c++) {
        g.pairs[c] = b->d_pairs[c];
        g.pao[c] = b->d_pair_ao[c];
        g.pp[c] = b->d_pp[c];
        g.npp[c] = b->npairs[c];
        g.Q[c] = b->d_Q[c];
    }
    g.tab = b->d_boys;
    g.tabf = b->d_boys_f;
    g.rows = b->d_boys_rows;
    g.P = P;
    g.Pref = incremental ? b->d_Pprev : nullptr;
    g.dP = b->d_work;
    if (GLOBAL) {
        ks_status st = launch_delta(b, P, g.Pref, only_active);
        if (st) return st;
    }
    g.part = b->d_jk_part;
    g.part_stride = (long)b->max_np * b->max_np;
    g.tol = b->opt.schwarz_tol > 0.0 ? b->opt.schwarz_tol : (b->opt.prec == KS_MIXED ? 1e-10 : 1e-12);
    g.cut = b->opt.prec == KS_MIXED ? kEriCutMixed : kEriCutFp64;
    g.only_active = only_active;
    int maxn = 0;
    for (auto& m : b->mol) maxn = std::max(maxn, m.nbf);
    KTimer tm(b, "jk_direct");
    if constexpr (GLOBAL) {
        static_assert(std::is_same<A, double>::value, "global partials are FP64");
        const size_t lds = (kBoysNTR * kBoysKR + 12 * (size_t)maxn) * sizeof(double);
        ks_status st;
        if ((st = launch_direct_rows<0, 0, 0, 0, R, PP>(b, g, lds, 1))) return st;
        if ((st = launch_direct_rows<1, 0, 0, 0, R, PP>(b, g, lds, 0))) return st;
        if ((st = launch_direct_rows<1, 0, 1, 0, R, PP>(b, g, lds, 0))) return st;
        if ((st = launch_direct_rows<1, 1, 0, 0, R, PP>(b, g, lds, 0))) return st;
        if ((st = launch_direct_rows<1, 1, 1, 0, R, PP>(b, g, lds, 0))) return st;
        return launch_direct_rows<1, 1, 1, 1, R, PP>(b, g, lds, 0);
    } else {
        const size_t lds = 3 * (size_t)maxn * maxn * sizeof(A);
        KS_HIP(hipFuncSetAttribute((const void*)direct_jk_kernel<A, R, PP>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL((direct_jk_kernel<A, R, PP>), dim3((unsigned)b->jk_items.size()), dim3(kDirectThreads), lds,
                           b->stream, g);
        KS_HIP(hipGetLastError());
        return KS_OK;
    }
}

ks_status launch_direct_jk(ks_batch* b, const double* P, double* J, double* K, bool only_active, bool incremental,
                           bool track)
{
    if (!b->schwarz_done) {
        ks_status st = launch_schwarz(b);
        if (st) return st;
    }
    if (!b->pairs_sorted) {     // the bra-major digestion relies on the order
        ks_status st = sort_pairs_by_schwarz(b);
        if (st) return st;
    }
    const int mode = jk_mode(b);
    const bool f64 = mode != 1;
    // integrals evaluated in FP64 in both paths (as in the stored build)
    ks_status st;
    if (b->pp == kPrimPairMax)
        st = mode == 0 ? run_direct_jk<double, double, false, kPrimPairMax>(b, P, only_active, incremental)
           : mode == 1 ? run_direct_jk<float, double, false, kPrimPairMax>(b, P, only_active, incremental)
                       : run_direct_jk<double, double, true, kPrimPairMax>(b, P, only_active, incremental);
    else
        st = mode == 0 ? run_direct_jk<double, double, false, kNPrimPair>(b, P, only_active, incremental)
           : mode == 1 ? run_direct_jk<float, double, false, kNPrimPair>(b, P, only_active, incremental)
                       : run_direct_jk<double, double, true, kNPrimPair>(b, P, only_active, incremental);
    if (st) return st;
    return launch_jk_reduce(b, f64, P, J, K, only_active, incremental, track);
}

}  // namespace ks
