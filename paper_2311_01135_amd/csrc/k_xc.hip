// Becke-partitioned atom-centred grid and the fused exchange-correlation
// integration (paper section 3.1: V_XC(rho); section 3.2 "Libxc": B3LYP in
// float32; section 5 "Recomputation": AO values recomputed on the grid
// instead of stored).
//
// Grid: per atom a Treutler-Ahlrichs M4 radial rule (xi = 1) x Gauss-Legendre
// in cos(theta) x trapezoid in phi, weighted by Becke fuzzy-cell functions
// (three smoothing steps, no size adjustment).
//
// XC: one work group walks a contiguous chunk of one molecule's grid in
// sub-blocks of BP points, with the molecule's density P and shell table in
// LDS.  Per sub-block it evaluates the AO values and gradients into AO-major
// LDS planes, forms X^T = P Phi^T with 16x16x4 MFMAs and, from each X tile
// still in registers, its share of rho = sum X Phi and grad rho =
// 2 sum X grad Phi; evaluates B3LYP (three wavefronts, one part each); forms
// W = w (v_rho/2 Phi + 2 v_sigma grad rho . grad Phi) in place of d/dx Phi;
// and accumulates A += Phi^T W with MFMAs into register tiles that persist
// over the whole chunk.  V_XC = sum_chunks (A + A^T) is summed in FP64
// afterwards.
#include "kernels.h"
#include "wave.h"

namespace ks {

// ---------------------------------------------------------------------------
// grid points and Becke weights
// ---------------------------------------------------------------------------
// Becke's smoothing polynomial applied three times, f3(mu); the cell
// function is s(mu) = (1 - f3(mu))/2, and f3 is odd, so s(-mu) = (1 + f3(mu))/2.
template <typename T>
__device__ __forceinline__ T becke_f3(T mu)
{
#pragma unroll
    for (int k = 0; k < 3; k++) mu = T(1.5) * mu - T(0.5) * mu * mu * mu;
    return mu;
}

// blockIdx.y = molecule; each thread one of its points.  LDS: atom
// positions, inverse interatomic distances, and per thread the distances to
// every atom and the cell products P_a (both transposed: [atom][thread]).
// Each atom pair (a < c) evaluates f3 once: s(mu_ac) multiplies P_a and
// s(mu_ca) = s(-mu_ac) multiplies P_c, so every P_a receives its factors in
// ascending order of the other atom.  Points are placed in FP64; the cell
// functions run in T (FP32 in the mixed path: half the LDS per thread, so
// twice the resident waves, at twice the vector rate).
template <typename T>
__global__ __launch_bounds__(64) void grid_kernel(const MolDesc* __restrict__ mols, const double* __restrict__ Rat,
                                                  const double* __restrict__ radial, const double* __restrict__ ang,
                                                  int nrad, int nth, int nph, int coarse, double* __restrict__ out)
{
    const int m = blockIdx.y;
    const MolDesc md = mols[m];
    const long base = coarse ? md.gridc0 : md.grid0, ng = coarse ? md.ngridc : md.ngrid;
    const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
    extern __shared__ double smem_grid[];
    const int na = md.natom;
    const int bs = blockDim.x, t = threadIdx.x;
    double* Ra = smem_grid;                       // [natom][3]
    T* invR = (T*)(Ra + 3 * na);                  // [natom][natom]: 1/|R_a - R_c|
    T* dist = invR + na * na;                     // [natom][bs]
    T* Pc = dist + na * bs;                       // [natom][bs]
    for (int i = threadIdx.x; i < 3 * na; i += blockDim.x) Ra[i] = Rat[3 * md.atom0 + i];
    for (int i = threadIdx.x; i < na * na; i += blockDim.x) {
        const int a = i / na, c = i % na;
        const double* pa = Rat + 3 * (md.atom0 + a);
        const double* pc = Rat + 3 * (md.atom0 + c);
        const double dx = pa[0] - pc[0], dy = pa[1] - pc[1], dz = pa[2] - pc[2];
        invR[i] = a == c ? T(0) : T(1.0 / sqrt(dx * dx + dy * dy + dz * dz));
    }
    __syncthreads();
    if (l >= ng) return;
    const int per_atom = nrad * nth * nph;
    const int A = (int)(l / per_atom);
    int rem = (int)(l % per_atom);
    const int i = rem / (nth * nph);
    rem %= nth * nph;
    const int j = rem / nph, k = rem % nph;
    const double ct = ang[j], st = sqrt(1.0 - ct * ct), ph = 2.0 * kPi * k / nph;
    const double r = radial[i];
    double p[3];
    p[0] = Ra[3 * A] + r * st * cos(ph);
    p[1] = Ra[3 * A + 1] + r * st * sin(ph);
    p[2] = Ra[3 * A + 2] + r * ct;
    for (int a = 0; a < na; a++) {
        const double dx = p[0] - Ra[3 * a], dy = p[1] - Ra[3 * a + 1], dz = p[2] - Ra[3 * a + 2];
        dist[a * bs + t] = T(sqrt(dx * dx + dy * dy + dz * dz));
        Pc[a * bs + t] = T(1);
    }
    T num = T(0), den = T(0);
    for (int a = 0; a < na; a++) {
        const T ra = dist[a * bs + t];
        const T* ir = invR + a * na;
        T Pa = Pc[a * bs + t];
        for (int c = a + 1; c < na; c++) {
            const T f = becke_f3<T>((ra - dist[c * bs + t]) * ir[c]);
            Pa *= T(0.5) * (T(1) - f);
            Pc[c * bs + t] *= T(0.5) * (T(1) + f);
        }
        if (a == A) num = Pa;
        den += Pa;
    }
    const double w = radial[nrad + i] * ang[nth + j] * (2.0 * kPi / nph) * ((double)num / (double)den);
    double* o = out + 4 * (base + l);
    o[0] = p[0];
    o[1] = p[1];
    o[2] = p[2];
    o[3] = w;
}

// Register form for the FP32 cell functions of molecules of at most NA
// atoms: each thread keeps its distances and cell products in registers
// (fully unrolled loops, guarded by the molecule's atom count, which is
// uniform over the work group) and reads the inverse interatomic distances
// from LDS at the same address on every lane.  The products are formed in
// the same order as in grid_kernel.
template <int NA>
__global__ __launch_bounds__(64) void grid_kernel_reg(const MolDesc* __restrict__ mols, const double* __restrict__ Rat,
                                                      const double* __restrict__ radial, const double* __restrict__ ang,
                                                      int nrad, int nth, int nph, int coarse, double* __restrict__ out)
{
    const int m = blockIdx.y;
    const MolDesc md = mols[m];
    const long base = coarse ? md.gridc0 : md.grid0, ng = coarse ? md.ngridc : md.ngrid;
    const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ double Ra[3 * NA];
    __shared__ float invR[NA * NA];                  // row stride NA
    const int na = md.natom;
    for (int i = threadIdx.x; i < 3 * na; i += blockDim.x) Ra[i] = Rat[3 * md.atom0 + i];
    for (int i = threadIdx.x; i < na * na; i += blockDim.x) {
        const int a = i / na, c = i % na;
        const double* pa = Rat + 3 * (md.atom0 + a);
        const double* pc = Rat + 3 * (md.atom0 + c);
        const double dx = pa[0] - pc[0], dy = pa[1] - pc[1], dz = pa[2] - pc[2];
        invR[a * NA + c] = a == c ? 0.0f : float(1.0 / sqrt(dx * dx + dy * dy + dz * dz));
    }
    __syncthreads();
    if (l >= ng) return;
    const int per_atom = nrad * nth * nph;
    const int A = (int)(l / per_atom);
    int rem = (int)(l % per_atom);
    const int i = rem / (nth * nph);
    rem %= nth * nph;
    const int j = rem / nph, k = rem % nph;
    const double ct = ang[j], st = sqrt(1.0 - ct * ct), ph = 2.0 * kPi * k / nph;
    const double r = radial[i];
    double p[3];
    p[0] = Ra[3 * A] + r * st * cos(ph);
    p[1] = Ra[3 * A + 1] + r * st * sin(ph);
    p[2] = Ra[3 * A + 2] + r * ct;
    float d[NA], P[NA];
#pragma unroll
    for (int a = 0; a < NA; a++) {
        d[a] = 0.0f;
        P[a] = 1.0f;
        if (a < na) {
            const double dx = p[0] - Ra[3 * a], dy = p[1] - Ra[3 * a + 1], dz = p[2] - Ra[3 * a + 2];
            d[a] = float(sqrt(dx * dx + dy * dy + dz * dz));
        }
    }
    float num = 0.0f, den = 0.0f;
#pragma unroll
    for (int a = 0; a < NA; a++) {
        if (a < na) {
            float Pa = P[a];
#pragma unroll
            for (int c = a + 1; c < NA; c++) {
                if (c < na) {
                    const float f = becke_f3<float>((d[a] - d[c]) * invR[a * NA + c]);
                    Pa *= 0.5f * (1.0f - f);
                    P[c] *= 0.5f * (1.0f + f);
                }
            }
            if (a == A) num = Pa;
            den += Pa;
        }
    }
    const double w = radial[nrad + i] * ang[nth + j] * (2.0 * kPi / nph) * ((double)num / (double)den);
    double* o = out + 4 * (base + l);
    o[0] = p[0];
    o[1] = p[1];
    o[2] = p[2];
    o[3] = w;
}

template <typename T>
static ks_status run_grid(ks_batch* b, hipStream_t s, bool coarse)
{
    long maxg = 0;
    int maxat = 0;
    for (auto& m : b->mol) {
        maxg = std::max(maxg, coarse ? m.ngridc : m.ngrid);
        maxat = std::max(maxat, m.natom);
    }
    int bs = 64;
    auto lds_for = [&](int n) {
        return sizeof(double) * 3 * maxat + sizeof(T) * ((size_t)maxat * maxat + 2 * (size_t)maxat * n);
    };
    const ks_options& o = b->opt;
    if constexpr (sizeof(T) == 4) {
        if (maxat <= 48) {
            auto go = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3((unsigned)((maxg + 63) / 64), b->n_mol), dim3(64), 0, s, b->d_mol,
                                   b->d_R, coarse ? b->d_radial_c : b->d_radial, coarse ? b->d_ang_c : b->d_ang,
                                   coarse ? o.coarse_rad : o.n_rad, coarse ? o.coarse_theta : o.n_theta,
                                   coarse ? o.coarse_phi : o.n_phi, (int)coarse, b->d_grid);
            };
            if (maxat <= 16) go(grid_kernel_reg<16>);
            else if (maxat <= 32) go(grid_kernel_reg<32>);
            else go(grid_kernel_reg<48>);
            KS_HIP(hipGetLastError());
            return KS_OK;
        }
    }
    while (bs > 16 && lds_for(bs) > 163840) bs /= 2;
    const size_t lds = lds_for(bs);
    if (lds > 163840) {
        set_error("grid: %d atoms exceed the LDS budget", maxat);
        return KS_EUNSUPPORTED;
    }
    KS_HIP(hipFuncSetAttribute((const void*)grid_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(grid_kernel<T>, dim3((unsigned)((maxg + bs - 1) / bs), b->n_mol), dim3(bs), lds, s,
                       b->d_mol, b->d_R, coarse ? b->d_radial_c : b->d_radial, coarse ? b->d_ang_c : b->d_ang,
                       coarse ? o.coarse_rad : o.n_rad, coarse ? o.coarse_theta : o.n_theta,
                       coarse ? o.coarse_phi : o.n_phi, (int)coarse, b->d_grid);
    KS_HIP(hipGetLastError());
    return KS_OK;
}

// The coarse start grid (when in use) first: the first iterations need only it.
ks_status launch_grid(ks_batch* b, hipStream_t s)
{
    KTimer tm(b, "grid", s);
    ks_status st;
    if (b->coarse && (st = b->opt.prec == KS_MIXED ? run_grid<float>(b, s, true) : run_grid<double>(b, s, true)))
        return st;
    return b->opt.prec == KS_MIXED ? run_grid<float>(b, s, false) : run_grid<double>(b, s, false);
}

// ---------------------------------------------------------------------------
// Elementary functions of the functional.  FP64: libm and IEEE division.
// FP32 (the mixed path, whose tolerance is 1e-4 Ha): the hardware
// reciprocal, square root, log2 and exp2 (about 1 ulp each); cbrt as
// exp2(log2(x)/3), asinh as log(x + sqrt(x^2 + 1)) for x >= 0.
// ---------------------------------------------------------------------------
namespace fm {
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double log_(double x) { return log(x); }
__device__ __forceinline__ float log_(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994531f; }
__device__ __forceinline__ double exp_(double x) { return exp(x); }
__device__ __forceinline__ float exp_(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ double cbrt_(double x) { return cbrt(x); }
__device__ __forceinline__ float cbrt_(float x) { return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 3.0f)); }
__device__ __forceinline__ double asinh_(double x) { return asinh(x); }
__device__ __forceinline__ float asinh_(float x) { return log_(x + sqrt_(x * x + 1.0f)); }
__device__ __forceinline__ double atan_(double x) { return atan(x); }
__device__ __forceinline__ float atan_(float x) { return atanf(x); }
}  // namespace fm

// ---------------------------------------------------------------------------
// B3LYP, closed shell: energy per volume e and v_rho = de/drho,
// v_sigma = de/dsigma (sigma = |grad rho|^2).
// e = 0.08 Slater + 0.72 B88 + 0.19 VWN + 0.81 LYP, evaluated as three
// weighted parts (exchange, VWN, LYP) that the XC kernel hands to three
// wavefronts; part k adds its e, v_rho, v_sigma.
// ---------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ void b3lyp_exchange(F rho, F sigma, F& e, F& vr, F& vs)
{
    const F r13 = fm::cbrt_(rho);
    // Slater exchange, -(3/4)(3/pi)^(1/3) rho^(4/3)
    const F cs = F(0.7385587663820224);
    const F eS = -cs * rho * r13;
    const F vS = F(-4.0 / 3.0) * cs * r13;
    // Becke 88, both spins: rho_s = rho/2, g_s = sqrt(sigma)/2, x = g_s / rho_s^(4/3)
    const F beta = F(0.0042), Cx = F(0.9305257363491000);   // (3/2)(3/(4 pi))^(1/3)
    const F rs13 = r13 * F(0.7937005259840998);               // (rho/2)^(1/3)
    const F rs43 = F(0.5) * rho * rs13;
    const F irs43 = fm::rcp(rs43);
    const F x = F(0.5) * fm::sqrt_(sigma) * irs43;
    const F ash = fm::asinh_(x);
    const F D = F(1) + F(6) * beta * x * ash;
    const F iD = fm::rcp(D);
    const F Dp = F(6) * beta * (ash + x * fm::rcp(fm::sqrt_(F(1) + x * x)));
    const F gx = x * iD;                      // g(x)/x with g = x^2/D
    const F gpx = (F(2) * D - x * Dp) * iD * iD;   // g'(x)/x
    const F eB = F(-2) * rs43 * (Cx + beta * x * gx);
    const F vB = F(-4.0 / 3.0) * rs13 * (Cx + beta * x * (gx - x * gpx));
    const F sB = F(-0.25) * beta * gpx * irs43;
    e = F(0.08) * eS + F(0.72) * eB;
    vr = F(0.08) * vS + F(0.72) * vB;
    vs = F(0.72) * sB;
}

template <typename F>
__device__ __forceinline__ void b3lyp_vwn(F rho, int vwn5, F& e, F& vr, F& vs)
{
    // VWN (paramagnetic), x_v = sqrt(r_s), r_s = (3/(4 pi rho))^(1/3)
    F b, c, x0;
    if (vwn5) { b = F(3.72744); c = F(12.9352); x0 = F(-0.10498); }
    else { b = F(13.0720); c = F(42.7198); x0 = F(-0.409286); }
    const F Av = F(0.0310907);
    const F rsv = F(0.6203504908994001) * fm::rcp(fm::cbrt_(rho));   // (3/(4 pi))^(1/3) rho^(-1/3)
    const F xv = fm::sqrt_(rsv);
    const F X = xv * xv + b * xv + c, X0 = x0 * x0 + b * x0 + c, Q = fm::sqrt_(F(4) * c - b * b);
    const F iX = fm::rcp(X), iQ = fm::rcp(Q);
    const F at = fm::atan_(Q * fm::rcp(F(2) * xv + b));
    const F bxX0 = b * x0 * fm::rcp(X0);
    const F epsv = Av * (fm::log_(xv * xv * iX) + F(2) * b * iQ * at
                         - bxX0 * (fm::log_((xv - x0) * (xv - x0) * iX) + F(2) * (b + F(2) * x0) * iQ * at));
    const F deps = Av * (F(2) * fm::rcp(xv) - (F(2) * xv + b) * iX - b * iX
                         - bxX0 * (F(2) * fm::rcp(xv - x0) - (F(2) * xv + b) * iX - (b + F(2) * x0) * iX));
    e = F(0.19) * rho * epsv;
    vr = F(0.19) * (epsv - xv * deps * F(1.0 / 6.0));
    vs = F(0);
}

template <typename F>
__device__ __forceinline__ void b3lyp_lyp(F rho, F sigma, F& e, F& vr, F& vs)
{
    // LYP, closed-shell gradient form; t = rho^(-1/3)
    const F la = F(0.04918), lb = F(0.132), lc = F(0.2533), ld = F(0.349);
    const F CF = F(2.8712340001881915);      // (3/10)(3 pi^2)^(2/3)
    const F t = fm::rcp(fm::cbrt_(rho)), den = F(1) + ld * t, iden = fm::rcp(den);
    const F Ee = fm::exp_(-lc * t) * iden;
    const F delta = lc * t + ld * t * iden;
    const F t5 = t * t * t * t * t;          // rho^(-5/3)
    const F abE = la * lb * Ee;
    const F eL = -la * rho * iden - abE * CF * rho + abE * F(1.0 / 72.0) * t5 * sigma * (F(3) + F(7) * delta);
    const F vL = -la * iden - la * ld * t * F(1.0 / 3.0) * iden * iden - abE * CF * (F(1) + delta * F(1.0 / 3.0))
                 + abE * F(1.0 / 216.0) * sigma * t5 * fm::rcp(rho)
                       * (F(7) * delta * delta - F(39) * delta - F(15) + F(7) * ld * ld * t * t * iden * iden);
    const F sL = abE * F(1.0 / 72.0) * t5 * (F(3) + F(7) * delta);
    e = F(0.81) * eL;
    vr = F(0.81) * vL;
    vs = F(0.81) * sL;
}

// ---------------------------------------------------------------------------
// MFMA wrappers: A operand lane l holds A[l%16][l/16], B operand B[l/16][l%16];
// output register r of lane l holds D[row(l, r)][l%16].
// ---------------------------------------------------------------------------
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
    typedef d4_t V;
    static __device__ __forceinline__ V run(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
    typedef f4_t V;
    static __device__ __forceinline__ V run(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// exp in the compute type: FP64 libm exp; FP32 hardware exp2 (v_exp_f32) of
// x log2(e), relative error ~|x| 1e-7 for the |x| < 40 used by the AO values.
__device__ __forceinline__ double fast_exp(double x) { return exp(x); }
__device__ __forceinline__ float fast_exp(float x) { return __expf(x); }

// padded copy of P in the compute type: Pt[m] is np x np, zero outside nbf.
template <typename T>
__global__ void pad_density_kernel(const MolDesc* __restrict__ mols, const MolState* __restrict__ state,
                                   const long* __restrict__ ptoff, const double* __restrict__ P, T* __restrict__ Pt,
                                   int only_active)
{
    const int m = blockIdx.y;
    if (only_active && state[m].status != KS_MOL_ACTIVE) return;
    const MolDesc md = mols[m];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= md.np * md.np) return;
    const int i = t / md.np, j = t % md.np;
    Pt[ptoff[m] + t] = (i < md.nbf && j < md.nbf) ? (T)P[md.mat0 + i * md.nbf + j] : T(0);
}

struct XcArgs {
    const MolDesc* mol;
    const MolState* state;
    const XcItem* items;
    const Shell* shells;
    const double* grid;
    const void* Pt;
    const long* ptoff;
    void* part;             // [items][np_max^2]
    double* part_exc;       // [items]
    long part_stride;
    int vwn5;
    int only_active;
    int ns_max;             // largest shell count of the batch (LDS shell table)
    int npm;                // primitives per shell in the shell table (3 STO-3G, 6 6-31G; zero-padded)
};

// Shell table of one molecule as the XC kernel keeps it in LDS: centres,
// exponents and coefficients in the compute type, AO offset and L.
template <typename T>
struct ShellLds {
    double* A;      // [ns][3]
    T* ac;          // [ns][12]: a0 a1 a2 c0 c1 c2, then a3 a4 a5 c3 c4 c5 (zero past the shell's count)
    int* info;      // [ns]: ao | L << 16
};

// Launch shapes.  BP points per sub-block, NW wavefronts per work group.
// LDS, each piece 32-byte aligned: points and per-wave sums (FP64), the
// shell table, per-point density and gradient, the three functional parts,
// the per-AO-tile density partials, the padded density P (row stride NP + 4)
// and four AO-major planes [AO][point] (row stride BP + 4): Phi, d/dx Phi
// (overwritten by W once the density is formed), d/dy Phi, d/dz Phi; the
// FP32 path adds a fifth, Phi as bf16 pairs.
__host__ __device__ constexpr size_t al32(size_t x) { return (x + 31) & ~(size_t)31; }
__host__ __device__ constexpr int xc_ldp(int np) { return np + 4; }
__host__ __device__ constexpr int xc_ldg(int bp) { return bp + 4; }
__host__ __device__ constexpr size_t xc_lds_bytes_for(size_t es, int bp, int nw, int np, int ns,
                                                      bool pglobal = false)
{
    return al32((size_t)bp * 4 * sizeof(double)) + al32((size_t)nw * sizeof(double))
           + al32((size_t)ns * 3 * sizeof(double)) + al32((size_t)ns * 2 * kPrimMax * es) + al32((size_t)bp * 4 * es)
           + al32((size_t)bp * 9 * es) + al32((size_t)(np / 16) * 4 * bp * es)
           + (pglobal ? 0 : al32((size_t)np * xc_ldp(np) * es))
           + al32((size_t)(es == sizeof(float) ? 5 : 4) * np * xc_ldg(bp) * es) + al32((size_t)ns * sizeof(int));
}

constexpr size_t kLdsMax = 163840;

// ---------------------------------------------------------------------------
// FP32 path: AO values and W are held as split pairs x = hi + lo of bf16
// values (hi = bf16(x), lo = bf16(x - hi); |x - hi - lo| <= 2^-17 |x|), one
// 32-bit word per element with hi in the low half.  A 16x16x32 bf16 MFMA over
// pair-interleaved operands sums hi*hi + lo*lo; a second one with one
// operand's halves swapped adds hi*lo + lo*hi, so two MFMAs form the exact
// product of the two pairs (fp32 accumulation) for 16 k at a time, against
// four 16x16x4 FP32 MFMAs at a quarter of the rate.  Only V_XC = Phi^T W + ...
// uses it.  The density and E_XC keep FP32 AO values and FP32 MFMAs: rounding
// P would perturb every point alike (a ~1e-5 Fock-matrix error that stalls
// the SCF at the mixed-path thresholds), and rounding Phi, which repeats on
// each radial shell, biases E_XC by ~1e-5 Ha.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned int bf16_pair(float x)
{
    const __bf16 h = (__bf16)x;
    const __bf16 l = (__bf16)(x - (float)h);
    return (unsigned int)__builtin_bit_cast(unsigned short, h) | ((unsigned int)__builtin_bit_cast(unsigned short, l) << 16);
}
__device__ __forceinline__ unsigned int pair_swap(unsigned int w) { return (w >> 16) | (w << 16); }
__device__ __forceinline__ f4_t mfma_pair(u32x4_t a, u32x4_t b, f4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                    c, 0, 0, 0);
}

// The MFMA k index runs over 16-wide blocks: within a block, lane group
// q = lane / 16 supplies k = 4 q + j to the j-th of four MFMAs, so a lane's
// four values along k are contiguous in LDS (one vector read) whenever the
// operand is stored k-contiguous.

// X^T tiles (t = wave + NW j, j < NJ; AO tile t / (BP/16), point tile
// t % (BP/16)) of X^T = P Phi^T over K = NP, then, from the tile in
// registers, this tile's share of rho = sum_mu X Phi and of
// sum_mu X grad Phi at its 16 points, written to rpart[AO tile][4][BP].
template <typename T, int BP, int NW, int NJ>
__device__ __forceinline__ void gemm_x_rho(const T* __restrict__ Pl, const T* __restrict__ Phi, T* __restrict__ rpart,
                                           int LDP, int LDG, int PL, int NP, int wave, int lane)
{
    typedef typename Mfma<T>::V V;
    constexpr int GT = BP / 16;
    const int l16 = lane & 15, q = lane >> 4;
    V c[NJ];
    int pa[NJ], pb[NJ];
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int t = wave + j * NW;
        pa[j] = ((t / GT) * 16 + l16) * LDP + 4 * q;
        pb[j] = 4 * q * LDG + (t % GT) * 16 + l16;
#pragma unroll
        for (int r = 0; r < 4; r++) c[j][r] = T(0);
    }
    for (int kk = 0; kk < NP; kk += 16) {
        V a[NJ];
        T bv[NJ][4];
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            a[j] = *(const V*)(Pl + pa[j] + kk);
#pragma unroll
            for (int i = 0; i < 4; i++) bv[j][i] = Phi[pb[j] + (kk + i) * LDG];
        }
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < NJ; j++) c[j] = Mfma<T>::run(a[j][i], bv[j][i], c[j]);
    }
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int t = wave + j * NW, mt = t / GT, gpt = (t % GT) * 16 + l16;
        T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int o = (mt * 16 + Mfma<T>::row(lane, r)) * LDG + gpt;
            const T x = c[j][r];
            s0 += x * Phi[o];
            s1 += x * Phi[PL + o];
            s2 += x * Phi[2 * PL + o];
            s3 += x * Phi[3 * PL + o];
        }
        s0 = sum_rows(s0);
        s1 = sum_rows(s1);
        s2 = sum_rows(s2);
        s3 = sum_rows(s3);
        if (q == 0) {
            T* rp = rpart + mt * 4 * BP + gpt;
            rp[0] = s0;
            rp[BP] = s1;
            rp[2 * BP] = s2;
            rp[3 * BP] = s3;
        }
    }
}

// acc[j] += tile (t = wave + NW j) of Phi^T W over the BP points of a
// sub-block; both operands AO-major, so each k block is two vector reads.
template <typename T, int NW, int BP, int MAXT, int NJ>
__device__ __forceinline__ void gemm_phit_w(const T* __restrict__ Phi, const T* __restrict__ Wt, int LDG, int NT,
                                            int wave, int lane, typename Mfma<T>::V (&acc)[MAXT])
{
    if constexpr (NJ <= MAXT) {
        typedef typename Mfma<T>::V V;
        const int l16 = lane & 15, q = lane >> 4;
        int pa[NJ], pb[NJ];
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            const int t = wave + j * NW;
            pa[j] = ((t / NT) * 16 + l16) * LDG + 4 * q;
            pb[j] = ((t % NT) * 16 + l16) * LDG + 4 * q;
        }
#pragma unroll
        for (int kk = 0; kk < BP; kk += 16) {
            V a[NJ], bv[NJ];
#pragma unroll
            for (int j = 0; j < NJ; j++) {
                a[j] = *(const V*)(Phi + pa[j] + kk);
                bv[j] = *(const V*)(Wt + pb[j] + kk);
            }
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < NJ; j++) acc[j] = Mfma<T>::run(a[j][i], bv[j][i], acc[j]);
        }
    }
}

// acc[j] += tile of Phi^T W from the Phi and W pair planes (both AO-major).
template <int NW, int BP, int MAXT, int NJ>
__device__ __forceinline__ void gemm_phit_w_pair(const unsigned int* __restrict__ Phi, const unsigned int* __restrict__ Wt,
                                                 int LDG, int NT, int wave, int lane, f4_t (&acc)[MAXT])
{
    if constexpr (NJ <= MAXT) {
        const int l16 = lane & 15, q = lane >> 4;
        int pa[NJ], pb[NJ];
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            const int t = wave + j * NW;
            pa[j] = ((t / NT) * 16 + l16) * LDG + 4 * q;
            pb[j] = ((t % NT) * 16 + l16) * LDG + 4 * q;
        }
#pragma unroll
        for (int kk = 0; kk < BP; kk += 16) {
            u32x4_t a[NJ], bv[NJ];
#pragma unroll
            for (int j = 0; j < NJ; j++) {
                a[j] = *(const u32x4_t*)(Phi + pa[j] + kk);
                bv[j] = *(const u32x4_t*)(Wt + pb[j] + kk);
            }
#pragma unroll
            for (int j = 0; j < NJ; j++) {
                u32x4_t bs;
#pragma unroll
                for (int i = 0; i < 4; i++) bs[i] = pair_swap(bv[j][i]);
                acc[j] = mfma_pair(a[j], bv[j], acc[j]);
                acc[j] = mfma_pair(a[j], bs, acc[j]);
            }
        }
    }
}

// Phi^T W for many tiles per wave (molecules beyond the LDS-resident
// density): groups of four tiles with compile-time accumulator indices; a
// group runs when any of its tiles is this wave's, and tiles past the last
// one repeat tile 0 into accumulators that are never written out.
template <int NW, int BP, int MAXT>
__device__ __forceinline__ void gemm_phit_w_pair_grouped(const unsigned int* __restrict__ Phi,
                                                         const unsigned int* __restrict__ Wt, int LDG, int NT,
                                                         int nj, int wave, int lane, f4_t (&acc)[MAXT])
{
    static_assert(MAXT % 4 == 0, "groups of four tiles");
    const int l16 = lane & 15, q = lane >> 4;
#pragma unroll
    for (int g0 = 0; g0 < MAXT; g0 += 4) {
        if (g0 < nj) {
            int pa[4], pb[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                int t = wave + (g0 + j) * NW;
                if (t >= NT * NT) t = 0;
                pa[j] = ((t / NT) * 16 + l16) * LDG + 4 * q;
                pb[j] = ((t % NT) * 16 + l16) * LDG + 4 * q;
            }
#pragma unroll
            for (int kk = 0; kk < BP; kk += 16) {
                u32x4_t a[4], bv[4];
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    a[j] = *(const u32x4_t*)(Phi + pa[j] + kk);
                    bv[j] = *(const u32x4_t*)(Wt + pb[j] + kk);
                }
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    u32x4_t bs;
#pragma unroll
                    for (int i = 0; i < 4; i++) bs[i] = pair_swap(bv[j][i]);
                    acc[g0 + j] = mfma_pair(a[j], bv[j], acc[g0 + j]);
                    acc[g0 + j] = mfma_pair(a[j], bs, acc[g0 + j]);
                }
            }
        }
    }
}

// PGL: the padded density is read from global memory (L2) instead of LDS,
// for molecules whose density does not fit next to the AO planes.
template <typename T, int BP, int NW, int MAXT, bool PGL = false>
__global__ __launch_bounds__(NW * 64) void xc_kernel(XcArgs g)
{
    constexpr int NTH = NW * 64;
    constexpr int PG = 64 / BP;       // point groups per wavefront (lane = point within a group)
    constexpr int NG = NW * PG;       // point groups per work group
    constexpr int GT = BP / 16;       // point tiles
    constexpr int LDG = xc_ldg(BP);
    static_assert(NW >= 3, "the functional's three parts run on three wavefronts");
    typedef typename Mfma<T>::V V;
    const XcItem it = g.items[blockIdx.x];
    const int m = it.mol;
    if (g.only_active && g.state[m].status != KS_MOL_ACTIVE) return;
    // SCF iterations use the grid of the molecule's stage; direct calls the main grid
    if (it.stage != (g.only_active ? g.state[m].stage : 0)) return;
    const MolDesc md = g.mol[m];
    const int N = md.nbf, NP = md.np, NT = NP >> 4, LDP = PGL ? NP : xc_ldp(NP), PL = NP * LDG;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l16 = lane & 15;
    const int gp = lane % BP, grp = wave * PG + lane / BP;   // point-per-lane view
    const int nj1 = (GT * NT - wave + NW - 1) / NW;          // X^T tiles of this wave
    const int nj2 = (NT * NT - wave + NW - 1) / NW;          // Phi^T W tiles of this wave

    extern __shared__ __align__(32) unsigned char smem_xc[];
    unsigned char* cur = smem_xc;
    auto take = [&](size_t bytes) {
        unsigned char* p = cur;
        cur += al32(bytes);
        return p;
    };
    double* pts = (double*)take(BP * 4 * sizeof(double));    // [BP][4]
    double* wsum = (double*)take(NW * sizeof(double));        // [NW]
    ShellLds<T> shl;
    shl.A = (double*)take((size_t)g.ns_max * 3 * sizeof(double));
    const int npm = g.npm;
    shl.ac = (T*)take((size_t)g.ns_max * 2 * kPrimMax * sizeof(T));
    T* coef = (T*)take(BP * 4 * sizeof(T));                   // [BP][4]: rho, grad rho
    T* fpart = (T*)take(BP * 9 * sizeof(T));                  // [3][BP][3]: e, v_rho, v_sigma per part
    T* rpart = (T*)take((size_t)NT * 4 * BP * sizeof(T));     // [NT][4][BP]
    constexpr bool kPair = sizeof(T) == 4;                    // FP32: Phi and W as bf16 pairs
    T* Pl = PGL ? (T*)((const T*)g.Pt + g.ptoff[m]) : (T*)take((size_t)NP * LDP * sizeof(T));   // [NP][LDP]
    T* Phi = (T*)take((size_t)(kPair ? 5 : 4) * PL * sizeof(T));   // 4 (FP32: 5) planes [NP][LDG]
    T* Wt = Phi + PL;                                         // W^T overwrites d/dx Phi
    unsigned int* Php = (unsigned int*)(Phi + 4 * PL);        // FP32: Phi as bf16 pairs
    shl.info = (int*)take((size_t)g.ns_max * sizeof(int));

    const T* __restrict__ Pt = (const T*)g.Pt + g.ptoff[m];
    const Shell* __restrict__ sh = g.shells + md.shell0;

    if constexpr (!PGL)
        for (int i = tid; i < NP * NP; i += NTH) Pl[(i / NP) * LDP + i % NP] = Pt[i];
    for (int i = tid; i < md.nshell; i += NTH) {
        const Shell& S = sh[i];
#pragma unroll
        for (int k = 0; k < 3; k++) shl.A[3 * i + k] = S.A[k];
        for (int k = 0; k < kPrimMax; k++) {
            const int h = k / kNPrim, j = k % kNPrim;
            shl.ac[2 * kPrimMax * i + 2 * kNPrim * h + j] = (T)S.a[k];
            shl.ac[2 * kPrimMax * i + 2 * kNPrim * h + kNPrim + j] = (T)S.c[k];
        }
        shl.info[i] = S.ao | (S.L << 16);
    }
    for (int i = tid; i < (kPair ? 5 : 4) * PL; i += NTH) Phi[i] = T(0);

    V acc[MAXT];
#pragma unroll
    for (int k = 0; k < MAXT; k++)
#pragma unroll
        for (int r = 0; r < 4; r++) acc[k][r] = T(0);

    double exc = 0.0, exc_c = 0.0;   // Neumaier pair of the functional lanes
    // points beyond the chunk sit far away with zero weight (all AO values vanish)
    const double far[3] = {sh[0].A[0] + 300.0, sh[0].A[1] + 300.0, sh[0].A[2] + 300.0};
    double nxt[4] = {far[0], far[1], far[2], 0.0};            // prefetched next point
    if (tid < BP && it.g0 + tid < it.g1) {
        const double* src = g.grid + 4 * (md.grid0 + it.g0 + tid);
        nxt[0] = src[0]; nxt[1] = src[1]; nxt[2] = src[2]; nxt[3] = src[3];
    }

    for (long g0 = it.g0; g0 < it.g1; g0 += BP) {
        __syncthreads();
        if (tid < BP) {
            pts[4 * tid] = nxt[0];
            pts[4 * tid + 1] = nxt[1];
            pts[4 * tid + 2] = nxt[2];
            pts[4 * tid + 3] = nxt[3];
            // issue the next sub-block's loads; they complete behind this one
            const long gn = g0 + BP + tid;
            if (gn < it.g1) {
                const double* src = g.grid + 4 * (md.grid0 + gn);
                nxt[0] = src[0]; nxt[1] = src[1]; nxt[2] = src[2]; nxt[3] = src[3];
            } else {
                nxt[0] = far[0]; nxt[1] = far[1]; nxt[2] = far[2]; nxt[3] = 0.0;
            }
        }
        __syncthreads();
        // AO values and gradients into the AO-major planes: lane = point,
        // each point group takes every NG-th shell (with one group per
        // wavefront the shell is uniform)
        {
            const double px = pts[4 * gp], py = pts[4 * gp + 1], pz = pts[4 * gp + 2];
            for (int s = grp; s < md.nshell; s += NG) {
                const T dx = (T)(px - shl.A[3 * s]), dy = (T)(py - shl.A[3 * s + 1]), dz = (T)(pz - shl.A[3 * s + 2]);
                const T r2 = dx * dx + dy * dy + dz * dz;
                const T* ac = shl.ac + 2 * kPrimMax * s;
                T R = T(0), dR = T(0);
                auto prim = [&](const T* q, int k) {   // q: a block of three exponents, three coefficients
                    const T ar = q[k] * r2;
                    if constexpr (sizeof(T) == 4) {
                        // the hardware exp2 flushes to 0 far below the FP32 range
                        const T e = q[kNPrim + k] * fast_exp(-ar);
                        R += e;
                        dR -= T(2) * q[k] * e;
                    } else if (ar < T(80)) {
                        const T e = q[kNPrim + k] * fast_exp(-ar);
                        R += e;
                        dR -= T(2) * q[k] * e;
                    }
                };
#pragma unroll
                for (int k = 0; k < kNPrim; k++) prim(ac, k);
                if (npm > kNPrim) {                              // 6-31G core shells
#pragma unroll
                    for (int k = 0; k < kNPrim; k++) prim(ac + 2 * kNPrim, k);
                }
                const int info = shl.info[s], mu = info & 0xffff;
                T* o = Phi + mu * LDG + gp;
                auto put_phi = [&](int off, T v) {
                    o[off] = v;
                    if constexpr (kPair) Php[(o - Phi) + off] = bf16_pair(v);
                };
                if ((info >> 16) == 0) {
                    put_phi(0, R);
                    o[PL] = dR * dx;
                    o[2 * PL] = dR * dy;
                    o[3 * PL] = dR * dz;
                } else {
                    const T d[3] = {dx, dy, dz};
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        put_phi(c * LDG, d[c] * R);
#pragma unroll
                        for (int k = 0; k < 3; k++)
                            o[(k + 1) * PL + c * LDG] = (k == c ? R : T(0)) + d[c] * d[k] * dR;
                    }
                }
            }
        }
        __syncthreads();
        // X^T = P Phi^T and the density partials, this wave's tiles,
        // dispatched once to a branch-free body with a compile-time tile
        // count.  The lane index passes through an empty asm so that the tile
        // addresses are formed here, per sub-block, instead of being hoisted
        // out of the loop for every case (which exhausts the registers).
        int lane_g = lane;
        asm volatile("" : "+v"(lane_g));
        switch (nj1) {
        case 1: gemm_x_rho<T, BP, NW, 1>(Pl, Phi, rpart, LDP, LDG, PL, NP, wave, lane_g); break;
        case 2: gemm_x_rho<T, BP, NW, 2>(Pl, Phi, rpart, LDP, LDG, PL, NP, wave, lane_g); break;
        case 3: gemm_x_rho<T, BP, NW, 3>(Pl, Phi, rpart, LDP, LDG, PL, NP, wave, lane_g); break;
        case 4: gemm_x_rho<T, BP, NW, 4>(Pl, Phi, rpart, LDP, LDG, PL, NP, wave, lane_g); break;
        case 5: gemm_x_rho<T, BP, NW, 5>(Pl, Phi, rpart, LDP, LDG, PL, NP, wave, lane_g); break;
        case 6: gemm_x_rho<T, BP, NW, 6>(Pl, Phi, rpart, LDP, LDG, PL, NP, wave, lane_g); break;
        default: break;
        }
        __syncthreads();
        // functional: wavefronts 0, 1, 2 evaluate the exchange, VWN and LYP
        // parts for every point of the sub-block (lane = point)
        if (wave < 3 && lane < BP) {
            const int gi = lane;
            T r = T(0), gx = T(0), gy = T(0), gz = T(0);
            for (int mt = 0; mt < NT; mt++) {
                const T* rp = rpart + mt * 4 * BP + gi;
                r += rp[0];
                gx += rp[BP];
                gy += rp[2 * BP];
                gz += rp[3 * BP];
            }
            gx *= T(2); gy *= T(2); gz *= T(2);
            if (wave == 0) {
                coef[4 * gi] = r; coef[4 * gi + 1] = gx; coef[4 * gi + 2] = gy; coef[4 * gi + 3] = gz;
            }
            const T w = (T)pts[4 * gi + 3];
            T e = T(0), vr = T(0), vs = T(0);
            if (r >= T(kRhoCut) && w != T(0)) {
                const T sg = gx * gx + gy * gy + gz * gz;
                if (wave == 0) b3lyp_exchange<T>(r, sg, e, vr, vs);
                else if (wave == 1) b3lyp_vwn<T>(r, g.vwn5, e, vr, vs);
                else b3lyp_lyp<T>(r, sg, e, vr, vs);
                const double we = (double)w * (double)e;
                const double tt = exc + we;
                if (fabs(exc) >= fabs(we)) exc_c += (exc - tt) + we; else exc_c += (we - tt) + exc;
                exc = tt;
            }
            T* fp = fpart + (wave * BP + gi) * 3;
            fp[0] = e; fp[1] = vr; fp[2] = vs;
        }
        __syncthreads();
        // W^T = c0 Phi + c . grad Phi in place of d/dx Phi, c0 = w v_rho / 2,
        // c = 2 w v_sigma grad rho; lane = point, each point group an AO range
        {
            const T w = (T)pts[4 * gp + 3];
            const T vr = fpart[gp * 3 + 1] + fpart[(BP + gp) * 3 + 1] + fpart[(2 * BP + gp) * 3 + 1];
            const T vs = fpart[gp * 3 + 2] + fpart[(BP + gp) * 3 + 2] + fpart[(2 * BP + gp) * 3 + 2];
            const T c0 = T(0.5) * w * vr, s2 = T(2) * w * vs;
            const T c1 = s2 * coef[4 * gp + 1], c2 = s2 * coef[4 * gp + 2], c3 = s2 * coef[4 * gp + 3];
            const int cw = (NP + NG - 1) / NG, m0 = grp * cw, m1 = min(NP, m0 + cw);
            // four AO rows at a time: all sixteen reads issued before the
            // first use, so their LDS latency overlaps
            int mu = m0;
            for (; mu + 4 <= m1; mu += 4) {
                T* o = Phi + mu * LDG + gp;
                T v[4][4];
#pragma unroll
                for (int r = 0; r < 4; r++)
#pragma unroll
                    for (int k = 0; k < 4; k++) v[r][k] = o[r * LDG + k * PL];
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const T wv = c0 * v[r][0] + c1 * v[r][1] + c2 * v[r][2] + c3 * v[r][3];
                    if constexpr (kPair) *(unsigned int*)(o + r * LDG + PL) = bf16_pair(wv);
                    else o[r * LDG + PL] = wv;
                }
            }
            for (; mu < m1; mu++) {
                T* o = Phi + mu * LDG + gp;
                const T wv = c0 * o[0] + c1 * o[PL] + c2 * o[2 * PL] + c3 * o[3 * PL];
                if constexpr (kPair) *(unsigned int*)(o + PL) = bf16_pair(wv);
                else o[PL] = wv;
            }
        }
        __syncthreads();
        // A += Phi^T W   (NP x BP) . (BP x NP), this wave's tiles
        lane_g = lane;
        asm volatile("" : "+v"(lane_g));
        if constexpr (kPair && MAXT > 9) {
            gemm_phit_w_pair_grouped<NW, BP, MAXT>(Php, (const unsigned int*)Wt, LDG, NT, nj2, wave, lane_g, acc);
        } else if constexpr (kPair) {
            const unsigned int* Pw = Php;
            const unsigned int* Ww = (const unsigned int*)Wt;
            switch (nj2) {
            case 1: gemm_phit_w_pair<NW, BP, MAXT, 1>(Pw, Ww, LDG, NT, wave, lane_g, acc); break;
            case 2: gemm_phit_w_pair<NW, BP, MAXT, 2>(Pw, Ww, LDG, NT, wave, lane_g, acc); break;
            case 3: gemm_phit_w_pair<NW, BP, MAXT, 3>(Pw, Ww, LDG, NT, wave, lane_g, acc); break;
            case 4: gemm_phit_w_pair<NW, BP, MAXT, 4>(Pw, Ww, LDG, NT, wave, lane_g, acc); break;
            case 5: gemm_phit_w_pair<NW, BP, MAXT, 5>(Pw, Ww, LDG, NT, wave, lane_g, acc); break;
            case 6: gemm_phit_w_pair<NW, BP, MAXT, 6>(Pw, Ww, LDG, NT, wave, lane_g, acc); break;
            case 7: gemm_phit_w_pair<NW, BP, MAXT, 7>(Pw, Ww, LDG, NT, wave, lane_g, acc); break;
            case 8: gemm_phit_w_pair<NW, BP, MAXT, 8>(Pw, Ww, LDG, NT, wave, lane_g, acc); break;
            case 9: gemm_phit_w_pair<NW, BP, MAXT, 9>(Pw, Ww, LDG, NT, wave, lane_g, acc); break;
            default: break;
            }
        } else
        switch (nj2) {
        case 1: gemm_phit_w<T, NW, BP, MAXT, 1>(Phi, Wt, LDG, NT, wave, lane_g, acc); break;
        case 2: gemm_phit_w<T, NW, BP, MAXT, 2>(Phi, Wt, LDG, NT, wave, lane_g, acc); break;
        case 3: gemm_phit_w<T, NW, BP, MAXT, 3>(Phi, Wt, LDG, NT, wave, lane_g, acc); break;
        case 4: gemm_phit_w<T, NW, BP, MAXT, 4>(Phi, Wt, LDG, NT, wave, lane_g, acc); break;
        case 5: gemm_phit_w<T, NW, BP, MAXT, 5>(Phi, Wt, LDG, NT, wave, lane_g, acc); break;
        case 6: gemm_phit_w<T, NW, BP, MAXT, 6>(Phi, Wt, LDG, NT, wave, lane_g, acc); break;
        case 7: gemm_phit_w<T, NW, BP, MAXT, 7>(Phi, Wt, LDG, NT, wave, lane_g, acc); break;
        case 8: gemm_phit_w<T, NW, BP, MAXT, 8>(Phi, Wt, LDG, NT, wave, lane_g, acc); break;
        case 9: gemm_phit_w<T, NW, BP, MAXT, 9>(Phi, Wt, LDG, NT, wave, lane_g, acc); break;
        default: break;
        }
    }
    // write this chunk's A and E_xc
    T* out = (T*)g.part + (size_t)blockIdx.x * g.part_stride;
#pragma unroll
    for (int k = 0; k < MAXT; k++) {
        const int t = wave + k * NW;
        if (t < NT * NT) {
            const int it2 = t / NT, jt = t % NT;
#pragma unroll
            for (int r = 0; r < 4; r++) out[(it2 * 16 + Mfma<T>::row(lane, r)) * NP + jt * 16 + l16] = acc[k][r];
        }
    }
    double tot = exc + exc_c;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) tot += __shfl_xor(tot, o, 64);
    __syncthreads();
    if (lane == 0) wsum[wave] = tot;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < NW; w++) s += wsum[w];
        g.part_exc[blockIdx.x] = s;
    }
}

// V_XC = sum over the molecule's chunks of (A + A^T); E_XC = sum of chunk sums.
template <typename T>
__global__ void xc_reduce_kernel(const MolDesc* __restrict__ mols, const MolState* __restrict__ state,
                                 const int* __restrict__ first, const int* __restrict__ first_c,
                                 const T* __restrict__ part, long stride,
                                 const double* __restrict__ part_exc, int only_active, double* __restrict__ V,
                                 double* __restrict__ exc)
{
    const int m = blockIdx.y;
    if (only_active && state[m].status != KS_MOL_ACTIVE) return;
    const MolDesc md = mols[m];
    const int N = md.nbf, NP = md.np;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int* fr = only_active && state[m].stage ? first_c : first;
    const int i0 = fr[m], i1 = fr[m + 1];
    if (t == 0) {
        double s = 0.0, c = 0.0;
        for (int i = i0; i < i1; i++) {
            const double x = part_exc[i], tt = s + x;
            if (fabs(s) >= fabs(x)) c += (s - tt) + x; else c += (x - tt) + s;
            s = tt;
        }
        exc[m] = s + c;
    }
    if (t >= N * N) return;
    const int mu = t / N, nu = t % N;
    double v = 0.0;
    for (int i = i0; i < i1; i++) {
        const T* p = part + (size_t)i * stride;
        v += (double)p[mu * NP + nu] + (double)p[nu * NP + mu];
    }
    V[md.mat0 + t] = v;
}

// Launch shape of the batch: the options' xc_points / xc_waves when given
// (and the LDS budget allows), else the measured default: 64-point
// sub-blocks for FP32 and 32 for FP64 with 8-wave groups, halved until the
// LDS budget (160 KB) holds.
static bool xc_shape_ok(int bp, int nw)
{
    return (bp == 16 || bp == 32 || bp == 64) && (nw == 4 || nw == 8 || nw == 16);
}

XcShape xc_shape(const ks_batch* b)
{
    XcShape s;
    const bool f32 = b->opt.prec == KS_MIXED;
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    s.bp = f32 ? 64 : 32;
    s.nw = 8;
    if (b->opt.xc_points > 0 || b->opt.xc_waves > 0) {
        const int bp = b->opt.xc_points > 0 ? b->opt.xc_points : s.bp;
        const int nw = b->opt.xc_waves > 0 ? b->opt.xc_waves : s.nw;
        if (xc_shape_ok(bp, nw)) { s.bp = bp; s.nw = nw; }
    }
    if (f32 && b->max_np > 96) {
        // beyond the LDS-resident density: P from L2, 16-point sub-blocks,
        // 8 waves (the Phi^T W tiles of up to 224 functions fit their registers)
        s.bp = 16;
        s.nw = 8;
        s.pglobal = true;
        s.lds = xc_lds_bytes_for(es, s.bp, s.nw, b->max_np, b->max_nshell, true);
        return s;
    }
    while (s.bp > 16 && xc_lds_bytes_for(es, s.bp, s.nw, b->max_np, b->max_nshell) > kLdsMax) s.bp /= 2;
    s.lds = xc_lds_bytes_for(es, s.bp, s.nw, b->max_np, b->max_nshell);
    return s;
}

int xc_block_points(const ks_batch* b) { return xc_shape(b).bp; }

template <typename T, int BP, int NW, int MAXT, bool PGL = false>
static ks_status launch_xc_shape(ks_batch* b, const XcArgs& g, size_t lds)
{
    KS_HIP(hipFuncSetAttribute((const void*)xc_kernel<T, BP, NW, MAXT, PGL>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    KTimer tx(b, "xc");
    hipLaunchKernelGGL((xc_kernel<T, BP, NW, MAXT, PGL>), dim3((unsigned)b->xc_items.size()), dim3(NW * 64), lds,
                       b->stream, g);
    KS_HIP(hipGetLastError());
    return KS_OK;
}

template <typename T>
static ks_status run_xc(ks_batch* b, const double* P, double* V, bool only_active)
{
    int maxnp2 = 0;
    for (auto& m : b->mol) maxnp2 = std::max(maxnp2, m.np * m.np);
    {
        KTimer tp(b, "xc_pad");
        hipLaunchKernelGGL(pad_density_kernel<T>, dim3((maxnp2 + 255) / 256, b->n_mol), dim3(256), 0, b->stream,
                           b->d_mol, b->d_state, b->d_ptoff, P, (T*)b->d_Pt, (int)only_active);
    }
    KS_HIP(hipGetLastError());
    XcArgs g;
    g.mol = b->d_mol;
    g.state = b->d_state;
    g.items = b->d_xc_items;
    g.shells = b->d_shells;
    g.grid = b->d_grid;
    g.Pt = b->d_Pt;
    g.ptoff = b->d_ptoff;
    g.part = b->d_xc_part;
    g.part_exc = b->d_xc_exc;
    g.part_stride = (long)b->max_np * b->max_np;
    g.ns_max = b->max_nshell;
    g.npm = b->pp == kPrimPairMax ? kPrimMax : kNPrim;
    g.vwn5 = b->opt.xc == KS_XC_B3LYP5;
    g.only_active = only_active;
    const XcShape s = xc_shape(b);
    const bool big = b->max_np > 80;     // 6 x 6 tiles of 16
    ks_status st;
    if (s.pglobal) {
        if constexpr (sizeof(T) == 4) {
            if (b->max_np > 224) {
                set_error("XC: %d padded basis functions exceed the 224 of the large-molecule kernel", b->max_np);
                return KS_EUNSUPPORTED;
            }
            st = launch_xc_shape<T, 16, 8, 28, true>(b, g, s.lds);
        } else {
            set_error("XC: FP64 molecules beyond the LDS-resident density are not supported");
            return KS_EUNSUPPORTED;
        }
    } else if (s.nw == 16) {
        if (s.bp == 64) st = big ? launch_xc_shape<T, 64, 16, 3>(b, g, s.lds) : launch_xc_shape<T, 64, 16, 2>(b, g, s.lds);
        else if (s.bp == 32) st = big ? launch_xc_shape<T, 32, 16, 3>(b, g, s.lds) : launch_xc_shape<T, 32, 16, 2>(b, g, s.lds);
        else st = big ? launch_xc_shape<T, 16, 16, 3>(b, g, s.lds) : launch_xc_shape<T, 16, 16, 2>(b, g, s.lds);
    } else if (s.nw == 8) {
        if (s.bp == 64) st = big ? launch_xc_shape<T, 64, 8, 5>(b, g, s.lds) : launch_xc_shape<T, 64, 8, 4>(b, g, s.lds);
        else if (s.bp == 32) st = big ? launch_xc_shape<T, 32, 8, 5>(b, g, s.lds) : launch_xc_shape<T, 32, 8, 4>(b, g, s.lds);
        else st = big ? launch_xc_shape<T, 16, 8, 5>(b, g, s.lds) : launch_xc_shape<T, 16, 8, 4>(b, g, s.lds);
    } else {
        if (s.bp == 64) st = big ? launch_xc_shape<T, 64, 4, 9>(b, g, s.lds) : launch_xc_shape<T, 64, 4, 7>(b, g, s.lds);
        else if (s.bp == 32) st = big ? launch_xc_shape<T, 32, 4, 9>(b, g, s.lds) : launch_xc_shape<T, 32, 4, 7>(b, g, s.lds);
        else st = big ? launch_xc_shape<T, 16, 4, 9>(b, g, s.lds) : launch_xc_shape<T, 16, 4, 7>(b, g, s.lds);
    }
    if (st) return st;
    int maxnn = 0;
    for (auto& m : b->mol) maxnn = std::max(maxnn, m.nbf * m.nbf);
    KTimer tr(b, "xc_reduce");
    hipLaunchKernelGGL(xc_reduce_kernel<T>, dim3((maxnn + 255) / 256, b->n_mol), dim3(256), 0, b->stream, b->d_mol,
                       b->d_state, b->d_xc_first, b->d_xc_first_c, (const T*)b->d_xc_part, g.part_stride, b->d_xc_exc,
                       (int)only_active, V, b->d_exc);
    KS_HIP(hipGetLastError());
    return KS_OK;
}

ks_status launch_xc(ks_batch* b, const double* P, double* V, bool only_active)
{
    ks_status st = grid_wait(b);
    if (st) return st;
    if (b->opt.prec == KS_MIXED) return run_xc<float>(b, P, V, only_active);
    return run_xc<double>(b, P, V, only_active);
}

size_t xc_lds_bytes(const ks_batch* b) { return xc_shape(b).lds; }

}  // namespace ks
