// Internal data layout of libks.so (shared by the host driver and the HIP
// kernels; nothing here is part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ks.h"

namespace ks {

// Largest molecule (basis functions) of the mixed path: up to 96 every
// kernel keeps its per-molecule matrices in LDS; above that J/K accumulate
// in global memory, XC reads the density from L2 and the eigensolver and
// the N x N products work in global memory.  The FP64 path stops at 82
// (its XC accumulators for larger molecules exceed the registers).
constexpr int kMaxNbf = 224;
constexpr int kNPrim = 3;       // STO-3G: three primitives per shell
constexpr int kNPrimPair = kNPrim * kNPrim;
constexpr int kPrimMax = 6;     // 6-31G: up to six (the core s shell)
constexpr int kPrimPairMax = kPrimMax * kPrimMax;
constexpr int kMaxDiis = 8;
constexpr double kPi = 3.14159265358979323846;
constexpr double kBohrAng = 0.52917721092;
constexpr double kRhoCut = 1e-12;      // points below this density carry no XC
// Convergence thresholds are raised to these in the mixed path: the FP32
// Fock matrix carries ~1e-6 noise, below which FP32 cannot resolve changes.
constexpr double kMixedETol = 1e-6;
constexpr double kMixedCommTol = 1e-5;
// Coarse start grid (options coarse_*): a molecule moves to the main grid
// once these hold on the coarse grid, or after kCoarseMaxIter iterations.
constexpr double kCoarseETol = 1e-4;
constexpr double kCoarseCommTol = 1e-3;
constexpr int kCoarseMaxIter = 12;
// Primitive ERI screening: a primitive quartet is skipped when its Gaussian
// prefactor 2 pi^(5/2) K_ab K_cd / (p q sqrt(p + q)) is below the cut (far
// below the FP64 parity tolerance, resp. the FP32 storage rounding).  kQMin
// bounds p, q from below (twice the smallest STO-3G exponent, 0.1689 of H)
// and kKMax bounds |K| from above (the largest is 26, F 1s with itself).
constexpr double kEriCutFp64 = 1e-20;
constexpr double kEriCutMixed = 1e-14;
constexpr double kQMin = 0.3;
constexpr double kKMax = 30.0;

// Boys-function table: F_m(T_i), T_i = i * kBoysDT, i < kBoysNT, m < kBoysM.
constexpr double kBoysDT = 0.05;
constexpr double kBoysTMax = 36.0;
constexpr int kBoysNT = 722;
constexpr int kBoysM = 12;
// Row table for the ERI kernels, small enough for LDS: for each total
// angular momentum L <= 4, row i holds F_L..F_{L+7} at T_i = i * kBoysDTR
// (eight values: a 64-byte row read with four 16-byte loads).
constexpr double kBoysDTR = 0.1;
constexpr int kBoysNTR = 361;
constexpr int kBoysKR = 8;
constexpr int kBoysLR = 5;

// A contracted shell: 2s and 2p of a heavy atom are separate shells that
// share exponents.  c[] already holds contraction x primitive normalisation
// x contracted renormalisation.
struct Shell {
    double A[3];
    double a[kPrimMax];
    double c[kPrimMax];
    double occ; // initial-guess occupation per function of the shell
    int L;      // 0 = s, 1 = p
    int ao;     // first AO index inside its molecule
    int atom;   // atom index inside its molecule
    int np;     // primitives (3 in STO-3G; 6, 3 or 1 in 6-31G)
};

// Primitive-pair data of a shell pair (McMurchie-Davidson Gaussian product):
// p = a + b, P = (a A + b B)/p, K = c_a c_b exp(-a b/p |A-B|^2) and 1/p,
// stored field-major over the pairs of a pair class (see pair_kernel).
constexpr int kPairFields = 6;   // p, Px, Py, Pz, K, 1/p

// Shell pair (global shell indices); sa carries the higher angular momentum.
struct Pair {
    int sa, sb;
};

// Quartet classes (bra pair class, ket pair class), pair classes ss=0, ps=1, pp=2.
constexpr int kNClass = 6;
__host__ __device__ constexpr int class_bra(int c) { return c == 0 ? 0 : (c <= 2 ? 1 : 2); }
__host__ __device__ constexpr int class_ket(int c) { return (c == 0 || c == 1 || c == 3) ? 0 : (c == 2 || c == 4 ? 1 : 2); }
__host__ __device__ constexpr bool class_tri(int c) { return c == 0 || c == 2 || c == 5; }
__host__ __device__ constexpr int class_ncomp(int c)
{
    return c == 0 ? 1 : (c == 1 ? 3 : (c == 2 || c == 3 ? 9 : (c == 4 ? 27 : 81)));
}

struct MolDesc {
    int natom, nbf, nocc, nshell;
    int atom0, shell0;      // offsets into the batch atom / shell arrays
    int np;                 // nbf rounded up to 16
    int ao0;                // first AO of this molecule in the batch AO table
    long mat0;              // element offset of this molecule's N x N blocks
    long grid0;             // first grid point
    long ngrid;
    long gridc0, ngridc;    // the coarse start grid (ngridc = 0 without one)
    int pair0[3];           // first pair of each pair class in the class lists
    int npair[3];
    long q0[kNClass];       // first quartet of each class in the batch-global class list
    long nq[kNClass];
    double enuc;
};

// Per-molecule SCF state kept on the device.
struct MolState {
    int status;             // KS_MOL_*
    int iter;
    int nhist;              // DIIS vectors held
    int head;               // DIIS ring position
    int final_;             // set when this iteration's F is the last one
    int stage;              // 1 while XC runs on the coarse start grid, then 0
    int it_full;            // first iteration on the main grid (convergence is tested after it)
    int pad;
    double E, Eprev, err;
    double dE;              // E - E of the previous iteration, as last tested
    double Eterms[6];
    double B[kMaxDiis * kMaxDiis];   // DIIS overlaps of the held error vectors
};

// XC work item: a contiguous range of one molecule's grid points.
struct XcItem {
    int mol;
    int stage;              // 0: main grid, 1: coarse start grid
    long g0, g1;            // points md.grid0 + g0 .. md.grid0 + g1 - 1 of the batch grid
};

struct JkItem {
    int mol, chunk, nchunk, pad;
};

}  // namespace ks

// ---------------------------------------------------------------------------
// host-side batch
// ---------------------------------------------------------------------------
struct ks_batch {
    ks_options opt;
    hipStream_t stream = nullptr;
    // The grid and Becke weights are built on a second stream while the ERIs
    // run on the batch stream; the batch stream waits on ev_grid before the
    // first use of the grid.
    hipStream_t aux = nullptr;
    hipEvent_t ev_main = nullptr, ev_grid = nullptr;
    bool grid_pending = false;
    hipGraphExec_t gexec = nullptr; // captured SCF iteration (options.graphs)
    int n_mol = 0;
    int max_np = 0;
    int max_nshell = 0;
    double a0 = 0.2;
    int pp = ks::kNPrimPair;        // primitive pairs per shell pair in the pair tables (9 STO-3G, 36 6-31G)
    std::vector<ks::MolDesc> mol;
    std::vector<ks::Shell> shells;
    std::vector<int> Z;
    std::vector<double> R;          // bohr
    long nmat = 0;                  // sum nbf^2
    long ngrid = 0;
    long npairs[3] = {0, 0, 0};
    long nq[ks::kNClass] = {0, 0, 0, 0, 0, 0};
    long nprimq = 0;

    // device memory (owned)
    std::vector<void*> allocs;
    size_t alloc_bytes = 0;         // device bytes held by this batch
    ks::MolDesc* d_mol = nullptr;
    ks::MolState* d_state = nullptr;
    ks::Shell* d_shells = nullptr;
    int2* d_aoinfo = nullptr;       // per batch AO: (global shell, component 0..2)
    double* d_R = nullptr;          // atom positions (bohr)
    double* d_Zc = nullptr;         // atom charges
    ks::Pair* d_pairs[3] = {nullptr, nullptr, nullptr};
    int2* d_pair_ao[3] = {nullptr, nullptr, nullptr};  // per pair: (AO of sa | (sa == sb) << 16, AO of sb)
    double* d_pp[3] = {nullptr, nullptr, nullptr};   // [5][9][npair] primitive-pair tables
    double* d_Q[3] = {nullptr, nullptr, nullptr};    // Schwarz factors max sqrt|(ab|ab)| per pair
    bool schwarz_done = false;
    bool pairs_sorted = false;      // pairs in decreasing Schwarz order (integral-direct builds)
    long* d_qoff[ks::kNClass] = {};  // prefix over molecules (n_mol + 1)
    void* d_eri[ks::kNClass] = {};   // component-major, FP64 or FP32
    double* d_boys = nullptr;
    double* d_boys_rows = nullptr;  // [kBoysLR][kBoysNTR][kBoysKR]
    float* d_boys_f = nullptr;
    double* d_radial = nullptr;     // r_i, w_i (n_rad each)
    double* d_ang = nullptr;        // cos theta_j, w_j (n_theta each)
    double* d_grid = nullptr;       // [ngrid + ngridc][4]: main grids, then the coarse start grids
    bool coarse = false;            // coarse start grid in use (options coarse_*)
    long ngridc = 0;
    double* d_radial_c = nullptr;   // coarse grid rules
    double* d_ang_c = nullptr;
    // matrices (nmat doubles each)
    double *d_S = nullptr, *d_T = nullptr, *d_V = nullptr, *d_H = nullptr, *d_X = nullptr;
    double *d_F = nullptr, *d_P = nullptr, *d_J = nullptr, *d_K = nullptr, *d_Vxc = nullptr;
    double *d_Fp = nullptr, *d_C = nullptr, *d_eps = nullptr, *d_work = nullptr;
    double *d_Fh = nullptr, *d_Eh = nullptr;    // DIIS history (diis_space * nmat each)
    double* d_Pprev = nullptr;      // density the resident J, K were built from (mixed path)
    double* d_Cp = nullptr;         // previous iteration's eigenvectors of F' (eigensolver warm start)
    int* d_have_warm = nullptr;     // [n_mol] d_Cp holds vectors for this molecule
    void* d_Pt = nullptr;           // padded density in the XC compute type (np^2 per molecule)
    long* d_ptoff = nullptr;        // offsets of d_Pt blocks
    long npt_total = 0;
    // J/K work
    std::vector<ks::JkItem> jk_items;
    ks::JkItem* d_jk_items = nullptr;
    void* d_jk_part = nullptr;      // [items][2][max_np^2]
    // XC work
    std::vector<ks::XcItem> xc_items;
    ks::XcItem* d_xc_items = nullptr;
    int* d_xc_first = nullptr;      // [n_mol + 1] first XC item of each molecule
    int* d_xc_first_c = nullptr;    // [n_mol + 1] first coarse-grid XC item of each molecule
    void* d_xc_part = nullptr;      // [items][np^2 max]
    double* d_xc_exc = nullptr;     // [items]
    double* d_exc = nullptr;        // [n_mol]
    double* d_eterms = nullptr;     // [n_mol][6] energy terms of fock_build
    int* d_nactive = nullptr;
    int* h_nactive = nullptr;       // pinned

    bool setup_done = false, eri_done = false, guess_done = false;
    int iter = 0;

    bool timing = false;
    std::vector<std::string> tnames;
    std::vector<double> tms;        // per name: total ms, launches
    struct Pending { int name; hipEvent_t e0, e1; };
    std::vector<Pending> pending;   // events not yet read back
};
