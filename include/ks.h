/*
 * ks.h -- C ABI of libks.so: restricted Kohn-Sham (B3LYP / STO-3G) Fock builds
 * and SCF solves for batches of molecules on one MI355X (gfx950).
 *
 * The method is the one of arxiv 2311.01135, section 3.1 ("DFT Primer"): the
 * inputs are atomic positions and atomic numbers; iteration 0 precomputes
 * V, T, S and the two-electron integrals I and initialises C; each iteration
 * forms rho = C D C^T (D = 2 on the N_e/2 lowest orbitals), V_XC(rho),
 * J_kl = sum_ij I_ijkl rho_ij and K_il = -1/2 sum_jk I_ijkl rho_jk, and
 * solves [V + T + J + K + V_XC] C = S C eps; the HL gap is read from eps.
 * Section 3.2 fixes B3LYP, float32 as the working precision, the 8-fold ERI
 * symmetry and the J/K digestion of the packed integrals; section 5
 * ("Recomputation", "Multiple IPUs") the integral-direct and split variants.
 *
 * Conventions (all entry points):
 *   - Every function returns ks_status (0 = KS_OK, < 0 = error) and never
 *     throws across the ABI; ks_last_error() returns a thread-local message
 *     for the last failing call on this thread.
 *   - Positions are in Angstrom and converted once with 0.52917721092 A/bohr;
 *     energies are in Hartree.
 *   - AO order is atom-major; per H atom 1s; per C/N/O/F atom 1s, 2s, 2px,
 *     2py, 2pz.  Contracted functions are normalised (S_mm = 1).
 *   - Per-molecule N x N matrices passed as device pointers are concatenated
 *     row-major blocks in molecule order: molecule m starts at element
 *     sum_{m' < m} nbf(m')^2.  ks_batch_sizes() gives nbf(m).
 *   - Device pointers are borrowed, FP64, and used in stream order on the
 *     stream given to ks_batch_create (NULL = the null stream).  Host output
 *     buffers are caller-allocated.  The library owns all other device
 *     memory, which ks_batch_destroy releases.
 *   - One handle is used by one host thread at a time.
 */
#ifndef KS_H
#define KS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KS_OK = 0,
    KS_EINVAL = -1,         /* bad argument or molecule (see ks_last_error) */
    KS_ENOMEM = -2,         /* device allocation or HBM budget */
    KS_EDEVICE = -3,        /* HIP runtime error */
    KS_ENOCONV = -4,        /* reserved */
    KS_EUNSUPPORTED = -5,   /* option or size outside what is built */
    KS_ESTATE = -6          /* call out of order (e.g. jk_build before eri_build) */
} ks_status;

typedef enum {
    KS_XC_HF = 0,           /* Hartree-Fock: no XC, full exchange */
    KS_XC_B3LYP = 1,        /* 0.08 Slater + 0.72 B88 + 0.19 VWN(RPA) + 0.81 LYP + 0.20 HF */
    KS_XC_B3LYP5 = 2        /* the same with VWN5 */
} ks_xc;

typedef enum {
    KS_FP64 = 0,            /* every step in FP64 */
    KS_MIXED = 1            /* stored ERIs in FP32 (evaluated in FP64, rounded once
                               on store); J/K digests the FP32 integrals against the
                               FP64 density with FP64 accumulation (FP32 above 82
                               functions); XC in FP32 (AO values, X = Phi P on FP32
                               MFMAs, the functional) with Phi^T W on bf16 split pairs
                               (operands within 2^-17 relative, FP32 accumulation)
                               and E_XC summed per point in FP64; Loewdin,
                               eigensolve, DIIS, Fock assembly and the energy sum in
                               FP64 */
} ks_precision;

/* per-molecule status (ks_get_result) */
#define KS_MOL_ACTIVE 0
#define KS_MOL_CONVERGED 1
#define KS_MOL_MAXITER 2
#define KS_MOL_DIVERGED 3

typedef struct {
    int xc;                 /* ks_xc */
    int prec;               /* ks_precision */
    int n_rad, n_theta, n_phi;   /* grid per atom: Treutler radial x Gauss-Legendre(cos theta) x trapezoid(phi) */
    double e_tol;           /* |E_k - E_{k-1}| threshold (Hartree) */
    double comm_tol;        /* max |X^T (FPS - SPF) X| threshold */
    int max_iter;
    int diis_space;         /* <= 8 */
    int jk_chunks;          /* work groups per molecule for J/K (0 = automatic) */
    int xc_chunks;          /* work groups per molecule for XC (0 = automatic) */
    int guess;              /* initial density: KS_GUESS_ATOM or KS_GUESS_CORE */
    int xc_points;          /* XC launch shape: grid points per sub-block, 16/32/64 (0 = tuned default) */
    int xc_waves;           /* XC launch shape: wavefronts per work group, 4, 8 or 16 (0 = tuned default) */
    int direct;             /* 1: integral-direct SCF (ERIs recomputed in every J/K build, never stored) */
    double schwarz_tol;     /* Schwarz screening: stored path, skip quartets with Q_ab Q_cd below it (0 = off);
                               direct path, skip quartets with Q_ab Q_cd max|dP| below it (0 = 1e-12 FP64,
                               1e-10 mixed) */
    int basis;              /* KS_BASIS_STO3G (H, C, N, O, F) or KS_BASIS_631G (H, C, N, O) */
    int graphs;             /* 1: from the second SCF iteration on, scf_step / scf_solve replay one
                               iteration's launches as a captured HIP graph (needs a non-NULL stream at
                               ks_batch_create; ignored while kernel timing is on).  0 = plain launches */
    int coarse_rad, coarse_theta, coarse_phi;
                            /* optional coarse-grid start (all three > 0 to enable, 0 = off; the paper,
                               section 3.1, evaluates V_XC on one grid throughout, and this start only
                               changes the path to the same converged result): every
                               molecule begins its SCF with XC on a coarse_rad x coarse_theta x coarse_phi
                               grid per atom and moves to the main grid once |dE| < 1e-4 Ha and the
                               commutator < 1e-3 there (or after 12 iterations).  DIIS keeps its history
                               across the move; convergence is only tested on the main grid, from its
                               second iteration, so results are those of the main grid.  Each count at
                               most the main grid's.  Measured best for 9-11-heavy-atom molecules on the
                               50 x 12 x 24 grid: 25 x 8 x 16. */
    int eri_threads[6];     /* ERI launch shape per quartet class ((ss|ss), (ps|ss), (ps|ps), (pp|ss),
                               (pp|ps), (pp|pp)): work-group size 64, 128 or 256 (0 = 128) */
    int eri_unroll[6];      /* the same classes: ket primitive pairs evaluated per unrolled group, 3 or
                               9 (0 = 3; STO-3G; 6-31G loops over each shell pair's real pairs) */
} ks_options;

/* Initial density.  The paper only says C_1 is initialised (section 3.1).
 * KS_GUESS_ATOM: diagonal superposition of neutral-atom occupations (H 1s 1;
 * C/N/O/F 1s 2, 2s 2, 2p (Z-4)/3 each) scaled to the electron count, used as
 * the first density.  KS_GUESS_CORE: orbitals of the core Hamiltonian. */
#define KS_GUESS_ATOM 0
#define KS_GUESS_CORE 1

/* Basis sets (paper section 4: STO-3G for the generated data; 6-31G is the
 * larger basis it also supports).  6-31G: six-primitive core s, 3 + 1 split
 * valence with sp shells sharing exponents (9 functions per C/N/O, 2 per
 * H); the initial density splits each atom's valence occupation evenly over
 * the inner and outer shells. */
#define KS_BASIS_STO3G 0
#define KS_BASIS_631G 1

/* Fills *o with the defaults: B3LYP, FP64, 50 x 12 x 24 grid, e_tol 1e-9,
 * comm_tol 1e-7, max_iter 100, diis_space 8, automatic chunking, atomic
 * guess.  With KS_MIXED the library raises e_tol to at least 1e-6 and
 * comm_tol to at least 1e-5, the resolution of an FP32 Fock matrix. */
void ks_default_options(ks_options* o);

typedef struct ks_batch ks_batch;

/* Creates a batch of n_mol molecules (paper section 3.1: positions and atomic
 * numbers in).  n_atoms[n_mol]; Z and xyz_angstrom are concatenated over the
 * molecules (3 coordinates per atom); charge[n_mol] or NULL for neutral.
 * stream is a hipStream_t or NULL.  Host prep runs here and the basis,
 * pair tables and grid nodes are uploaded; no integrals are computed yet.
 * Errors: KS_EINVAL for an odd electron count, an element outside
 * {H, C, N, O, F}, non-finite coordinates or atoms closer than 0.1 bohr;
 * KS_EUNSUPPORTED for a molecule with more than 82 basis functions in
 * KS_FP64 or 224 in KS_MIXED (up to 96 the per-molecule matrices of every
 * kernel sit in LDS; larger mixed-path molecules use global-memory J/K
 * accumulation, an L2-resident density in XC and a global-memory
 * eigensolver, at lower speed);
 * KS_ENOMEM / KS_EDEVICE for allocation or runtime failures.  On error *out
 * is NULL and nothing is leaked. */
ks_status ks_batch_create(const ks_options* opt, int n_mol, const int* n_atoms, const int* Z,
                          const double* xyz_angstrom, const int* charge, void* stream,
                          ks_batch** out);

/* Sizes of molecule mol: basis functions, occupied orbitals, packed unique
 * ERIs nbf2*(nbf2+1)/2 with nbf2 = nbf*(nbf+1)/2, and grid points.  Any
 * output pointer may be NULL. */
ks_status ks_batch_sizes(const ks_batch* b, int mol, int* nbf, int* nocc, long* n_eri, long* n_grid);

/* Number of unique contracted shell quartets of the whole batch (2s and 2p
 * counted as separate shells), i.e. the ERI work items of eri_build. */
ks_status ks_batch_quartets(const ks_batch* b, long* n_quartets, long* n_primitive_quartets);

/* One-electron integrals S, T, V (paper section 3.1, iteration 0), Loewdin
 * X = S^-1/2, the grid with Becke weights and the core-Hamiltonian guess.
 * Called by scf_solve/scf_step when needed; explicit calls are for parity
 * tests.  KS_EINVAL if a molecule's overlap has an eigenvalue below 1e-8. */
ks_status ks_setup(ks_batch* b);

/* Electron-repulsion integrals over the unique shell quartets (8-fold
 * symmetry, paper section 3.2 "Libcint"), resident on the device in FP64
 * (KS_FP64) or FP32 (KS_MIXED). */
ks_status eri_build(ks_batch* b);

/* J and K of every molecule for the densities P_dev (paper section 3.1:
 * J_kl = sum_ij I_ijkl P_ij, and K_il = sum_jk I_ijkl P_jk, i.e. the
 * paper's K without its -1/2).  P_dev, J_dev, K_dev: device FP64 blocks as
 * in the conventions.  KS_ESTATE before eri_build. */
ks_status jk_build(ks_batch* b, const void* P_dev, void* J_dev, void* K_dev);

/* V_XC and E_XC for the densities P_dev on the Becke grid (B3LYP; zero for
 * KS_XC_HF).  Vxc_dev: device FP64 blocks; Exc_host[n_mol] host doubles. */
ks_status xc_build(ks_batch* b, const void* P_dev, void* Vxc_dev, double* Exc_host);

/* Fock matrices F = H + J - (a0/2) K + V_XC for P_dev (or the resident
 * density when P_dev is NULL) and the energy terms, host E_terms[n_mol*6] =
 * {tr PH, 1/2 tr PJ, -a0/4 tr PK, E_xc, E_nn, E_total}.  F_dev may be NULL. */
ks_status fock_build(ks_batch* b, const void* P_dev, void* F_dev, double* E_terms);

/* One SCF iteration for every active molecule (Fock build, DIIS, eigen-
 * solve, new density, convergence test).  *n_active = molecules still
 * iterating afterwards. */
ks_status scf_step(ks_batch* b, int* n_active);

/* Iterates until every molecule has converged or reached max_iter.  A
 * molecule that does not converge gets status KS_MOL_MAXITER; the call
 * still returns KS_OK. */
ks_status scf_solve(ks_batch* b);

/* scf_solve for n batches at once: every round queues one SCF iteration of
 * each batch that still has active molecules on that batch's own stream,
 * then waits for them in order, so the batches' kernels overlap on the GPU
 * (a batch's small per-molecule steps run beside another batch's XC and J/K
 * work).  Batches must be distinct and should use distinct streams
 * (ks_batch_create's stream argument); on a shared stream the result is the
 * same, only without overlap.  Molecules are independent, so each batch's
 * results equal those of scf_solve on it alone.  Returns the first error of
 * any batch (KS_EINVAL for NULL arguments or n <= 0). */
ks_status scf_solve_many(ks_batch* const* batches, int n);

/* Results of molecule mol (host buffers; eps[nbf] and P[nbf*nbf] may be
 * NULL).  gap = eps_LUMO - eps_HOMO (> 0); eps are the eigenvalues of the
 * last un-extrapolated Fock matrix and P the density that produced it. */
ks_status ks_get_result(const ks_batch* b, int mol, double* E, double* eps, double* P, double* homo,
                        double* lumo, double* gap, int* status, int* n_iter);

/* Packed unique ERIs of molecule mol in FP64 (out[n_eri]), index
 * ij(ij+1)/2 + kl with ij = i(i+1)/2 + j, i >= j, k >= l, ij >= kl. */
ks_status ks_get_eri(const ks_batch* b, int mol, double* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): ks_get_eri
 * without its temporary device buffer.  Copies the packed ERIs lo ..
 * lo + count - 1 of molecule mol (FP64, the order of ks_get_eri) to the host
 * buffer out[count], staged through a library-owned device array of
 * KS_ERI_WINDOW_MAX doubles (8 MiB, held by each device the library runs on
 * until the process ends); the whole list is read in windows.  Allocates
 * nothing.  Errors: KS_EINVAL for a bad molecule, NULL out, count < 0,
 * count > KS_ERI_WINDOW_MAX or a window outside [0, n_eri); KS_ESTATE before
 * eri_build or for an integral-direct batch; KS_EDEVICE if the array's
 * device address cannot be found.  Every call on one device shares that
 * array, so calls that overlap on one device (other host threads, other
 * batches' streams) race; calls from one thread in turn are safe. */
#define KS_ERI_WINDOW_MAX 1048576
ks_status ks_get_eri_window(const ks_batch* b, int mol, long lo, long count, double* out);

/* Copies a resident N x N matrix of molecule mol to the host:
 * which = 0 S, 1 T, 2 V(nuclear), 3 X = S^-1/2, 4 F, 5 P, 6 J, 7 K, 8 V_xc. */
ks_status ks_get_matrix(const ks_batch* b, int mol, int which, double* out);

/* Grid points (x, y, z, w) in bohr of molecule mol: out[n_grid*4]. */
ks_status ks_get_grid(const ks_batch* b, int mol, double* out);

/* Convergence monitor of molecule mol after the last scf_step: the energy of
 * the last Fock build, its change from the previous iteration and the max
 * norm of the orthogonalised commutator X^T (FPS - SPF) X. */
ks_status ks_get_convergence(const ks_batch* b, int mol, double* E, double* dE, double* err);

/* Results of every molecule of the batch in one call (the outputs of paper
 * section 3.1: energy, orbital energies, density and HOMO-LUMO gap), for
 * callers that retire whole batches (host buffers; any pointer may be NULL;
 * KS_EINVAL for a NULL batch, KS_EDEVICE if a copy fails): E, homo,
 * lumo, gap, status, n_iter and n_coarse [n_mol] as ks_get_result and
 * ks_get_iterations give them; eps [sum of nbf] with molecule m's orbital
 * energies after those of molecules 0..m-1; P [sum of nbf^2] with molecule
 * m's row-major N x N density after those of molecules 0..m-1.  One
 * device-to-host copy per array. */
ks_status ks_get_results(const ks_batch* b, double* E, double* homo, double* lumo, double* gap, int* status,
                         int* n_iter, int* n_coarse, double* eps, double* P);

/* Iterations of molecule mol so far: all of them (*n_iter) and those whose XC
 * ran on the coarse start grid (*n_coarse; 0 without one).  Either pointer
 * may be NULL. */
ks_status ks_get_iterations(const ks_batch* b, int mol, int* n_iter, int* n_coarse);

/* Kernel timing.  ks_set_timing(b, 1) clears the counters and records a pair
 * of HIP events on the batch stream around every launch of each kernel
 * family ("eri", "jk", "xc", ...) without host synchronisation;
 * ks_kernel_times() waits for the recorded events and returns, per family,
 * the average device milliseconds per launch (names/ms arrays of length cap;
 * returns the number of families); ks_kernel_counts() the launch counts. */
void ks_set_timing(ks_batch* b, int on);
int ks_kernel_times(const ks_batch* b, const char** names, double* ms, int cap);
int ks_kernel_counts(const ks_batch* b, double* launches, int cap);

/* Releases the batch and all of its device memory.  NULL-safe. */
void ks_batch_destroy(ks_batch* b);

/* Thread-local description of the last error on this thread ("" if none). */
const char* ks_last_error(void);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of SCF requests.  The paper generates its
 * dataset as a stream of independent molecules (section 4); here requests of
 * uneven size arrive at any time, are admitted while the HBM budget allows,
 * keep their density, Fock matrix and DIIS history on the device, advance one
 * SCF iteration per ks_server_progress call together with every other
 * resident molecule, and retire as soon as they converge.
 * ------------------------------------------------------------------------ */
typedef struct ks_server ks_server;

/* opt as for ks_batch_create (NULL = defaults; jk_chunks / xc_chunks of 0
 * become 8 / 16 so that a molecule's arithmetic is the same in any batch);
 * hbm_budget in bytes (0 = 80% of the free device memory); max_batch caps
 * the molecules admitted per admission wave (<= 0: 64). */
ks_status ks_server_create(const ks_options* opt, size_t hbm_budget, int max_batch, ks_server** out);

/* Queues one molecule (Angstrom, charge) and returns its ticket.  The
 * molecule is validated here (KS_EINVAL / KS_EUNSUPPORTED as for
 * ks_batch_create); nothing runs on the device until ks_server_progress. */
ks_status ks_server_submit(ks_server* s, int n_atoms, const int* Z, const double* xyz_angstrom, int charge,
                           long* ticket);

/* One scheduling round: one SCF iteration of every resident molecule (each
 * resident batch on its own stream), admission of queued requests while the
 * budget allows (their integrals and grid are built while the iterations
 * run), then retirement of converged molecules and release of empty batches.
 * *n_finished = requests completed in this call.  The budget check uses an
 * estimate of each request's device bytes; when a batch creation still runs
 * out of device memory its requests stay queued until a resident batch is
 * released (with nothing resident the wave is retried with one request, and
 * a single request that does not fit is rejected: ks_server_poll then
 * returns KS_ENOMEM for it).  Other admission failures reject the wave and
 * are returned. */
ks_status ks_server_progress(ks_server* s, int* n_finished);

/* Result of a ticket: KS_OK when finished (outputs filled; latency_s from
 * submit to retirement), KS_ESTATE while queued or resident, the admission
 * error when the request was rejected.  Output pointers may be NULL. */
ks_status ks_server_poll(const ks_server* s, long ticket, double* E, double* homo, double* lumo, double* gap,
                         int* status, int* n_iter, double* latency_s);

/* Queue length, resident (still iterating) molecules, completed requests and
 * device bytes held by resident batches. */
ks_status ks_server_stats(const ks_server* s, int* queued, int* resident, long* done, size_t* bytes_in_use);

/* Testing hook for the admission error path: the next n admission attempts
 * of this server fail with KS_ENOMEM before touching the device, as if the
 * batch creation had run out of device memory.  KS_EINVAL for a NULL handle
 * or n < 0. */
ks_status ks_server_fail_admissions(ks_server* s, int n);

/* Releases every resident batch.  NULL-safe. */
void ks_server_destroy(ks_server* s);

#ifdef __cplusplus
}
#endif

#endif /* KS_H */
