/*
 * afqmc_kpt.h -- C ABI of the k-point AFQMC walker-batch step on MI355X (gfx950).
 *
 * Method: phaseless auxiliary-field QMC with the two-electron integrals held as
 * momentum-blocked Cholesky vectors (Malone, Zhang, Morales, "Accelerating
 * Auxiliary-Field Quantum Monte Carlo Simulations of Solids with Graphical
 * Processing Units", arXiv:2003.09468).  Section references below are to that
 * paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - k-points form a Gamma-centred Monkhorst-Pack mesh; k is linearised
 *    row-major, k = (k0*mesh[1] + k1)*mesh[2] + k2; k - Q and -Q are taken
 *    componentwise modulo the mesh.
 *  - Complex numbers are interleaved (re, im) pairs: complex128 = 2 doubles,
 *    complex64 = 2 floats.  All arrays are row-major, last index fastest.
 *  - L[Q][k][i][l][g]: Cholesky block for momentum transfer Q, band i at k and
 *    band l at k - Q ("k-Point Representation", momentum convention of L^{Q,k}).
 *    The caller guarantees the time-reversal relation
 *    conj(L[Q][k][i][l][g]) == L[-Q][k-Q][l][i][g] (same section).
 *  - Closed shell: one walker determinant U[w] ((nk*m) x (nk*nocc), dense)
 *    serves both spins; the overlap with the trial is det(A^H U)^2.
 *  - Every pointer is a DEVICE pointer unless marked "host".  The caller owns
 *    and frees every buffer; the library allocates nothing.  Complex arrays
 *    must be 16-byte aligned, float64 arrays 8-byte, int32 arrays 4-byte and
 *    workspaces 256-byte aligned (AFQMC_EALIGN otherwise).
 *  - Calls are asynchronous and ordered on the given HIP stream (a
 *    hipStream_t passed as void*; NULL is the default stream).
 *  - Arguments are validated on the host before any HIP call; a failed check
 *    returns a negative status and launches nothing.  A HIP launch error
 *    returns AFQMC_EHIP.  No call aborts, exits or throws.
 *  - Per-walker numerical failures (singular overlap, non-finite values,
 *    phaseless kill) are reported in status[w] and never fail the call.
 *  - Energies are per supercell; per cell = E / nk.  The ion-ion energy is 0.
 *  - Batches ("Implementation on GPUs": batched processing of walkers and of
 *    independent small operations).  Every entry point takes an array of nprob
 *    problems, which may differ in mesh, m, nocc, nchol, nwalk, prec and dt.
 *    Each stage of the entry runs as one launch for up to 8 problems that share
 *    a kernel variant (precision, size class); stages follow one another on the
 *    stream.  The workspace of a batch is the concatenation of the problems'
 *    workspaces (afqmc_kpt_workspace_bytes returns the total).  Per-call buffers
 *    that are separate arguments (x, xbar, X, vhs, E, gE, gGh) hold the
 *    problems' slices packed one after another at the byte offsets given by
 *    afqmc_kpt_buffer_layout; for nprob = 1 the slice is the whole buffer.
 */
#ifndef AFQMC_KPT_H
#define AFQMC_KPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AFQMC_OK = 0,
  AFQMC_EINVAL = -1,      /* bad dimension, dt or flag */
  AFQMC_ENULL = -2,       /* a required pointer is NULL */
  AFQMC_EALIGN = -3,      /* a pointer is not 16-byte aligned */
  AFQMC_EWORKSPACE = -4,  /* workspace NULL or smaller than afqmc_kpt_workspace_bytes */
  AFQMC_ENODEV = -5,      /* no usable gfx950 device */
  AFQMC_EHIP = -6,        /* a HIP call or kernel launch failed */
  AFQMC_EUNSUPPORTED = -7 /* sizes outside what the kernels implement */
} afqmc_status;

/* Precision of the large complex contractions (force bias L.G, HS potential,
 * Taylor propagation, exchange).  Overlap, Green's function inverse, QR and
 * all energy sums are FP64 in every mode.
 *   FP64:   complex128 operands, FP64 MFMA.
 *   FP32:   complex64 operands (L32, Lh32), FP32 MFMA with FP32 accumulation.
 *   BF16X3: the force bias, the HS potential, the Taylor products and the exchange
 *           contraction of the local energy take their operands split x = hi + lo
 *           into two bfloat16 numbers (from the FP32-rounded value) and multiply them
 *           in three BF16 MFMA passes (hi hi + hi lo + lo hi) with FP32
 *           accumulation; the Taylor polynomial is evaluated in nested form,
 *           T0 + X/1 (T0 + X/2 (... (T0 + X/6 T0))), X = -sqrt(dt) vhs; the energy
 *           adjoint is FP32. */
typedef enum {
  AFQMC_PREC_FP64 = 0,
  AFQMC_PREC_FP32 = 1,
  AFQMC_PREC_BF16X3 = 2,
  AFQMC_PREC_INT8X5 = 3,  /* local energy only, see AFQMC_PREC_PLACE */
  AFQMC_PREC_INT8X4 = 4   /* local energy only, see AFQMC_PREC_PLACE */
} afqmc_prec;

/* AFQMC_PREC_INT8X5, an energy precision: the exchange contraction of afqmc_kpt_energy on
 * int8 MFMA with exact int32 accumulation (an Ozaki-type split).  Every row of the real
 * operands [Re | Im] of Lh (per Q, k, a, g, over r) and of Gh (per walker, row and column
 * block, over r) is scaled by a power of two s with |x| < s / 2 and cut into five signed
 * 7-bit digits, x = s (d1 / 128 + d2 / 128^2 + ... + d5 / 128^5) + rest, |d| <= 64; the
 * digit products of levels i + j <= 6 are summed exactly in int32 per level, the levels
 * combined exactly in FP64 and scaled by the two powers of two.  Each product of the
 * contraction is then exact up to 1.5 * 2^-35 s s' (truncated digits and dropped levels),
 * 2^-35 = 2.9e-11.  The one-body and Coulomb parts, the pairing and all sums are FP64; the
 * adjoint (afqmc_kpt_energy_backward) runs in FP64.  Needs Lh8 (written by prepare) and
 * m <= 64.
 * AFQMC_PREC_INT8X4: the same with four digits per operand (levels i + j <= 5, two thirds
 * of the int8 MFMA work), each product exact up to 1.25 * 2^-28 s s' (2^-28 = 3.7e-9). */

/* Precision placement ("GPU Implementation": the paper runs the whole method in single
 * precision; here each group of contractions has its own).  The prec field of a problem is
 * either an afqmc_prec value, which applies to every contraction, or
 *   AFQMC_PREC_PLACE(step, energy)
 * with step the precision of the force bias, HS potential and Taylor products (every
 * entry but the two below) and energy the precision of afqmc_kpt_energy and
 * afqmc_kpt_energy_backward (also when afqmc_kpt_step evaluates the energy).  Example:
 * AFQMC_PREC_PLACE(AFQMC_PREC_BF16X3, AFQMC_PREC_FP64) propagates with BF16X3 and
 * evaluates the local energy and its adjoint in FP64.  The arrays each stage reads must be
 * present (e.g. Lhs and Ls for a BF16X3 step, Lh32 for a reduced energy); prepare writes
 * all of them. */
#define AFQMC_PREC_PLACE(step, energy) ((step) | (((energy) + 1) << 4))
/* (step: FP64, FP32 or BF16X3; energy: any afqmc_prec) */

/* Per-walker status bits. */
#define AFQMC_WALKER_SINGULAR 1  /* overlap matrix A^H U had a zero pivot */
#define AFQMC_WALKER_NONFINITE 2 /* a non-finite overlap or weight */
#define AFQMC_WALKER_KILLED 4    /* phaseless cut: cos(dtheta) <= 0 set the weight to 0 */

/* Flags of afqmc_kpt_propagate. */
#define AFQMC_PROPAGATE_ORTHO 1  /* re-orthonormalise the walkers after the step */
#define AFQMC_PROPAGATE_REDUCED_GH 4 /* in the FP32 and BF16X3 step precisions, form the new
                                        Gh = (U O^-1)^T by an FP32 product (the overlap, its
                                        inverse, the log determinant and the weights stay
                                        FP64), for a Gh that only feeds the next force bias,
                                        which reads it at that precision anyway; ignored in
                                        FP64 and overridden by AFQMC_PROPAGATE_ORTHO, which
                                        forms Gh in FP64 */

/* Entry-point ids for afqmc_kpt_workspace_bytes. */
typedef enum {
  AFQMC_ENTRY_PREPARE = 0,
  AFQMC_ENTRY_GREENS = 1,
  AFQMC_ENTRY_VBIAS = 2,
  AFQMC_ENTRY_VHS = 3,
  AFQMC_ENTRY_PROPAGATE = 4,
  AFQMC_ENTRY_ORTHO = 5,
  AFQMC_ENTRY_ENERGY = 6,
  AFQMC_ENTRY_ENERGY_BACKWARD = 7,
  AFQMC_ENTRY_STEP = 8,           /* afqmc_kpt_step, graphs and afqmc_kpt_autotune */
  AFQMC_ENTRY_POPULATION = 9      /* afqmc_kpt_population_control */
} afqmc_entry;

/* Flags of afqmc_kpt_step and afqmc_kpt_graph_create (AFQMC_PROPAGATE_ORTHO
 * re-orthonormalises after the last step). */
#define AFQMC_STEP_ENERGY 2      /* local energy after the last step (into E) */

/* Per-call buffers, for afqmc_kpt_buffer_layout. */
typedef enum {
  AFQMC_BUF_FIELDS = 0,  /* x    [nwalk][nk][nchol][2] float64 (one step) */
  AFQMC_BUF_XBAR = 1,    /* xbar [nwalk][nk][nchol][2] complex128 */
  AFQMC_BUF_X = 2,       /* X    [nwalk][nk][nchol] complex128 */
  AFQMC_BUF_VHS = 3,     /* vhs  [nwalk][nk*m][nk*m] complex128 (FP64) or complex64 (FP32) */
  AFQMC_BUF_ENERGY = 4,  /* E    [nwalk][3] complex128 */
  AFQMC_BUF_GE = 5,      /* gE   [nwalk] complex128 */
  AFQMC_BUF_GGH = 6      /* gGh  [nwalk][nk*nocc][nk*m] complex128 */
} afqmc_buffer;

/* One system and its walker batch. */
typedef struct afqmc_kpt_problem {
  int32_t mesh[3];   /* Monkhorst-Pack mesh */
  int32_t nk;        /* = mesh[0]*mesh[1]*mesh[2] */
  int32_t m;         /* bands per k-point */
  int32_t nocc;      /* occupied orbitals per spin per k-point, nocc <= m */
  int32_t nchol;     /* Cholesky vectors per Q */
  int32_t nwalk;     /* walkers in the batch */
  int32_t prec;      /* afqmc_prec, or AFQMC_PREC_PLACE(step, energy) */
  double dt;         /* imaginary time step, > 0 */
  /* static data */
  const void* L;     /* [nk][nk][m][m][nchol] complex128, input */
  const void* A;     /* [nk][m][nocc] complex128 trial orbitals (block diagonal in k), input */
  void* Lh;          /* [nk][nk][nocc][m][nchol] complex128, written by prepare:
                        Lh[Q][k][a][r][g] = sum_p conj(A[k][p][a]) L[Q][k][p][r][g] */
  void* h1h;         /* [nk][nocc][m] complex128, written by prepare: A[k]^H H1[k] */
  void* bhalf;       /* [nk][m][m] complex128, written by prepare: exp(-dt/2 (H1 + V0)) */
  void* L32;         /* [nk][nk][m][m][nchol] complex64 copy of L; step prec FP32 only */
  void* Lh32;        /* [nk][nk][nocc][m][nchol] complex64 copy of Lh; needed when the step
                        or the energy precision is FP32 or BF16X3 (else NULL) */
  void* Lhs;         /* [nk][nk][nchol][nocc][4][32*ceil(m/32)] bfloat16 (uint16) split planes
                        of Lh (re hi, re lo, im hi, im lo; r padded with zeros), written by
                        prepare; needed when the step or the energy precision is BF16X3 */
  void* Ls;          /* half store of L ("k-Point Representation": L^{-Q,k-Q} is the
                        conjugate transpose of L^{Q,k}): for the nq momentum transfers Q whose
                        index does not exceed that of -Q, in increasing Q,
                        [nq][ceil(nchol/32)][nk*m*m (k p r)][4][32] bfloat16 (uint16) split
                        planes of L[Q] (re hi, re lo, im hi, im lo) in chunks of 32 Cholesky
                        indices, g padded with zeros, followed by int32 Q[nq]; written by
                        prepare; step prec BF16X3 only (else NULL).  nq = (nk + s) / 2,
                        s = prod_d (2 if mesh[d] is even else 1) the number of Q = -Q */
  /* walker state */
  void* U;           /* [nwalk][nk*m][nk*nocc] complex128 walker orbitals, in/out */
  void* Gh;          /* [nwalk][nk*nocc][nk*m] complex128 half-rotated Green's function */
  void* logdet;      /* [nwalk] complex128, log det(A^H U) (imaginary part in (-pi, pi]) */
  double* weight;    /* [nwalk] walker weights */
  int32_t* status;   /* [nwalk] AFQMC_WALKER_* bits (sticky: OR-ed in, never cleared) */
  /* energy shift of the projector exp(-dt (H - E_T)) */
  double* etrial;    /* [1] float64 E_T per supercell (Ha), device, or NULL for no shift:
                        every step multiplies each weight by exp(dt E_T), a common factor
                        that keeps the weights of long runs finite; read by the weight
                        update, written by afqmc_kpt_update_etrial */
  /* energy precision AFQMC_PREC_INT8X5 or AFQMC_PREC_INT8X4 only (else NULL), written by
     prepare (five digits in both) */
  void* Lh8;         /* int8 digits of Lh: [nk][nk][nchol][nocc] rows of 5 x KP8 digits
                        (digit d1 .. d5, each over kk = 0 .. KP8-1: Re Lh[Q][k][a][kk][g]
                        for kk < m, Im Lh[..][kk - m][g] for m <= kk < 2m, 0 beyond;
                        KP8 = 64 ceil(2m / 64)), followed by the rows' int32 exponents
                        e ([nk][nk][nchol][nocc], s = 2^e); bytes:
                        nk^2 nchol nocc (5 KP8 + 4) */
  /* spins of the walkers (AFQMC_SPIN_*); 0 for the closed shell */
  int32_t spin;
} afqmc_kpt_problem;

/* Spins ("Introduction to AFQMC": the Hamiltonian sums over the spins of both electrons).
 * AFQMC_SPIN_CLOSED: one determinant serves both spins (the closed shell; nocc electrons
 * of each spin per k-point).  AFQMC_SPIN_UP / AFQMC_SPIN_DOWN: a collinear walker set with
 * one determinant per spin, each against its own block-diagonal trial, held as two
 * problems: the up half at index i of the problem array, the down half at i + 1, in every
 * call that takes either.  The halves describe one system: equal mesh, m, nchol, nwalk,
 * prec and dt, the same L pointer, and the same H1 in afqmc_kpt_prepare (the static arrays
 * derived from L alone, bhalf, L32 and Ls, may be shared or separate); nocc (electrons of
 * that spin per k-point) and A may differ.  Each half has its own U, Gh, logdet, weight and
 * status (distinct pointers; the Lh arrays and h1h come from its own trial).  Semantics:
 *   fields: the down half uses the up half's fields x (its own slot is not read);
 *   force bias: X = sum over both spins of tr(Lh^s Gh^s) (half the sum of the two
 *     halves' closed-shell traces), xbar from it; both halves' xbar and X slots hold them;
 *   propagation: both determinants take the same one- and two-body operators
 *     (afqmc_kpt_step forms the HS potential once per pair, in the up half's vhs slice, and
 *     leaves the down half's slice unwritten);
 *   weights: the overlap is det(O_up) det(O_down); the update multiplies both halves'
 *     weights by the same factor (the phaseless angle of the product's ratio, the up half's
 *     etrial), writes each half's own logdet and ORs the status bits of either half into
 *     both, so that weights started equal stay equal;
 *   energy: E1 and EX summed over the spins, EC = 1/2 sum_{Q,g} X_Q X_-Q of the pair's X;
 *     both halves' E rows hold the pair's energy;
 *   adjoint: gGh of each half is dE/dGh of that spin; the down half uses the up half's gE;
 *   population control: the down half uses the up half's xi, so that the two halves'
 *     (equal) weights give the same copies.
 * A problem with an invalid spin value or an unmatched half makes the call return
 * AFQMC_EINVAL before any HIP call. */
typedef enum {
  AFQMC_SPIN_CLOSED = 0,
  AFQMC_SPIN_UP = 1,
  AFQMC_SPIN_DOWN = 2
} afqmc_spin;

/* Workspace (device bytes) the given entry point needs for these problems.
 * bytes: host pointer.  The same workspace may be reused across calls that
 * are ordered on one stream. */
afqmc_status afqmc_kpt_workspace_bytes(const afqmc_kpt_problem* p, int nprob, int entry,
                                       size_t* bytes);

/* One-time preparation ("k-Point Representation": half-rotated Cholesky
 * matrix; "Introduction to AFQMC": one-body propagator with H1' = H1 + v0).
 *   H1: [nk][m][m] complex128 Hermitian one-body blocks (device).
 * Writes Lh, h1h, bhalf (and L32, Lh32 when prec = FP32), with
 *   V0[k] = -1/2 sum_{Q,g} L[Q][k][:,:,g] L[Q][k][:,:,g]^H and
 *   bhalf[k] = exp(-dt/2 (H1[k] + V0[k])) (FP64 Taylor series with scaling
 *   and squaring).  Does not touch the walker state. */
afqmc_status afqmc_kpt_prepare(const afqmc_kpt_problem* p, int nprob, const void* H1,
                               void* ws, size_t ws_bytes, void* stream);

/* Overlap and half-rotated Green's function (Green's-function equations of the
 * standard representation; blocked by the trial's k structure):
 *   O = A^H U (nk*nocc square), logdet = log det O, Gh = (U O^{-1})^T,
 * all FP64, via blocked Gauss-Jordan inversion with partial (row) pivoting.
 * Reads U; writes Gh, logdet and ORs status.  Requires nk*nocc <= 256. */
afqmc_status afqmc_kpt_greens(const afqmc_kpt_problem* p, int nprob,
                              void* ws, size_t ws_bytes, void* stream);

/* Force bias (k-point force-bias equation, with the -sqrt(dt) of the standard
 * force bias and phases c+ = i, c- = 1):
 *   X[w][Q][g]    = 2 sum_k sum_{a,r} Lh[Q][k][a][r][g] Gh[w][(k a), ((k-Q) r)]
 *   xbar[w][Q][g][0] = -sqrt(dt) (i/2) (X[w][Q][g] + X[w][-Q][g])
 *   xbar[w][Q][g][1] = -sqrt(dt) (1/2) (X[w][Q][g] - X[w][-Q][g])
 * xbar: [nwalk][nk][nchol][2] complex128 out; X: [nwalk][nk][nchol] complex128
 * out.  Reads Gh and Lh (Lh32 for FP32). */
afqmc_status afqmc_kpt_vbias(const afqmc_kpt_problem* p, int nprob, void* xbar, void* X,
                             void* ws, size_t ws_bytes, void* stream);

/* HS potential (k-point HS matrix, single contraction over the combined field):
 *   xt = x - xbar, xi[w][Q][g] = 1/2 [ i (xt+_Q + xt+_-Q) + (xt-_Q - xt-_-Q) ],
 *   vhs[w][(k p), ((k-Q) r)] = -sum_g L[Q][k][p][r][g] xi[w][Q][g]
 * so that the two-body propagator is exp(-sqrt(dt) vhs).
 *   x:    [nwalk][nk][nchol][2] float64 auxiliary fields (the +/- potentials)
 *   xbar: [nwalk][nk][nchol][2] complex128 from afqmc_kpt_vbias
 *   vhs:  [nwalk][nk*m][nk*m], complex128 (FP64) or complex64 (FP32), out. */
afqmc_status afqmc_kpt_vhs(const afqmc_kpt_problem* p, int nprob, const double* x,
                           const void* xbar, void* vhs, void* ws, size_t ws_bytes,
                           void* stream);

/* Walker propagation and hybrid phaseless weights ("Introduction to AFQMC":
 * symmetric propagator, importance function and weight update):
 *   U <- bhalf . T6(-sqrt(dt) vhs) . bhalf . U,  T6(V) U = sum_{j<=6} V^j U / j!
 * computed term by term (T_j = V T_{j-1} / j); then the new Gh and logdet, and
 *   log I = 2 (logdet' - logdet) + sum_{Q,g,+/-} (x xbar - xbar^2 / 2),
 *   dtheta = arg exp(2 (logdet' - logdet)),
 *   weight <- |I| max(0, cos dtheta) exp(dt E_T) weight   (E_T = *etrial, or 0 if NULL).
 * With AFQMC_PROPAGATE_ORTHO the walkers are re-orthonormalised afterwards
 * (see afqmc_kpt_orthonormalize).  vhs, x, xbar as in afqmc_kpt_vhs.  afqmc_kpt_step sets
 * AFQMC_PROPAGATE_REDUCED_GH for every step whose Gh feeds only the next force bias (all
 * but a last step without AFQMC_PROPAGATE_ORTHO). */
afqmc_status afqmc_kpt_propagate(const afqmc_kpt_problem* p, int nprob, const void* vhs,
                                 const double* x, const void* xbar, int flags,
                                 void* ws, size_t ws_bytes, void* stream);

/* Walker re-orthonormalisation (once per block, "Scaling and Performance"):
 * U <- Q of the thin QR factorisation U = Q R with diag(R) real positive
 * (FP64 Cholesky-QR applied twice), then Gh and logdet are recomputed.
 * Gh and the local energy are unchanged by it.  Requires nk*nocc <= 256
 * (AFQMC_EUNSUPPORTED otherwise, also for AFQMC_PROPAGATE_ORTHO elsewhere). */
afqmc_status afqmc_kpt_orthonormalize(const afqmc_kpt_problem* p, int nprob,
                                      void* ws, size_t ws_bytes, void* stream);

/* Local energy (k-point local-energy equation, evaluated with the paper's
 * energy algorithm, steps 1-3):
 *   E[w][0] = E1B = 2 sum_k sum_{a,r} h1h[k][a][r] Gh[w][(k a), (k r)]
 *   E[w][1] = EC  = 1/2 sum_{Q,g} X[w][Q][g] X[w][-Q][g]
 *   E[w][2] = EX  = -sum_{Q,k,k'} sum_{a,b,g} T1[b,a,g] T2[a,b,g],
 *     T1[b,a,g] = sum_r Lh[Q][k][a][r][g]      Gh[w][((k'-Q) b), ((k-Q) r)]
 *     T2[a,b,g] = sum_s Lh[-Q][k'-Q][b][s][g]  Gh[w][(k a), (k' s)]
 * E: [nwalk][3] complex128 out, per supercell.  The T intermediates never
 * reach memory; all sums are FP64.  Requires nocc <= 16. */
afqmc_status afqmc_kpt_energy(const afqmc_kpt_problem* p, int nprob, void* E,
                              void* ws, size_t ws_bytes, void* stream);

/* The local energy of afqmc_kpt_energy (same kernels, same results bit for bit) for
 * callers that cannot allocate device memory: code under HIP graph capture, serving loops
 * and harnesses that forbid hipMalloc.  Instead of a caller workspace the scratch regions
 * of the energy (Cholesky traces, split-K and exchange partials) live in a fixed device
 * array of AFQMC_ENERGY_NOALLOC_MAX_BYTES, one per device, held from the first call on
 * that device until the process ends; the call allocates nothing (no hipMalloc, no
 * library allocation).  The caller still passes the problems and E.
 *   Returns AFQMC_EWORKSPACE when the batch needs more scratch than that (the bytes
 *   afqmc_kpt_workspace_bytes reports for AFQMC_ENTRY_ENERGY); the 3x3x3, m = 26,
 *   nchol = 208, 64-walker energy needs about 50 MB.
 *   Every call on a device shares that device's array, and nothing in it needs to start
 *   at zero: calls that overlap on one device (two streams, two threads) race and give
 *   wrong energies; order them on one stream. */
#define AFQMC_ENERGY_NOALLOC_MAX_BYTES (64u << 20)
afqmc_status afqmc_kpt_energy_noalloc(const afqmc_kpt_problem* p, int nprob, void* E,
                                      void* stream);

/* Adjoint of the local energy with respect to Gh (generalized Fock matrix):
 *   gGh[w][(k1 al), (k2 rho)] = gE[w] * dE_L[w] / dGh[w][(k1 al), (k2 rho)],
 *   E_L = E1B + EC + EX (holomorphic in Gh, so this is the plain complex
 *   derivative), which equals
 *   2 [ h1h[k1][al][rho] d(k1,k2) + sum_g Lh[Q0][k1][al][rho][g] X[w][-Q0][g]
 *       - sum_{Q,b,g} T1_{(Q,k1,k2)}[b,al,g] Lh[-Q][k2-Q][b][rho][g] ],  Q0 = k1 - k2.
 * The exchange intermediates T1 are recomputed, not stored.
 *   gE:  [nwalk] complex128 cotangent, or NULL for 1.
 *   gGh: [nwalk][nk*nocc][nk*m] complex128 out. */
afqmc_status afqmc_kpt_energy_backward(const afqmc_kpt_problem* p, int nprob, const void* gE,
                                       void* gGh, void* ws, size_t ws_bytes, void* stream);

/* Mixed estimate of the energy per problem ("Standard Representation": the
 * weighted average of the walkers' local energies):
 *   Emix[i] = sum_w weight[w] (E[w][0] + E[w][1] + E[w][2]) / sum_w weight[w]
 * with E from afqmc_kpt_energy (AFQMC_BUF_ENERGY layout) and the problems' current
 * weights; walkers with weight 0 (killed, singular) drop out.  Emix: [nprob]
 * complex128, device; NaN when every weight of a problem is 0.  FP64 sums. */
afqmc_status afqmc_kpt_mixed_energy(const afqmc_kpt_problem* p, int nprob, const void* E,
                                    void* Emix, void* stream);

/* Population control between blocks by the comb (the paper's blocks imply a branching
 * step that it does not spell out; this is the standard comb, a stochastic
 * reconfiguration driven by one uniform number per problem).  With the cumulative
 * weights c_i = w_0 + ... + w_i, summed in FP64 in walker order, and c = c_{nwalk-1},
 * copy j (0 <= j < nwalk) of the new population is the walker i with
 *   c_{i-1} <= (j + xi) (c / nwalk) < c_i        (c_{-1} = 0),
 * taken no later than the last walker of positive weight; so a walker of weight w_i
 * gets floor or ceil of nwalk w_i / c copies, and one of weight 0 none.  U, Gh, logdet
 * and status of the chosen walkers are copied in place and every weight becomes
 * c / nwalk.  A problem with a negative or non-finite weight, or a total that is not
 * positive, is left unchanged (parent[j] = j).
 *   xi:     [nprob] host array, each in [0, 1)
 *   parent: NULL, or [nprob] host array whose entries are NULL or device [nwalk] int32
 *           outputs (the walker each copy came from)
 * Workspace: AFQMC_ENTRY_POPULATION (a copy of U and Gh).  FP64 arithmetic. */
afqmc_status afqmc_kpt_population_control(const afqmc_kpt_problem* p, int nprob,
                                          const double* xi, int32_t* const* parent, void* ws,
                                          size_t ws_bytes, void* stream);

/* Energy shift between blocks: E_T <- (1 - blend) E_T + blend Re(Emix[i]) for every problem
 * i whose mixed estimate Emix[i] (from afqmc_kpt_mixed_energy, device [nprob] complex128)
 * is finite; E_T is left as it is otherwise.  Requires etrial in every problem; blend in
 * (0, 1].  Device-side, so a captured block can include it.  FP64. */
afqmc_status afqmc_kpt_update_etrial(const afqmc_kpt_problem* p, int nprob, const void* Emix,
                                     double blend, void* stream);

/* One level of a blocking analysis. */
typedef struct afqmc_reblock_level {
  int64_t n;       /* blocks at this level */
  double mean;     /* their mean (the same at every level up to the dropped tail) */
  double err;      /* standard error of the mean, sqrt(s^2 / n), s^2 with n - 1 */
  double err_err;  /* its uncertainty, err / sqrt(2 (n - 1)) */
} afqmc_reblock_level;

/* Blocking analysis of a serially correlated series, e.g. the mixed energies of successive
 * blocks (the error bars of the paper's results): level 0 is the series x[0..n-1], level
 * l + 1 the means of neighbouring pairs of level l (an odd last element dropped), down to
 * two blocks.  *optimal is the first level whose block size B = 2^l satisfies
 * B^3 > 2 n (err_l / err_0)^4 (Lee, Needs and Towler, Phys. Rev. E 83, 066706 (2011)),
 * or -1.  Host arrays: x [n]; levels [max_levels] out (the first min(*nlevels,
 * max_levels) written).  Sums in FP64 in series order.  Needs no device. */
afqmc_status afqmc_kpt_reblock(const double* x, int64_t n, afqmc_reblock_level* levels,
                               int max_levels, int* nlevels, int* optimal);

/* The standard (dense) representation of the system ("Standard Representation"): one
 * set of Cholesky vectors of the whole supercell basis, N = nk m orbitals, n = nk nocc
 * occupied, nk nchol Hermitian vectors.  For every Q whose index does not exceed that of
 * -Q (increasing Q): Q = -Q gives the nchol supercell operators LL_Q; a pair (Q, -Q) the
 * 2 nchol vectors (LL_Q + LL_Q^H)/sqrt 2, then i (LL_Q - LL_Q^H)/sqrt 2, which carry the
 * same two-body integrals and the same V0.  Writes, for a 1x1x1-mesh problem with m = N,
 * nocc = n, nchol = nk nchol (run through the same entry points):
 *   Ld:  [1][1][N][N][nk nchol] complex128, Hermitian per vector
 *   H1d: [1][N][N] complex128, block diagonal of H1 ([nk][m][m] complex128, device)
 *   Ad:  [1][N][n] complex128, block diagonal of the trial A
 * Reads L and A of the first problem of p (nprob = 1, closed shell).  The dense walkers are
 * the k-point ones unchanged ([nwalk][N][n]).  Returns AFQMC_EUNSUPPORTED when the dense
 * problem exceeds the sizes the kernels run (N > 64 or n > 16). */
afqmc_status afqmc_kpt_dense_system(const afqmc_kpt_problem* p, int nprob, const void* H1,
                                    void* Ld, void* H1d, void* Ad, void* stream);

/* The fields of the dense system that give the same HS exponent as the k-point fields x
 * ([nwalk][nk][nchol][2] float64): for a pair, x_A = (x+_Q + x+_-Q)/sqrt 2 and
 * x_B = (x-_-Q - x-_Q)/sqrt 2 (an orthogonal change of the Gaussian fields; the other two
 * directions neither enter the exponent nor carry a force bias); for Q = -Q, x+_Q.
 *   xd: [nwalk][1][nk nchol][2] float64 out (the minus fields 0: a Hermitian vector has no
 *   minus potential). */
afqmc_status afqmc_kpt_dense_fields(const afqmc_kpt_problem* p, int nprob, const double* x,
                                    double* xd, void* stream);

/* Non-uniform band counts ("k-Point Representation": m is the average number of bands per
 * k-point).  A system with mk[k] bands at k-point k is the uniform system with m >= max mk
 * bands per k-point whose extra bands are zero rows and columns of L, H1 and the trial and
 * zero rows of the walkers: those bands carry no matrix element, the propagator keeps the
 * walkers' zero rows zero (the identity block of exp(-dt/2 (H1 + V0)), a zero block of the
 * HS potential), and every overlap, trace and contraction is that of the ragged system.
 * afqmc_kpt_pad_bands writes the padded arrays from packed ragged ones; every entry point
 * then runs on the padded problem unchanged.
 *   p:    one padded problem (nprob = 1); mesh, nk, m, nocc, nchol and nwalk are read, its
 *         pointers are not; nk <= AFQMC_PAD_MAX_NK
 *   mk:   [nk] host int32, nocc <= mk[k] <= m
 *   L_r:  blocks (Q, k), Q-major then k, each [mk[k]][mk[k-Q]][nchol] complex128
 *   H1_r: blocks k, each [mk[k]][mk[k]] complex128
 *   A_r:  blocks k, each [mk[k]][nocc] complex128
 *   U_r:  [nwalk][sum_k mk[k]][nk*nocc] complex128 (rows of k-point k after those of k - 1)
 *   L, H1, A, U: the padded [nk][nk][m][m][nchol], [nk][m][m], [nk][m][nocc] and
 *         [nwalk][nk*m][nk*nocc] complex128 outputs, zero beyond the ragged blocks.
 * All device pointers; an input may be NULL, and its output is then not written. */
#define AFQMC_PAD_MAX_NK 128
afqmc_status afqmc_kpt_pad_bands(const afqmc_kpt_problem* p, int nprob, const int32_t* mk,
                                 const void* L_r, const void* H1_r, const void* A_r,
                                 const void* U_r, void* L, void* H1, void* A, void* U,
                                 void* stream);

/* The ragged walkers and half-rotated Green's functions of a padded problem (the inverse of
 * the walker padding above): U [nwalk][nk*m][nk*nocc] -> U_r [nwalk][sum mk][nk*nocc] and
 * Gh [nwalk][nk*nocc][nk*m] -> Gh_r [nwalk][nk*nocc][sum mk], complex128 device arrays
 * (either pair may be NULL).  Same p, nprob and mk rules as afqmc_kpt_pad_bands. */
afqmc_status afqmc_kpt_unpad_bands(const afqmc_kpt_problem* p, int nprob, const int32_t* mk,
                                   const void* U, const void* Gh, void* U_r, void* Gh_r,
                                   void* stream);

/* Packed layout of one per-call buffer for a batch (host).  offsets: host
 * array of nprob + 1 entries; offsets[i] is the byte offset of problem i's
 * slice (a multiple of 256) and offsets[nprob] the end of the last slice, i.e.
 * the bytes to allocate. */
afqmc_status afqmc_kpt_buffer_layout(const afqmc_kpt_problem* p, int nprob, int buf,
                                     size_t* offsets);

/* nsteps walker steps of every problem of the batch (the propagation of
 * "Introduction to AFQMC" with the k-point force bias and HS potential), each
 * step being afqmc_kpt_vbias, afqmc_kpt_vhs and afqmc_kpt_propagate in turn:
 *   x:    fields of all steps; step s, problem i at byte offset
 *         s * offsets[nprob] + offsets[i] (AFQMC_BUF_FIELDS layout)
 *   xbar: force bias of the current step (AFQMC_BUF_XBAR layout), out
 *   vhs:  HS potential of the current step (AFQMC_BUF_VHS layout), out
 *   E:    local energy after the last step (AFQMC_BUF_ENERGY layout), out,
 *         with AFQMC_STEP_ENERGY, else may be NULL.
 * flags: AFQMC_PROPAGATE_ORTHO (after the last step), AFQMC_STEP_ENERGY.
 * Workspace: AFQMC_ENTRY_STEP. */
afqmc_status afqmc_kpt_step(const afqmc_kpt_problem* p, int nprob, const double* x, int nsteps,
                            void* xbar, void* vhs, void* E, int flags, void* ws,
                            size_t ws_bytes, void* stream);

/* Times the compiled tile candidates of the Taylor, HS-potential and
 * force-bias contractions on this batch and keeps the fastest for later calls
 * with the same shapes (process-wide cache, thread-safe).  Overwrites vhs
 * (AFQMC_BUF_VHS layout) and the workspace (AFQMC_ENTRY_STEP); the walker
 * state is not touched.  Synchronises the stream; not allowed while the
 * stream is being captured. */
afqmc_status afqmc_kpt_autotune(const afqmc_kpt_problem* p, int nprob, void* vhs, void* ws,
                                size_t ws_bytes, void* stream);

/* A captured block of steps: afqmc_kpt_step with these exact arguments,
 * recorded once into a HIP graph and replayed by afqmc_kpt_graph_launch.  The
 * graph keeps the addresses: the buffers and workspace must stay allocated
 * until afqmc_kpt_graph_destroy, and the caller refreshes the fields in x
 * between launches.  The problem array is copied.  Creation records launches
 * only (nothing runs); it must not overlap a capture on the same thread. */
typedef struct afqmc_kpt_graph_s* afqmc_kpt_graph;
afqmc_status afqmc_kpt_graph_create(const afqmc_kpt_problem* p, int nprob, const double* x,
                                    int nsteps, void* xbar, void* vhs, void* E, int flags,
                                    void* ws, size_t ws_bytes, afqmc_kpt_graph* graph);
afqmc_status afqmc_kpt_graph_launch(afqmc_kpt_graph graph, void* stream);
afqmc_status afqmc_kpt_graph_destroy(afqmc_kpt_graph graph);

/* Kernel classes of the optional event timing. */
typedef enum {
  AFQMC_KC_TAYLOR = 0,        /* one Taylor term of the two-body propagator */
  AFQMC_KC_VHS = 1,           /* HS-potential contraction (with the field combination) */
  AFQMC_KC_VBIAS = 2,         /* force-bias contraction and reduction */
  AFQMC_KC_GREENS = 3,        /* overlap inverse / log det and the Gh solve */
  AFQMC_KC_BHALF = 4,         /* one-body half step */
  AFQMC_KC_WEIGHTS = 5,       /* phaseless weight update */
  AFQMC_KC_ORTHO = 6,         /* Cholesky-QR passes */
  AFQMC_KC_EXCHANGE = 7,      /* paired exchange contraction of the local energy */
  AFQMC_KC_ENERGY_REST = 8,   /* one-body, Coulomb and final energy reduction */
  AFQMC_KC_EXCHANGE_BWD = 9,  /* exchange part of the energy adjoint */
  AFQMC_KC_COUNT = 10
} afqmc_kernel_class;

/* Diagnostics for callers that measure kernels (host).  While enabled, every launch of
 * a kernel class is bracketed by two hipEvents recorded on the launch stream; at most
 * `capacity` launches are recorded between reads (later ones are not timed).  Enabling
 * resets the totals; disabling keeps them readable.  Calls that overlap on one process
 * share the recorder. */
afqmc_status afqmc_kpt_timing_enable(int enable, int capacity);

/* Accumulated time (ms) and number of timed launches of one kernel class since the last
 * enable; waits for the recorded events. */
afqmc_status afqmc_kpt_timing_read(int kclass, double* total_ms, long long* launches);

/* Static string for a status code (host). */
const char* afqmc_kpt_strerror(int status);

/* Library version string (host). */
const char* afqmc_kpt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AFQMC_KPT_H */
