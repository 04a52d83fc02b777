/* bandsolve.h -- C ABI of libbandsolve, batched band-SLAE solvers for
 * MI355X (gfx950).
 *
 * The library solves many independent pentadiagonal (kind 5) or tridiagonal
 * (kind 3) systems at once -- the N systems that each sweep of an ADI scheme
 * for a parabolic PDE produces, d times per time step (Veneva & Ayriyan,
 * arXiv:1804.09666, Sec. 1).  Methods:
 *   - NPDM / NTDM: LU-based direct solvers for PD / TD matrices (Sec. 1;
 *     complexity 19N-29 and 9N+2, Sec. 4);
 *   - MNPDM: NPDM that skips the work on the sparse outer diagonals
 *     (Sec. 1; 13N+7K-14, Sec. 4);
 *   - ILU(0) of the band and the Stone method SIP (Sec. 2, Algorithm 1),
 *     optionally with Hotelling-Bodewig approximate inverses of L and U in
 *     place of the triangular solves (Remark of Sec. 2; Appendix).
 *
 * MEMORY.  Every array argument is a DEVICE pointer owned by the caller; the
 * library keeps no pointer after a call returns and allocates nothing.
 * Scratch memory, where a call needs any, is the caller's `workspace`, sized
 * by bs_workspace_bytes().
 *
 * LAYOUT.  Batch-interleaved: element (row i, system s) of every per-row array
 * is at p[i*ld + s], 0 <= i < n, 0 <= s < batch, ld >= batch.  Consecutive
 * systems are contiguous, so one row of 64 systems is one 512-byte (FP64)
 * transaction; ld a multiple of 64 is recommended.  Row i of a system reads
 *     e_i x_{i-2} + c_i x_{i-1} + d_i x_i + a_i x_{i+1} + b_i x_{i+2} = y_i
 * with diags[0]=e, [1]=c, [2]=d, [3]=a, [4]=b.  Kind 3 reads only c, d, a
 * (diags[0] and diags[4] may be NULL).  The corner slots e_0, e_1, c_0,
 * a_{n-1}, b_{n-2}, b_{n-1} lie outside the matrix: their values are never
 * used (they may hold anything, NaN included; the memory must exist, as
 * every array spans n*ld elements).  Inputs are never written.  x may alias
 * rhs.
 *
 * PRECISION.  dtype BS_F64: every array is double.  dtype BS_F32 (fused
 * band_solve only, n >= 8): diags, rhs and x are stored as float.  The
 * pivots and the forward (L) recurrences always run in FP64 on the values
 * read.  By default (BS_OPT_F32_STATE = 1, systems of n <= 4096) the per-row
 * results of the forward sweep are kept in FP32 and the backward (U)
 * substitution and the final x run in FP32 (forward error a few FP32
 * roundings of ||x||; the FP64 state takes twice the registers and half the
 * rows per block).  With BS_OPT_F32_STATE = 0, and for longer systems, every
 * step runs in FP64 and only the storage rounding differs from FP64.
 * band_solve_refine takes FP64 arrays, solves with FP32 storage and restores
 * FP64 accuracy by iterative refinement.
 *
 * STREAMS.  `stream` is a hipStream_t passed as void* (NULL = the default
 * stream).  Every call only enqueues work on it and returns; results, info,
 * iters and relres are valid once the stream has reached that point.
 *
 * ERRORS.  The return value is a bs_status decided on the host, before
 * anything is enqueued, except BS_ELAUNCH (a launch failed; some work of the
 * call may already be enqueued).  Numerical outcomes are written per system,
 * asynchronously, to `info`:
 *     0      success
 *     i+1    (> 0) the first pivot that is exactly zero or not finite is in
 *            row i; x of that system is unspecified
 *    -1      SIP: not converged within max_iter
 *    -2      SIP: diverged (residual not finite, or relative residual above
 *            1e3 * max(1, relative residual of x0))
 *    -3      MNPDM: the outer-entry list of the system is not strictly
 *            ascending or names a row outside 0..n-1
 *    -4      split-row band_solve with x aliasing rhs: the blocks that share
 *            the system did not all arrive within BS_OPT_EXCHANGE_WAIT_US
 *            (default one second; x unspecified; without aliasing the rows
 *            of the blocks that gave up are solved sequentially instead)
 *    -1, -2  band_solve_refine: not converged within max_steps / residual not
 *            finite (as for SIP)
 */
#ifndef BANDSOLVE_H
#define BANDSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum bs_status_code {
  BS_OK = 0,
  BS_EINVAL = 1,     /* an argument is out of range, NULL or misaligned   */
  BS_ELAUNCH = 2,    /* a kernel launch failed (HIP error)                 */
  BS_EWORKSPACE = 3, /* ws_bytes smaller than bs_workspace_bytes() asks    */
  BS_ENODEV = 4      /* no usable gfx950 device for the current HIP device */
};

enum bs_dtype_code { BS_F64 = 0, BS_F32 = 1 };

enum bs_op_code {
  BS_OP_FACTOR = 0,       /* band_factor                                   */
  BS_OP_SOLVE = 1,        /* band_solve with factors == NULL (fused)       */
  BS_OP_SOLVE_FACTORED = 2, /* band_solve with factors from band_factor    */
  BS_OP_MNPDM = 3,        /* band_solve_mnpdm                              */
  BS_OP_SIP = 4,          /* sip_solve                                     */
  BS_OP_REFINE = 5,       /* band_solve_refine (dtype BS_F64)              */
  BS_OP_ADI = 6           /* band_solve_adi (dtype BS_F64)                 */
};

/* Human-readable name of a status code (static string). */
const char* bs_status_str(int32_t status);

/* Library ABI version (major*100 + minor). */
int32_t bs_version(void);

/* Bytes of device workspace the call `op` needs for (kind, dtype, n, batch,
 * ld) under the current options; 0 when it needs none.  Returns (size_t)-1
 * for arguments the call would reject.  Host-only, never touches the GPU. */
size_t bs_workspace_bytes(int32_t op, int32_t kind, int32_t dtype, int64_t n,
                          int64_t batch, int64_t ld);

/* Process-wide tuning options (not per-call state; read at every call).
 *   BS_OPT_DIRECT_PATH     fused band_solve kernel and the ILU(0) of
 *                          band_factor and sip_solve: 0 and 2 rows of a
 *                          system split over lanes (default; one lane per
 *                          system for small n), 1 one lane per system
 *   BS_OPT_PART_PD_VARIANT index of the split-row PD kernel variant
 *   BS_OPT_PART_TD_VARIANT index of the split-row TD kernel variant
 *   BS_OPT_SIP_PATH        sip_solve kernel: 0 and 2 rows of a system split
 *                          over lanes where the HB steps allow it (up to three
 *                          steps per launch where their halos fit) or both
 *                          solves are exact (default),
 *                          1 one lane per system, 3 (4) rows split over lanes
 *                          with one step (at most two steps) per launch (same
 *                          iterates as 0)
 *   BS_OPT_EXCHANGE_WAIT_US longest wait, in microseconds (0 .. 10^7, default
 *                          10^6), of a split-row block for the other blocks of
 *                          its system before it gives up and the system's
 *                          info becomes -4
 *   BS_OPT_F32_STATE       FP32 storage (dtype BS_F32): 1 (default) keeps
 *                          the per-row state of the split kernels in FP32,
 *                          0 in FP64; 2 + k forces compact variant k (tuning)
 * bs_set_option returns BS_EINVAL for an unknown key or a value out of range;
 * bs_get_option returns -1 for an unknown key. */
enum bs_option_code {
  BS_OPT_DIRECT_PATH = 0,
  BS_OPT_PART_PD_VARIANT = 1,
  BS_OPT_PART_TD_VARIANT = 2,
  BS_OPT_SIP_PATH = 3,
  BS_OPT_EXCHANGE_WAIT_US = 4,
  BS_OPT_F32_STATE = 5
};
int32_t bs_set_option(int32_t key, int64_t value);
int64_t bs_get_option(int32_t key);

/* Shape of split-row variant `index` of `kind`: shape[0] = rows per lane M,
 * shape[1] = lanes per system in a block PW (a tile of M*PW rows),
 * shape[2] = systems per block G, shape[3] = most tiles per system TMAX (the
 * variant handles 8 <= n <= M*PW*TMAX).  BS_EINVAL if there is no such
 * variant. */
int32_t bs_part_variant(int32_t kind, int32_t index, int32_t shape[4]);

/* ILU(0) of every system: the band Doolittle factorization A = L U with L
 * unit lower (l2, l1 on diagonals -2, -1) and U upper (u0, u1, u2 on 0, +1,
 * +2, u2 = b), which for a band is its exact LU (Sec. 2: ILU(0) keeps the
 * zero pattern of A; a band has no fill outside it).
 *   l2_i = e_i / u0_{i-2};  l1_i = (c_i - l2_i u1_{i-2}) / u0_{i-1};
 *   u0_i = (d_i - l2_i u2_{i-2}) - l1_i u1_{i-1};  u1_i = a_i - l1_i u2_{i-1}.
 * factors: kind 5 -> 4 arrays [l2 | l1 | u0 | u1], kind 3 -> 2 arrays
 * [l1 | u0], each n*ld elements in the batch-interleaved layout (array k at
 * factors + k*n*ld).  Entries outside the band (l2 of rows 0,1, l1 of row 0,
 * u1 of row n-1) are written as 0.  info[s]: 0 or i+1 for the first bad u0_i.
 * dtype must be BS_F64.
 * When the batch alone cannot fill the GPU, the rows of each system are cut
 * into chunks that start a few dozen rows early, as if the matrix began
 * there (the recurrence forgets its start geometrically on diagonally
 * dominant systems); a second pass recomputes the first two rows of every
 * chunk from the stored rows before it and compares bit patterns, and
 * factorizes a system again sequentially if any differs.  Factors and info
 * are therefore always the sequential recurrence's to the last bit; only the
 * time depends on the matrix.  BS_OPT_DIRECT_PATH = 1 keeps one lane per
 * system. */
int32_t band_factor(int32_t kind, int32_t dtype, int64_t n, int64_t batch,
                    int64_t ld, const void* const diags[5], void* factors,
                    int32_t* info, void* stream);

/* Solve A x = rhs for every system.
 * factors == NULL: fused factor + solve, NPDM (kind 5) or NTDM (kind 3)
 *   (Sec. 1): LU without pivoting, L = (e, gamma, mu), U unit upper
 *   (alpha, beta); info[s] reports the first bad pivot.  With one lane per
 *   system (option BS_OPT_DIRECT_PATH = 1) the arithmetic is that of the
 *   sequential recurrence.  By default the rows of a system are split over
 *   many lanes (a partitioned elimination: chunks of rows eliminated on
 *   their own, then a reduced system on the chunk interfaces), which
 *   changes the rounding only: one launch for n up to M*PW*TMAX of the
 *   configured variant, three launches (tile maps, per-system reduction,
 *   finish) and a redo launch for longer systems.  dtype BS_F32 needs this
 *   split path (n >= 8).
 *   Breakdown on the split path: a system whose partitioned elimination
 *   meets a pivot or a 2x2 interface block that is not finite or not larger
 *   than 2^-12 times the magnitude of the terms it is formed from (a local
 *   pivot: the sum |e|+|c|+|d|+|a|+|b| of its row) is solved again by the
 *   sequential recurrence, in the same call; its x and info are then the
 *   sequential method's to the last bit (for BS_F32 storage: in FP64 on the
 *   stored values, x rounded once).  So a zero or tiny diagonal at the start
 *   of a chunk, where the sequential pivot is regular, gives info = 0, and a
 *   sequential pivot that cancels inside a chunk (where the chunk's own
 *   recurrence has forgotten its start and meets it too) gives the
 *   sequential info.  A sequential pivot that vanishes in one of the first
 *   rows of a chunk other than the first is not met by the partitioned
 *   elimination, which solves the system (regular there) and reports 0;
 *   BS_OPT_DIRECT_PATH = 1 reports such breakdowns as NPDM does.
 * factors != NULL: substitution with the factors of band_factor (same kind
 *   and layout): L z = rhs, U x = z.  info[s] is set to 0.  Where the batch
 *   is small the rows of each sweep are split over lanes as in band_factor
 *   (chunks started early, a bitwise proof at every chunk boundary, a
 *   sequential redo where it fails: x is the sequential sweeps' to the last
 *   bit); z then goes through the workspace (n * ceil(batch/64)*64 doubles,
 *   then one int32 flag per system).
 * workspace / ws_bytes: as bs_workspace_bytes(BS_OP_SOLVE or
 *   BS_OP_SOLVE_FACTORED, ...); may be NULL / 0 when that is 0.  When the
 *   rows of a system span several blocks, the blocks meet at counters in the
 *   workspace: its contents must be zero before its first use with
 *   band_solve, and every completed call leaves them zero again (blocks
 *   that gave up waiting still leave, and the last one resets the counters;
 *   zero the workspace again only if a call was interrupted).  A block that
 *   gives up writes no x; the last block of its system then solves that
 *   block's rows with the sequential recurrence, unless x aliases rhs (the
 *   other blocks have overwritten rhs rows): info -4, x unspecified.  The
 *   workspace also holds the planes of the sequential redo (3 for kind 5, 2
 *   for kind 3, n * ceil(batch/64)*64 doubles each), touched only by systems
 *   that are redone.  Calls that share one workspace must not run
 *   concurrently.
 *   The factored substitution uses its workspace for z and needs no zeroing. */
int32_t band_solve(int32_t kind, int32_t dtype, int64_t n, int64_t batch,
                   int64_t ld, const void* const diags[5], const void* factors,
                   const void* rhs, void* x, int32_t* info, void* workspace,
                   size_t ws_bytes, void* stream);

/* band_solve (factors == NULL) for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the scratch that band_solve takes from `workspace`
 * comes from a static device array of BS_NOALLOC_SCRATCH_BYTES bytes that
 * every GPU the library runs on holds from module load until the process
 * ends.  Same kernels, so x and info are band_solve's to the bit.  The call
 * allocates nothing; its first call on a device looks the array's address up
 * (hipGetSymbolAddress) once for that device.  Each call clears the meeting
 * counters it needs (a fill kernel on `stream`).  BS_EWORKSPACE when the
 * shape needs more than BS_NOALLOC_SCRATCH_BYTES (bs_workspace_bytes of
 * BS_OP_SOLVE; e.g. PD FP64 up to about n * batch = 5.3e6 with the default
 * path); other checks as band_solve.  All calls on one GPU share the one
 * array: calls that overlap in time on one GPU (on different streams or from
 * different threads) race, and must be serialised by the caller. */
#define BS_NOALLOC_SCRATCH_BYTES (128u << 20)
int32_t band_solve_noalloc(int32_t kind, int32_t dtype, int64_t n, int64_t batch, int64_t ld,
                           const void* const diags[5], const void* rhs, void* x, int32_t* info,
                           void* stream);

/* One ADI sweep assembled inside the solver: for every line s (column s of
 * the batch-interleaved [n, ld] input v, the field the sweep starts from),
 * solve (I - tau L(k(v))) w = v for u_t = (k(u) u_x)_x, k(u) = 1 + u^2 (the
 * nonlinear parabolic problem of Sec. 1), r = tau / h^2:
 *   interior rows  c_i = -r k_{i-1/2},  a_i = -r k_{i+1/2},
 *                  d_i = 1 + r (k_{i-1/2} + k_{i+1/2}),  rhs_i = v_i,
 *                  k_{i+1/2} = (k(v_i) + k(v_{i+1})) / 2;
 *   zero-flux boundary rows, rhs 0: kind 3 (first order, tridiagonal) [1, -1]
 *   and [-1, 1]; kind 5 (second order, pentadiagonal) [-3, 4, -1] and
 *   [1, -4, 3].
 * The coefficients are formed in registers in this order (each product and
 * sum rounded on its own): the sweep reads v once and writes x once, 16 bytes
 * per row instead of the 56 (PD) of band_solve on assembled diagonals, and
 * the result is bitwise band_solve's on those diagonals.  Split-row kernels
 * only: 8 <= n <= M*PW*TMAX of the first two variants of `kind`; FP64;
 * x may alias v; workspace as bs_workspace_bytes(BS_OP_ADI, ...) (meeting
 * counters: zero before first use, left zero). */
int32_t band_solve_adi(int32_t kind, int64_t n, int64_t batch, int64_t ld, double r,
                       const double* v, double* x, int32_t* info, void* workspace,
                       size_t ws_bytes, void* stream);

/* Mixed-precision NPDM / NTDM with iterative refinement.  The matrix and rhs
 * are FP64; the solves run in reduced precision and FP64 residuals on the
 * matrix correct the result:
 *     x = 0; r = rhs
 *     repeat: solve A d = r in reduced precision; x += d;
 *             r = rhs - A x (FP64)
 *     until ||r||_inf < tol ||rhs||_inf, per system, or max_steps solves.
 * With the compact FP32 state (BS_OPT_F32_STATE = 1, n <= 4096) each solve
 * is the split kernel with FP32 per-row state on the FP64 A and r (FP64
 * pivots; no FP32 copy of A is made) and adds d into x as it stores it.
 * Otherwise (longer systems, or BS_OPT_F32_STATE = 0) A32 = fl32(A) is
 * formed once and each step solves A32 d = fl32(r) with the fused FP32
 * band_solve.  Refinement converges when cond(A) times the FP32 rounding
 * unit is well below 1 (diagonally dominant ADI sweeps: a few steps to
 * 1e-12).  Systems that have converged are frozen; once all have, the
 * remaining launches return at once (no host synchronisation, so the call
 * can be captured in a graph).
 * diags (FP64, kind 3 needs c, d, a), rhs, x: batch-interleaved, n*ld each;
 * x is output only and must not alias rhs.  n >= 8.
 * steps[s]: FP32 solves the system took; relres[s]: final
 * ||r||_inf / ||rhs||_inf (0 for rhs = 0); info[s]: 0, -1 (not converged
 * within max_steps), -2 (residual not finite), i+1 (bad pivot of the
 * reduced-precision solve at row i) or -4 (as band_solve).
 * workspace: bs_workspace_bytes(BS_OP_REFINE, kind, BS_F64, ...) bytes,
 * 256-byte aligned, zero before its first use (as for band_solve; the call
 * leaves its counters at zero again). */
int32_t band_solve_refine(int32_t kind, int64_t n, int64_t batch, int64_t ld,
                          const double* const diags[5], const double* rhs, double* x,
                          double tol, int32_t max_steps, int32_t* steps, double* relres,
                          int32_t* info, void* workspace, size_t ws_bytes, void* stream);

/* MNPDM (Sec. 1): pentadiagonal solve in which the outer diagonals e and b
 * are given sparsely.  cda = {c, d, a} (batch-interleaved, n*ld each).
 * For system s, list entry k (0 <= k < kmax) is at outer_row[k*ld + s] (an
 * int32 row index, -1 = unused; used entries strictly ascending and first),
 * with values outer_e[k*ld + s] (coefficient e of that row) and
 * outer_b[k*ld + s] (coefficient b of that row).  All other e_i, b_i are 0.
 * Products with absent entries are skipped; on finite data the result equals
 * NPDM on the full diagonals.  kmax may be 0 (then the three list pointers
 * may be NULL).  dtype must be BS_F64.
 * Kernels: as band_solve -- by default the rows of a system are split over
 * lanes (n <= M*PW*TMAX of the first two PD variants; the diagonals e, b are
 * never read as arrays, so a row costs c, d, a, rhs and x only), the
 * workspace then holds the meeting counters (zero before first use, left
 * zero); otherwise one lane walks each system.  With an invalid list (info
 * -3) x of that system is unspecified. */
int32_t band_solve_mnpdm(int32_t dtype, int64_t n, int64_t batch, int64_t ld,
                         const void* const cda[3], int32_t kmax,
                         const int32_t* outer_row, const void* outer_e,
                         const void* outer_b, const void* rhs, void* x,
                         int32_t* info, void* workspace, size_t ws_bytes,
                         void* stream);

/* Stone method / SIP (Sec. 2, Algorithm 1) for pentadiagonal systems.
 * factors: ILU(0) factors from band_factor (kind 5), or NULL to have them
 *   computed into the workspace first.
 * x: in = x0 (zeros, previous time step, or a learned guess), out = result.
 * hb_s_L, hb_s_U: Hotelling-Bodewig steps X_{j+1} = X_j (2I - T X_j),
 *   X_0 = diag(T)^{-1} (Appendix), used in place of the L and U solves
 *   (Remark of Sec. 2).  A negative value keeps the exact substitution for
 *   that factor; both negative runs Algorithm 1 as written
 *   (x <- U^{-1} L^{-1} (K x + b), K = LU - A).  Otherwise the step is
 *   x <- x + X_U X_L (b - A x).  Allowed: s <= 6, or any s with 2^s >= n
 *   (HB is then exact and the exact substitution is used).
 * Stop when ||b - A x||_inf < tol * ||b||_inf (relative form of the paper's
 *   errorMargin test, checked before every step) or after max_iter steps.
 * iters[s] (int32), relres[s] (double, final relative residual) and info[s]
 * (0, -1, -2 or a pivot row + 1) are written per system.  dtype BS_F64.
 * Kernels: with HB for both factors (s_L, s_U >= 0, 2^s < n, and
 *   2^s_L + 2^s_U <= 96) the rows of a system are split over many lanes and
 *   every launch takes three steps over all rows where 2^s_L + 2^s_U <= 16,
 *   two where it is <= 48, else one; its last block to finish applies the
 *   stopping test at each step count in turn: about (max_iter + 1) / 3 (or
 *   / 2, / 1) launches are enqueued, and those after the last system has
 *   stopped return at once.  The iterates do not depend on the steps per
 *   launch.  With exact solves for both factors (Algorithm 1 as printed)
 *   and a batch too small to fill the GPU with one lane per system, each
 *   step is a row-parallel pass (residual, its norm, K x + b; the last block
 *   applies the test) and the split substitution of band_solve with
 *   factors: max_iter steps are enqueued, those after the last system has
 *   stopped return at once, and iterates, counts, residuals and statuses
 *   are bitwise those of one lane per system.  Otherwise one lane walks each
 *   system in one persistent launch.
 * workspace: bs_workspace_bytes(BS_OP_SIP, ...) bytes, 256-byte aligned; its
 *   contents need no initialisation.  x and rhs must not alias (BS_EINVAL). */
int32_t sip_solve(int32_t dtype, int64_t n, int64_t batch, int64_t ld,
                  const void* const diags[5], const void* factors,
                  const void* rhs, void* x, double tol, int32_t max_iter,
                  int32_t hb_s_L, int32_t hb_s_U, int32_t* iters,
                  double* relres, int32_t* info, void* workspace,
                  size_t ws_bytes, void* stream);

/* Explicit Hotelling-Bodewig approximate inverses of the ILU(0) factors
 * (Remark of Sec. 2; Appendix): for T = L (unit lower: l2, l1 below the
 * diagonal) and T = U (u0 on it, u1 and u2 = b above; for kind 3: l1, and u0,
 * u1 = a), s steps of X_{j+1} = X_j (2I - T X_j) from X_0 = diag(T)^{-1}.
 * X_s is a band matrix on T's side of the diagonal of width
 * K = min(n - 1, q (2^s - 1)), q = 2 (kind 5) or 1 (kind 3).
 * factors: band_factor's output for the same kind and ld, for systems whose
 *   info is 0 (a zero u0 makes X_0 = diag(U)^{-1} infinite and the system's
 *   X_U non-finite; nothing else reports it); diags: A's diagonals (only the
 *   upper ones are read: b for kind 5, a for kind 3).
 * XL (s_L steps) and XU (s_U steps): K + 1 planes of n*ld doubles in the
 *   batch-interleaved layout; plane d holds X_L[i, i - d] (XL) or
 *   X_U[i, i + d] (XU) at d*n*ld + i*ld + s, and 0 where i - d < 0 or
 *   i + d >= n.  Either may be NULL (that factor is skipped), not both.
 * Every product is summed over its inner index in ascending order with one
 *   rounding per multiply and per add, so each entry is bitwise the same
 *   recursion on dense n x n matrices.
 * workspace: hb_inverse_band_workspace_bytes(...) bytes, 8-byte aligned, no
 *   initialisation needed; (size_t)-1 for a bad kind, n or batch < 1,
 *   batch >= 2^28, ld < batch, n * ld >= 2^40, s < 0 or s > 30, or a grid
 *   beyond 2^31 - 1 blocks.  Device pointers, FP64.
 * BS_EINVAL for bad sizes or NULL / misaligned pointers, BS_EWORKSPACE when
 *   ws_bytes is short.  One launch per step and factor on `stream` while the
 *   output band is narrower than 16, two from there on. */
size_t hb_inverse_band_workspace_bytes(int32_t kind, int64_t n, int64_t batch, int64_t ld,
                                       int32_t s_L, int32_t s_U);
int32_t hb_inverse_band(int32_t kind, int64_t n, int64_t batch, int64_t ld,
                        const void* const diags[5], const double* factors, int32_t s_L,
                        int32_t s_U, double* XL, double* XU, void* workspace, size_t ws_bytes,
                        void* stream);

/* ---- Uneven batches --------------------------------------------------------
 * NPDM / NTDM (Sec. 1) for `count` systems of different lengths n[i] >= 8 in
 * one solve.  Layout: systems sorted by length (longest first) in groups of
 * 16; group g is an [n_g][16] block (n_g = its longest member), so row r of
 * system i is element offset[i] + 16 r of every array (e, c, d, a, b, rhs, x;
 * FP64), and its status goes to info[slot[i]] (info has 16 * groups
 * entries).  Elements of a block beyond a system's own length are never read
 * or written; corner slots as for band_solve.
 * Three launches over all groups (tile maps, per-system reduction, finish);
 * the tile shape is one of bs_varlen_variants() compiled variants
 * (bs_varlen_variant_shape: rows per lane M, lanes per system PW). */
typedef struct {
  int64_t count;       /* systems                                              */
  int64_t groups;      /* groups of 16                                         */
  int64_t elems;       /* elements every per-row array must hold               */
  int64_t tiles[4];    /* tiles of the whole batch for each variant (unused 0) */
  size_t table_bytes;  /* bytes of the device table                            */
  int64_t nmax;        /* longest system                                       */
} bs_varlen_info;

int32_t bs_varlen_variants(void);
int32_t bs_varlen_variant_shape(int32_t variant, int32_t shape[2]);

/* Host-only planning: fills *info, offset[count] and slot[count] (host
 * arrays, nullable) and, when table != NULL, the table (host buffer of
 * info->table_bytes) that the caller copies to a 256-byte-aligned device
 * buffer for the solves.  BS_EINVAL for count < 1 or any n[i] < 8. */
int32_t bs_varlen_layout(int64_t count, const int64_t* n, int64_t* offset, int32_t* slot,
                         void* table, bs_varlen_info* info);

/* Workspace bytes of band_solve_varlen for `variant` ((size_t)-1 if invalid);
 * no initialisation needed. */
size_t bs_varlen_workspace_bytes(int32_t kind, const bs_varlen_info* info, int32_t variant);

/* Solve every system of the uneven batch (asynchronous on `stream`).  info[slot]
 * as band_solve (0, or i+1 for the first bad pivot of the elimination). */
int32_t band_solve_varlen(int32_t kind, const bs_varlen_info* vinfo, const void* table,
                          int32_t variant, const void* const diags[5], const void* rhs, void* x,
                          int32_t* info, void* workspace, size_t ws_bytes, void* stream);

/* Autotuner: runs every variant `reps` times on the caller's batch (after one
 * warm-up each), writes the mean time per solve to ms[variant] (nullable) and
 * the fastest variant to *best.  Synchronises with `stream`; x and info hold
 * the last run's results.  The workspace must fit every variant. */
int32_t bs_varlen_tune(int32_t kind, const bs_varlen_info* vinfo, const void* table,
                       const void* const diags[5], const void* rhs, void* x, int32_t* info,
                       void* workspace, size_t ws_bytes, int32_t reps, float* ms,
                       int32_t* best, void* stream);

/* Layout conversion for callers whose lines are system-contiguous (the
 * lines along the fast axis of a row-major grid, as in the ADI sweeps of
 * Sec. 1): bs_pack_interleave writes dst[i*ld + s] = src[s*src_pitch + i]
 * and bs_unpack_interleave writes dst[s*dst_pitch + i] = src[i*ld + s], for
 * i < n, s < batch (FP64, device pointers, 8-byte aligned; the padding
 * columns s >= batch of an interleaved array are neither read nor written).
 * BS_EINVAL for n or batch < 1, ld < batch, a pitch < n, NULL pointers or
 * n, batch >= 2^26. */
int32_t bs_pack_interleave(int64_t n, int64_t batch, const double* src, int64_t src_pitch,
                           double* dst, int64_t ld, void* stream);
int32_t bs_unpack_interleave(int64_t n, int64_t batch, const double* src, int64_t ld,
                             double* dst, int64_t dst_pitch, void* stream);

/* Measurement helper, not a solver: out[i] = in[0][i] + ... + in[nin-1][i]
 * for i < count, as one streaming pass (16-byte non-temporal loads and
 * stores, no dependence between elements).  With nin = 6 it moves the bytes
 * of the fused PD solve (six arrays read, one written), so its rate is the
 * practical HBM ceiling of that traffic pattern on the device.  Device
 * pointers, 16-byte aligned; count even, 1 <= nin <= 6.  BS_EINVAL otherwise. */
int32_t bs_stream_probe(int64_t count, int32_t nin, const double* const in[6], double* out,
                        void* stream);

#ifdef __cplusplus
}
#endif

#endif /* BANDSOLVE_H */
