/*
 * bst.h -- C ABI of the MI355X block-sparse U(1) tensor library.
 *
 * The library implements the hot path of the tensor-network method of
 * arXiv:2401.01921 ("The Cytnx Library for Tensor Networks"): contraction of
 * Abelian (U(1) charge-conserving) block-sparse tensors -- charge-sector
 * matching, leg permutation and per-sector GEMMs -- and its use in the DMRG
 * two-site effective-Hamiltonian product H_eff.psi = L.psi.W.W.R inside a
 * Lanczos ground-state solver (Sec. "Benchmarks", Fig. Hpsi_fig; Sec.
 * "Eigenvalue decomposition", LinOp/Lanczos).
 *
 * Conventions shared by every call
 * --------------------------------
 * Leg (bond): a direction (+1 incoming, -1 outgoing), and a list of sectors,
 *   each an integer U(1) charge q and a dimension g >= 1 (Sec. "Bond with
 *   quantum numbers").  Charges on one leg need not be distinct.
 * Valid block: a tuple of sector indices (one per leg) whose flux, the sum of
 *   the incoming charges minus the sum of the outgoing charges, is zero
 *   (Sec. "UniTensor with Symmetries").  Only valid blocks are stored.
 * Block order: lexicographic in the sector indices with leg 0 most
 *   significant (the order of the block list printed for the rank-3 example
 *   of Sec. "Symmetric UniTensor").
 * Data layout: one flat buffer per tensor holding the valid blocks one after
 *   another in block order, each block a dense row-major array (Sec.
 *   "Tensor", App. "Contiguous").  Element type float64 at the boundary.
 * Labels: every leg has a label, unique within its tensor (Sec. "Viewing/
 *   Changing labels"); contraction sums over the labels two tensors share
 *   (Sec. "Tensor contraction").
 *
 * Memory and ownership
 * --------------------
 * Tensor descriptors and plans are host objects owned by the library and
 * released with bst_tensor_destroy / bst_plan_destroy.  All numeric buffers
 * (inputs, outputs, workspace) are device pointers owned by the caller; the
 * library never allocates, frees or retains device memory.  Plan tables are
 * uploaded into the caller's workspace on the first execute with that
 * workspace pointer and are assumed to stay there: after the caller frees,
 * reallocates or overwrites a workspace it used with a plan, it calls
 * bst_plan_forget_workspace(plan) before the plan's next call (a plan that
 * last used another pointer re-uploads by itself).  Work is enqueued on the
 * caller's HIP stream (passed as void*).
 *
 * Errors
 * ------
 * Every call returns a bst_status; on failure bst_last_error() returns a
 * message (thread-local, valid until the next call on the same thread).
 * No C++ exception crosses the ABI.  Faults of asynchronously enqueued
 * kernels surface on a later call as BST_E_DEVICE.
 */
#ifndef BST_H
#define BST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BST_OK = 0,
  BST_E_INVALID = 1,   /* bad argument: null pointer, dim < 1, bad rank, size */
  BST_E_DIRECTION = 2, /* contracted legs with the same direction (Sec. "Bond")  */
  BST_E_QNUM = 3,      /* contracted legs with different charge lists            */
  BST_E_DIM = 4,       /* contracted legs with different sector dims             */
  BST_E_LABEL = 5,     /* duplicate or unknown label                            */
  BST_E_NOBLOCK = 6,   /* sector tuple is not a valid block (Sec. "Accessing
                          elements of a symmetric tensor")                     */
  BST_E_STRUCTURE = 7, /* operands whose block structures do not fit the op    */
  BST_E_DEVICE = 8,    /* HIP runtime error                                    */
  BST_E_NOTCONV = 9    /* Lanczos produced no usable step                      */
} bst_status;

/* Arithmetic form of the per-sector products.  Inputs and outputs stay
 * float64; the form decides what the MFMA units compute:
 *   BST_FP64   float64 operands, float64 accumulate;
 *   BST_FP32   operands rounded to float32 (nearest-even), float32 accumulate;
 *   BST_BF16X3 each operand split a = a0 + a1 into bfloat16 (nearest-even,
 *              a1 = bf16(a - a0)); a0b0 + a0b1 + a1b0 accumulated in float32;
 *   BST_BF16X6 three-term split a0 + a1 + a2 and the six products whose
 *              plane orders add up to at most 2, accumulated in float32.
 * Intermediates of H_eff are float64 in BST_FP64 and float32 otherwise. */
typedef enum { BST_FP64 = 0, BST_FP32 = 1, BST_BF16X3 = 2, BST_BF16X6 = 3 } bst_precision;

typedef struct bst_tensor bst_tensor;
typedef struct bst_plan bst_plan;

/* ---- tensors (host metadata only) ------------------------------------ */

/* Builds the descriptor of a block-sparse tensor (Sec. "Bond with quantum
 * numbers", Sec. "Creating a symmetric UniTensor").
 *   rank     number of legs, 0..8
 *   dir      [rank] +1 (incoming) or -1 (outgoing)
 *   nsec     [rank] number of sectors of each leg, >= 1
 *   qn       [sum nsec] charges, leg by leg
 *   dim      [sum nsec] sector dims, leg by leg, each >= 1
 *   labels   [rank] NUL-terminated labels, unique
 *   out      receives the descriptor
 * A tensor with no valid block is legal (numel 0).  Errors: BST_E_INVALID,
 * BST_E_LABEL. */
bst_status bst_tensor_create(int32_t rank, const int32_t* dir, const int32_t* nsec,
                             const int32_t* qn, const int64_t* dim,
                             const char* const* labels, bst_tensor** out);

/* The same with one or more abelian symmetries (Sec. "Symmetry and quantum
 * numbers", Sec. "Creating bonds with quantum numbers"): every sector
 * carries one charge per symmetry.  A U(1) component combines by addition;
 * a Z_n component by addition modulo n; both are negated on outgoing legs.
 * A block is valid when every component of its combined charge vanishes
 * (exactly for U(1), modulo n for Z_n).
 *   nsym     number of symmetries, 1..8
 *   sym      [nsym] 0 for U(1), n >= 2 for Z_n
 *   qn       [sum nsec * nsym] charges, sector by sector, nsym per sector;
 *            Z_n charges in [0, n)
 * The other arguments are those of bst_tensor_create; bst_tensor_create is
 * this call with nsym = 1 and sym = {0}.  Contraction requires equal
 * symmetries on the contracted legs (BST_E_QNUM otherwise).  Errors:
 * BST_E_INVALID (bad nsym or modulus), BST_E_QNUM (a Z_n charge out of
 * range), BST_E_LABEL. */
bst_status bst_tensor_create_sym(int32_t rank, const int32_t* dir, const int32_t* nsec,
                                 int32_t nsym, const int32_t* sym, const int32_t* qn,
                                 const int64_t* dim, const char* const* labels, bst_tensor** out);
bst_status bst_tensor_destroy(bst_tensor* t);

/* The symmetries of a tensor: their number, and (if moduli is non-null) the
 * moduli (0 = U(1)) into moduli[cap].  Error BST_E_INVALID if cap is short. */
bst_status bst_tensor_symmetry(const bst_tensor* t, int32_t* nsym, int32_t* moduli, int32_t cap);

/* All charges of a leg, sector by sector, nsym per sector, into
 * qn[nsec * nsym] (bst_tensor_leg gives the first component only). */
bst_status bst_tensor_leg_charges(const bst_tensor* t, int32_t leg, int32_t* qn);

/* Rank, number of valid blocks and total element count. */
bst_status bst_tensor_info(const bst_tensor* t, int32_t* rank, int64_t* nblocks, int64_t* numel);

/* Leg description: direction, sector count, and (if the arrays are non-null)
 * the charges (first symmetry) and dims, and the label copied into a buffer
 * of label_cap bytes.  Error BST_E_INVALID for a bad leg index or a short buffer. */
bst_status bst_tensor_leg(const bst_tensor* t, int32_t leg, int32_t* dir, int32_t* nsec,
                          int32_t* qn, int64_t* dim, char* label, size_t label_cap);

/* Block b (0-based, canonical order): sector indices [rank], shape [rank]
 * and element offset into the flat buffer.  Any output pointer may be null.
 * Error BST_E_INVALID for b out of range. */
bst_status bst_tensor_block(const bst_tensor* t, int64_t b, int32_t* qn_idx, int64_t* shape,
                            int64_t* offset);

/* Block number of the sector tuple qn_idx [rank]; BST_E_NOBLOCK if the tuple
 * has nonzero flux (Sec. "Accessing elements of a symmetric tensor"). */
bst_status bst_tensor_find_block(const bst_tensor* t, const int32_t* qn_idx, int64_t* b);

/* ---- network contraction order ------------------------------------------ */

/* Optimal pairwise contraction order of a network of n tensors (Sec.
 * "Network", "Setting the contraction order"): dynamic programming over
 * subsets with cost capping.  Cost of one pairwise contraction = product of
 * the dims of every index it involves (each once); the order minimises the
 * sum.  Host only.
 *   n       number of tensors, 1..16
 *   nlegs   [n] number of indices of each tensor
 *   legs    [sum nlegs] index ids (0..nid-1), tensor by tensor; an id on
 *           two tensors is contracted, an id on one tensor stays open
 *   nid     number of distinct ids, 0..64
 *   dims    [nid] total dim of each id, >= 1
 *   pairs   [2 (n-1)] receives the steps in order: step k contracts nodes
 *           pairs[2k] and pairs[2k+1], where nodes 0..n-1 are the inputs
 *           and node n + k is the result of step k (null: not written)
 *   cost    receives the total cost (null: not written)
 * Errors: BST_E_INVALID (sizes, an id on more than two tensors or twice on
 * one tensor). */
bst_status bst_network_order(int32_t n, const int32_t* nlegs, const int32_t* legs, int32_t nid,
                             const int64_t* dims, int32_t* pairs, double* cost);

/* ---- plans ------------------------------------------------------------ */

/* Permute (Sec. "Permute", App. "Contiguous"): new leg i is the old leg
 * labelled new_order[i]; every block is transposed accordingly and the
 * blocks are stored in the canonical order of the new leg order.
 *   in         input descriptor
 *   new_order  [rank] labels
 *   out_meta   receives the output descriptor (caller destroys)
 *   plan       receives the plan; execute with in = {X}, out = {Y}.
 * Errors: BST_E_LABEL. */
bst_status bst_permute_plan(const bst_tensor* in, const char* const* new_order,
                            bst_tensor** out_meta, bst_plan** plan);

/* Contract A and B over all labels they share (Sec. "Tensor contraction").
 * Each shared leg must have opposite directions (BST_E_DIRECTION) and the
 * same charge list (BST_E_QNUM) and dims (BST_E_DIM) in the same order.  The
 * result has A's free legs in A's order followed by B's free legs in B's
 * order and holds every valid block (zero where nothing contributes).
 * Execute with in = {A, B}, out = {C}. */
bst_status bst_contract_plan(const bst_tensor* A, const bst_tensor* B, bst_precision prec,
                             bst_tensor** C_meta, bst_plan** plan);

/* Two-site effective Hamiltonian (Sec. "Benchmarks", Fig. Hpsi_fig):
 *   out[a,s1,s2,b] = sum L[a,w1,a'] W1[w1,s1,t1,w2] W2[w2,s2,t2,w3]
 *                        R[b,w3,b'] psi[a',t1,t2,b']
 * contracted in the order L -> psi -> W1 -> W2 -> R.  Leg order of the
 * operands: L[a, w, a'], W[w_left, s_ket, s_bra, w_right], R[b, w, b'],
 * psi[a, s1, s2, b].  The pairs (L.a', psi.a), (L.w, W1.w_left),
 * (W1.s_bra, psi.s1), (W1.w_right, W2.w_left), (W2.s_bra, psi.s2),
 * (W2.w_right, R.w), (R.b', psi.b) must be contractible; L.a, W1.s_ket,
 * W2.s_ket and R.b must equal psi's legs, so out has psi's block table.
 * Execute with in = {L, W1, W2, R, psi}, out = {out}. */
bst_status bst_heff_plan(const bst_tensor* L, const bst_tensor* W1, const bst_tensor* W2,
                         const bst_tensor* R, const bst_tensor* psi, bst_precision prec,
                         bst_plan** plan);

/* Merges n H_eff plans into one: each step of all n applies runs as one
 * grouped launch.  Execute with in = {L_0, W1_0, W2_0, R_0, psi_0, L_1, ...}
 * (5n pointers) and out = {out_0, ..., out_{n-1}}.  The sub-plans stay owned
 * by the caller and may be destroyed after this call. */
bst_status bst_heff_batch_plan(int32_t n, const bst_plan* const* plans, bst_plan** batch);

/* Device workspace the plan needs (bytes, 256-byte aligned pointer). */
bst_status bst_plan_workspace(const bst_plan* p, size_t* bytes);

/* Algorithmic work of one execute: flops (2mnk over valid block products,
 * all steps) and the number of GEMM problems and tiles of the main steps. */
typedef struct {
  double flops;
  double gemm_flops;
  double bytes;          /* algorithmic HBM bytes at float64 storage          */
  int64_t gemm_problems;
  int64_t gemm_tiles;
  int64_t launches;      /* kernels enqueued per execute                      */
  int32_t nsteps;        /* steps (kernel launches) of one execute            */
} bst_plan_stats;
bst_status bst_plan_info(const bst_plan* p, bst_plan_stats* st);

/* One step (one kernel launch) of a plan: its name, algorithmic flops, and
 * algorithmic HBM bytes (each operand read once, each result written once)
 * with float64 intermediates and with float32 intermediates. */
typedef struct {
  char name[32];
  double flops;
  double bytes_fp64;
  double bytes_fp32;
  int64_t items;         /* tiles / work items of the launch                   */
} bst_step_info;
bst_status bst_plan_step_info(const bst_plan* p, int32_t step, bst_step_info* info);

/* Overrides the arithmetic form of an H_eff (or contract) plan. */
bst_status bst_plan_set_precision(bst_plan* p, bst_precision prec);

/* Record the plan's kernels in a hipGraph on the next execute and replay the
 * graph afterwards (on = 1), or launch kernels directly (on = 0). */
bst_status bst_plan_use_graph(bst_plan* p, int32_t on);

/* Enqueues the plan on stream (a hipStream_t, or null for the default
 * stream).  in / out are device pointers to float64 data in canonical
 * layout; ws points to bst_plan_workspace() bytes of device memory that no
 * other concurrent execute uses.  Returns after enqueueing. */
bst_status bst_execute(bst_plan* p, const void* const* in, void* const* out, void* ws,
                       void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * bst_execute with the workspace taken from a fixed device array of
 * BST_STATIC_WORKSPACE_BYTES that the library holds on every device it runs
 * on until the process ends.  No allocation and no graph capture (kernels are
 * launched directly whatever bst_plan_use_graph says).  The array needs no
 * initial contents: every kernel writes what it later reads.  All calls on a
 * device share that device's array, so calls that overlap on one device
 * (other streams or threads) race; serialise them.  Errors: BST_E_INVALID if
 * bst_plan_workspace of the plan exceeds BST_STATIC_WORKSPACE_BYTES (nothing
 * is enqueued), and the errors of bst_execute. */
#define BST_STATIC_WORKSPACE_BYTES (64u << 20)
bst_status bst_execute_static(bst_plan* p, const void* const* in, void* const* out, void* stream);

/* Times every compiled tile shape of each GEMM step on the given buffers,
 * keeps the fastest per step and (if the environment variable BST_TUNE_CACHE
 * names a file) records the choice there.  Each candidate is timed after a
 * read of a 512 MiB buffer (allocated for the call, freed before it returns)
 * and after the steps before it, as an iterative caller would run it.  With
 * FP64 on padded layouts it also chooses between the float64-panel and the
 * per-block-pair kernels, and with BF16X3 between the two-kernel L.psi + MPO
 * steps and the fused kernel, by whole-apply time; BST_FP64_PANELS /
 * BST_FP64_BLOCKS and BST_FUSED_MPO=0/1 fix those choices instead.  Both
 * choices go into the tile cache.  Synchronises the stream. */
bst_status bst_plan_autotune(bst_plan* p, const void* const* in, void* const* out, void* ws,
                             void* stream, int32_t reps);

/* Records the plan's chosen tile shapes (from bst_plan_autotune or
 * bst_plan_set_tile) in the file named by BST_TUNE_CACHE, keeping the file's
 * entries for other structures; plans created later with the same GEMM
 * structure start from these choices.  Error BST_E_INVALID if the variable
 * is not set.  Host only. */
bst_status bst_plan_record_tiles(const bst_plan* p);

/* Number of compiled GEMM kernel variants (tile shape, with or without LDS
 * staging) available to the plan's GEMM steps in the given form, and a manual
 * choice of one of them for every GEMM step (0 <= tile < count). */
bst_status bst_plan_tile_count(const bst_plan* p, bst_precision form, int32_t* count);
bst_status bst_plan_set_tile(bst_plan* p, bst_precision form, int32_t tile);

/* Tile shapes chosen for the plan's GEMM steps, as text ("step:BMxBN;...")
 * written into buf (NUL-terminated, truncated to cap). */
bst_status bst_plan_tiles(const bst_plan* p, char* buf, size_t cap);

/* Per-step kernel times (ms) of the last bst_plan_profile call. */
bst_status bst_plan_profile(bst_plan* p, const void* const* in, void* const* out, void* ws,
                            void* stream, int32_t reps, double* step_ms, int32_t cap,
                            int32_t* nsteps);

bst_status bst_plan_destroy(bst_plan* p);

/* Makes the plan's next call upload its tables into the workspace again
 * (after the caller changed or reallocated the workspace memory), and drops
 * a captured hipGraph.  Never fails on a valid plan. */
bst_status bst_plan_forget_workspace(bst_plan* p);

/* ---- Lanczos ground state (Sec. "Eigenvalue decomposition") ----------- */

typedef struct {
  int32_t flags;        /* in: BST_LANCZOS_TIMING records HIP events around
                           every kernel and fills kernel_ms / kernel_calls    */
  int32_t steps;        /* Lanczos steps kept (<= nsteps; fewer on breakdown) */
  double theta;         /* lowest Ritz value of the tridiagonal matrix        */
  double beta_min;      /* smallest off-diagonal beta of the kept steps       */
  double residual;      /* |H y - E y| with the float64 operator, |y| = 1     */
  double alpha[128];    /* diagonal of the tridiagonal matrix (first 128)     */
  double beta[128];     /* off-diagonal (first 128)                           */
  /* Summed kernel time (ms) and launch count per kernel class, with
   * BST_LANCZOS_TIMING: 0 L.psi GEMM, 1 MPO apply, 2 T3.R GEMM, 3 MPO
   * coefficients and bf16 splits, 4 dot kernel (default schedule: u_j.z;
   * three-pass: V^T w), 5 basis pass (default: the step's single pass over
   * the basis; three-pass: w -= V c and V^T w), 6 third pass (three-pass
   * only: w -= V d and |w|^2), 7 other vector and scalar kernels.         */
  double kernel_ms[8];
  int32_t kernel_calls[8];
} bst_lanczos_info;
#define BST_LANCZOS_TIMING 1
/* Run the textbook schedule (three passes over the basis per step) instead
 * of the default single pass with delayed projection. */
#define BST_LANCZOS_THREE_PASS 2
/* Store the Krylov rows, and H u_j, as float32 with the BF16X3 / BF16X6
 * matvec forms (every dot, coefficient, reduction and the tridiagonal solve
 * stay float64).  By default every form keeps float64 rows, i.e. the full
 * reorthogonalisation runs on float64 vectors; the three-pass schedule and
 * the FP64 / FP32 forms ignore this flag. */
#define BST_LANCZOS_F32_BASIS 4
/* Out (set in info->flags on return): H u_j was kept as float32 during the
 * steps.  With BF16X3 / BF16X6 matvecs the products accumulate in float32,
 * so this stores the same values in half the bytes; float64 rows and every
 * dot and scalar stay float64.  BST_LANCZOS_Z64 in the environment keeps
 * H u_j float64. */
#define BST_LANCZOS_Z32 16

/* Workspace of bst_lanczos_ground for a plan and step count. */
bst_status bst_lanczos_workspace(const bst_plan* heff, int32_t nsteps, size_t* bytes);

/* Lowest eigenpair of the H_eff of `heff` (a bst_heff_plan), which must be
 * symmetric.  Lanczos with full reorthogonalisation: v1 = psi0/|psi0|; per
 * step w = H v_j in the form `matvec_prec`, w projected against all
 * previous vectors with float64 arithmetic (the reference order: two classical
 * Gram-Schmidt passes), alpha_j, beta_j = |w|, v_{j+1} = w/beta_j; the steps stop at the first
 * beta_j <= 1e-12 max(|alpha|, beta_j).  By default a step reads the basis
 * once: the operator is applied to the residual of the previous step before
 * its full projection, the image of that projection under the operator is
 * taken from the Lanczos relation, and the projection is applied (finishing
 * v_j) in the same pass that forms the three-term residual and measures it
 * against the basis (delayed reorthogonalisation after Swirydowicz et al.
 * 2021 and Bielich et al. 2022); alpha and beta equal those of two full
 * classical Gram-Schmidt passes in exact arithmetic.
 * BST_LANCZOS_THREE_PASS in info->flags runs the textbook order (three
 * passes over the basis per step).  The basis rows are float64 unless
 * BST_LANCZOS_F32_BASIS is set with BF16X3 / BF16X6.  The
 * float64 tridiagonal eigensolve (Sturm bisection, inverse iteration) gives
 * the Ritz pair (theta, y = V s).  With refine != 0, one float64 apply gives
 * E = y.Hy / y.y; otherwise E = theta.
 *   ops        {L, W1, W2, R} device pointers (float64, canonical layout)
 *   psi0       device pointer, start vector (psi's layout)
 *   psi_out    device pointer, receives y / |y| (may alias nothing else)
 *   energy     receives E
 *   info       may be null; info->flags is read on entry
 * Blocks until the result is on the host.  BST_E_NOTCONV if psi0 is zero. */
bst_status bst_lanczos_ground(bst_plan* heff, const void* const* ops, const void* psi0,
                              int32_t nsteps, bst_precision matvec_prec, int32_t refine,
                              void* psi_out, double* energy, bst_lanczos_info* info, void* ws,
                              void* stream);

/* ---- complex float64 data ---------------------------------------------- */

/* Complex element type (Sec. "Creating a non-symmetric UniTensor",
 * paragraph "Complex elements and data types"; used by the quantum-circuit
 * simulation of App. "Quantum Circuit Simulation"): the same
 * block structure and block order, each element two float64 (real, then
 * imaginary), so a complex tensor of numel elements occupies 2 * numel
 * doubles.  Plans built by the calls below take and produce such buffers in
 * bst_execute; everything else about them is as for their float64
 * counterparts.  Labels beginning with "#re" are reserved (BST_E_LABEL). */

/* Permute of complex data (bst_permute_plan semantics; rank 1..7). */
bst_status bst_permute_plan_c128(const bst_tensor* in, const char* const* new_order, bst_tensor** out_meta,
                                 bst_plan** plan);

/* Contraction of complex tensors (bst_contract_plan semantics and checks;
 * A rank 1..7, B rank 1..6, C rank at most 7): C = sum A B with complex
 * products.  Runs as the
 * real grouped GEMM of A's interleaved (re, im) form with B expanded once
 * per element into [[Br, Bi], [-Bi, Br]] (a workspace buffer of 4 * numel(B)
 * doubles), so every form of `prec` applies to the real arithmetic. */
bst_status bst_contract_plan_c128(const bst_tensor* A, const bst_tensor* B, bst_precision prec,
                                  bst_tensor** C_meta, bst_plan** plan);

/* ---- symmetric SVD with truncation (Sec. "Singular value decomposition":
 *      paragraphs "With truncation" and "SVD for symmetric UniTensor") ------ */

/* Opaque plan of the SVD of one tensor structure. */
typedef struct bst_svd bst_svd;

/* Plans the SVD of tensor M seen as a matrix whose rows are its first
 * rowrank legs and whose columns are the others (Sec. "Matrix form of a
 * UniTensor").  The matrix splits into one block matrix M_q per charge q of
 * the new bond: its rows are the row-leg sector tuples of combined flux q
 * (sum of direction times charge, modulo n for Z_n), its columns the
 * column-leg tuples of flux -q, tuples in lexicographic order and each
 * tuple's elements row-major.  The sectors of the new bond are ordered as
 * their charges first appear over the column tuples in lexicographic order.
 * Host bookkeeping only.  Errors: BST_E_INVALID (null, rowrank outside
 * 1..rank-1, a sector matrix above 2^31 rows or columns). */
bst_status bst_svd_plan(const bst_tensor* M, int32_t rowrank, bst_svd** out);

/* Sector count, total singular values (sum of min(rows, cols)) and the
 * workspace bytes the plan's calls need (256-byte aligned device memory,
 * caller-owned; the plan's tables are uploaded on first use of a pointer,
 * see bst_svd_forget_workspace). */
bst_status bst_svd_info(const bst_svd* p, int32_t* nsectors, int64_t* nvalues, size_t* ws_bytes);

/* Charge (nsym components) and shape of sector k of the new bond. */
bst_status bst_svd_sector(const bst_svd* p, int32_t k, int32_t* charge, int64_t* rows, int64_t* cols);

/* Enqueues the full SVD of every sector matrix of M (device pointer, M's
 * layout) into the workspace: one-sided Jacobi on the tall orientation of
 * each M_q, float64, sweeps until no pair of columns is rotated
 * (|x_i.x_j| <= 4 eps sqrt(p) |x_i||x_j|, p the long side, at most 60
 * sweeps); singular values sorted in descending order per sector.  The
 * singular vectors of a zero singular value are returned as zero vectors
 * on the long side.  Results stay in the workspace for bst_svd_truncate
 * and bst_svd_write.  A sector matrix above 128 KiB (long side x short side
 * float64 values) runs each round of its sweeps as one launch across the
 * device; the call then waits for the stream after every sweep to test
 * convergence (otherwise it only enqueues), and the other sectors' sweeps
 * run meanwhile on a second stream the plan keeps (default priority, made
 * on first use on the current device; joined to `stream` before the call
 * returns). */
bst_status bst_svd_execute(bst_svd* p, const void* M, void* ws, void* stream);

/* Chooses the kept singular values across all sectors (after
 * bst_svd_execute on the same workspace and stream): every sector k keeps
 * its min(min_blockdim[k], rows, cols) largest values (min_blockdim may be
 * null: zeros); the remaining room up to keepdim goes to the largest other
 * values that are not below err, ties to the earlier sector, then the
 * earlier value (the values are not normalised).  kept (host, nsectors
 * entries) receives the count per sector, s_err (host, may be null) the
 * largest value not kept (0 if none).  Blocks until the counts are on the
 * host.  Errors: BST_E_INVALID (keepdim < 0, err < 0 or NaN, a negative
 * min_blockdim). */
bst_status bst_svd_truncate(bst_svd* p, int64_t keepdim, double err, const int64_t* min_blockdim,
                            void* ws, void* stream, int64_t* kept, double* s_err);

/* Descriptors of the truncated factors for the counts kept[nsectors]:
 * U[row legs..., bond] with the new bond outgoing and V^dagger[bond,
 * column legs...] with it incoming, both labelled `bond`, whose sectors are
 * the sectors with kept > 0 (in bond order) with dims kept[k]; a sector
 * truncated to nothing leaves the bond.  Errors: BST_E_INVALID (a count
 * outside 0..min(rows, cols), every sector empty), BST_E_LABEL (bond equals
 * a leg label). */
bst_status bst_svd_factors(const bst_svd* p, const int64_t* kept, const char* bond, bst_tensor** U,
                           bst_tensor** Vd);

/* Writes the kept columns of U, the kept singular values and the kept rows
 * of V^dagger (device pointers, layouts of bst_svd_factors; S receives
 * sum(kept) values, sector by sector in bond order, descending inside a
 * sector).  absorb = 1 multiplies the values into U's columns, 2 into
 * V^dagger's rows, 0 leaves both orthonormal.  Blocks until the write has
 * run.  Errors: BST_E_INVALID. */
bst_status bst_svd_write(bst_svd* p, const int64_t* kept, int32_t absorb, void* U, void* S, void* Vd,
                         void* ws, void* stream);

/* Convergence report of the last bst_svd_execute on this workspace: per
 * sector, in sector order, the number of Jacobi sweeps that rotated at
 * least one pair (nsectors int32 values into host memory `sweeps`).  A
 * converged sector ran one more sweep that rotated nothing; 60, the cap,
 * means it stopped there; a sector with one column reports 0.  Waits for
 * `stream`.  Errors: BST_E_INVALID. */
bst_status bst_svd_sweeps(const bst_svd* p, const void* ws, void* stream, int32_t* sweeps);

/* Forget which workspace holds the plan's tables (call before reusing a
 * plan after freeing or overwriting its workspace). */
bst_status bst_svd_forget_workspace(bst_svd* p);

/* Release an SVD plan (null is allowed; always BST_OK). */
bst_status bst_svd_destroy(bst_svd* p);

/* ---- calibration (the device's practical rates, measured with this
 *      library's own code) ------------------------------------------------ */

/* Workgroups of every calibration launch (256 lanes each). */
int32_t bst_calib_grid(void);

/* Enqueues a streaming copy of `bytes` (a multiple of 16) from src to dst,
 * both 16-byte aligned device pointers: every byte is read once and written
 * once with 16-byte non-temporal accesses.  Errors: BST_E_INVALID. */
bst_status bst_calib_copy(const void* src, void* dst, size_t bytes, void* stream);

/* Enqueues a streaming read of `bytes` (a multiple of 16) at src; each
 * workgroup writes the sum of its elements to partial[bst_calib_grid()]
 * (device), so the reads cannot be dropped.  Errors: BST_E_INVALID. */
bst_status bst_calib_read(const void* src, size_t bytes, double* partial, void* stream);

/* Enqueues iters rounds of eight independent MFMA instructions per wave on
 * register operands, on every wave of bst_calib_grid() workgroups of 4 waves:
 * form BST_FP64 uses the 16x16x4 float64 instruction, BST_BF16X3 the
 * 16x16x32 bfloat16 one (float32 accumulate).  *flops receives the flops of
 * the launch; out (device) receives 256 * bst_calib_grid() doubles.
 * Errors: BST_E_INVALID for another form or iters < 1. */
bst_status bst_calib_mfma(bst_precision form, int64_t iters, double* out, double* flops,
                          void* stream);

/* Message of the last failed call on this thread ("" if none). */
const char* bst_last_error(void);

/* Library version string. */
const char* bst_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BST_H */
