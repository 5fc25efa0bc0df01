/*
 * fx.h - C ABI of the fused element-wise expression library (libfx.so) for
 * AMD Instinct MI355X (gfx950).
 *
 * What it implements: the compile-time expression fusion of Curtin, Edel and
 * Sanderson, "Fast GPU Linear Algebra via Compile Time Expression Fusion".
 * An expression such as Z = X % Y + 2*W (% = Schur product, Sec. 4) is
 * captured as a C++ type (Sec. 3, the X.t()+3 example), and one kernel reads
 * every input once and writes the output once, with no temporaries (Sec. 3,
 * skeleton kernels; Sec. 5, "single pass").  The fused entry points below
 * are instances of that front end for fixed expressions; fx_tape_* (when
 * present) evaluates trees only known at run time.
 *
 * Conventions shared by every call:
 *   - Matrices are dense, column-major, leading dimension n_rows: element
 *     (r, c) lives at linear index r + c*n_rows (Sec. 3, element access of a
 *     plain matrix).  Vectors are n x 1.
 *   - All data pointers are DEVICE pointers owned by the caller.  The
 *     library never frees or retains them after the enqueued work completes.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *     enqueues work on it and returns at once; results are ready when the
 *     stream is synchronised (Sec. 2: asynchronous dispatch, synchronisation
 *     on demand, cf. coot_synchronise()).
 *   - Scalar reduction results are written to device memory as FP64 so the
 *     call stays asynchronous; reading them synchronises.
 *   - `cfg` may be NULL; any zero field is chosen by the library.
 *   - Every call returns an fx_status.  Arguments are validated on the host
 *     before anything is enqueued; on error nothing is enqueued and
 *     fx_last_error() (thread-local) describes the problem.  Faults inside a
 *     kernel surface at the caller's next synchronisation.
 *   - n = 0 (or an empty shape) is a valid no-op; a scalar reduction of
 *     nothing writes 0.
 *   - Pointers need only the alignment of their element type; 16-byte
 *     vector loads are used when every pointer of a call is 16-byte aligned,
 *     element-wise loads otherwise.
 *   - An element-wise output may be exactly one of the inputs (in place);
 *     partial overlap is not allowed.
 *   - Inputs are read with streaming (nontemporal) loads.  An element-wise
 *     output larger than 256 MiB (MI355X's last-level cache) that is written
 *     with 16-byte vectors is written with streaming stores, so it is not
 *     left in that cache; smaller outputs use ordinary stores.
 *
 * Workspaces: reductions that combine results across blocks take a caller
 * allocated device workspace of fx_workspace_bytes() bytes, which must be
 * zero-filled once before its first use; the library leaves it zeroed again
 * after every call (its counters reset themselves).  One workspace must not
 * be used by two calls that may run concurrently.
 */
#ifndef FX_H
#define FX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage types.  BF16/F16 are computed in FP32 (low-precision storage,
 * Sec. 5 future work); F64 in FP64; U32 in u32 arithmetic mod 2^32. */
typedef enum { FX_F32 = 0, FX_F64 = 1, FX_BF16 = 2, FX_F16 = 3, FX_U32 = 4 } fx_dtype;

typedef enum {
  FX_OK = 0,
  FX_E_ARG = 1,         /* NULL pointer, negative size, bad enum value */
  FX_E_SHAPE = 2,       /* incompatible dimensions */
  FX_E_DTYPE = 3,       /* dtype not supported by this call */
  FX_E_WORKSPACE = 4,   /* workspace missing or too small */
  FX_E_HIP = 5,         /* HIP runtime error (text in fx_last_error) */
  FX_E_UNSUPPORTED = 6, /* launch configuration outside the compiled set */
  FX_E_CONFIG = 7       /* malformed launch configuration */
} fx_status;

/* Launch configuration; 0 in a field means "library default".
 *   block:     threads per block, a multiple of 64 in [64, 512]
 *   ept:       independent vector loads per input per thread, 1/2/4/8
 *              (tapes: 1/2/4)
 *   vec_bytes: bytes per vector load: one element or 16; tapes over types
 *              of at most 4 bytes also take 8.  Other values: FX_E_UNSUPPORTED
 *   split:     element-wise and full reductions: number of blocks (grid);
 *              column sums: blocks per column; row sums: column chunks. */
typedef struct { int32_t block, ept, vec_bytes, split; } fx_launch;

typedef struct { int64_t n_rows, n_cols; } fx_shape;

/* Reduction kinds (Sec. 3 names accu(); the others follow Armadillo, whose
 * API the library mirrors, Sec. 2). */
typedef enum {
  FX_R_ACCU = 1,   /* sum of all elements -> double             */
  FX_R_COLSUM = 2, /* sum(E, 0): 1 x n_cols, accumulator dtype  */
  FX_R_ROWSUM = 3, /* sum(E, 1): n_rows x 1, accumulator dtype  */
  FX_R_NORM = 4,   /* Frobenius norm sqrt(sum E^2) -> double    */
  FX_R_DOT = 5     /* sum A_i * B_i -> double                   */
} fx_reduce_kind;

/* Element-wise operators of the unfused baseline (one kernel each). */
typedef enum {
  FX_OP_NEG = 1, FX_OP_ABS = 2, FX_OP_EXP = 3, FX_OP_SQRT = 4,      /* unary  */
  FX_OP_LOG = 5, FX_OP_TANH = 6, /* unary, the paper's Sec. 4 expressions */
  FX_OP_ADD = 10, FX_OP_SUB = 11, FX_OP_SCHUR = 12, FX_OP_DIV = 13, /* binary */
  FX_OP_XOR = 14,                                                   /* u32    */
  FX_OP_SADD = 20,  /* k + A */
  FX_OP_SMUL = 21,  /* k * A */
  FX_OP_SDIV = 22,  /* A / k */
  FX_OP_SRDIV = 23, /* k / A */
  FX_OP_SSUB = 24,  /* A - k */
  FX_OP_SRSUB = 25, /* k - A */
  FX_OP_SPOW = 26,  /* pow(A, k); k = 1..4 evaluate as products of A, as in
                       the fused expressions */
  FX_OP_LEAF = 30,  /* tape node: an input array     */
  FX_OP_CONST = 31  /* tape node: a scalar constant  */
} fx_op;

/* The workload expressions, for fx_unfused() and fx_workspace_bytes(). */
typedef enum {
  FX_EXPR_C1_Z = 1,       /* Z = X % Y + 2*W  (U32: Z = (X ^ Y) + 3*W)  */
  FX_EXPR_ACCU_XY = 2,    /* accu(X % Y)                                */
  FX_EXPR_C2_Z = 3,       /* Z = (X + Y) % exp(-abs(W)) / (1 + X % X)   */
  FX_EXPR_C2_COLSUM = 4,  /* sum(C2 expression, 0)                      */
  FX_EXPR_C2_ROWSUM = 5,  /* sum(C2 expression, 1)                      */
  FX_EXPR_NORM_DIFF = 6,  /* norm_fro(X - Y)                            */
  FX_EXPR_COLSUM_XY = 7,  /* sum(X % Y, 0)                              */
  FX_EXPR_AXY_EXPW = 8    /* Z = a*X % Y + exp(-W)                      */
} fx_expr_id;

/* ---- library ------------------------------------------------------------ */

/* Version string; never NULL. */
const char* fx_version(void);

/* Text of the last error raised on the calling thread ("" if none). */
const char* fx_last_error(void);

/* Blocks until all work enqueued on `stream` has finished (the library's
 * coot_synchronise(), Sec. 2).  Returns FX_E_HIP if that work faulted. */
int fx_synchronize(void* stream);

/* Workspace bytes needed by reduction `kind` (FX_R_*) over an expression of
 * storage dtype `dt` and shape `shape` under launch configuration `cfg`
 * (NULL = defaults).  The size covers both the fused calls and a run-time
 * tape of the same kind (whose unset fields take the interpreter's
 * defaults).  Returns 0 on bad arguments. */
size_t fx_workspace_bytes(int kind, fx_dtype dt, fx_shape shape, const fx_launch* cfg);

/* The configuration the library would use for reduction kind `kind`
 * (0 = element-wise) with these arguments, written to *out.  Returns
 * FX_E_CONFIG / FX_E_ARG on invalid input. */
int fx_resolve_launch(int kind, fx_dtype dt, fx_shape shape, const fx_launch* cfg,
                      fx_launch* out);

/* ---- fused entry points (compile-time expression templates) --------------
 * Each is one kernel launch that reads each distinct input once and writes
 * its output once (Sec. 3, skeleton kernels; Sec. 5). */

/* Z[i] = X[i]*Y[i] + 2*W[i] for i < n (FP dtypes);
 * Z[i] = (X[i] ^ Y[i]) + 3*W[i] mod 2^32 (FX_U32). */
int fx_c1_z(fx_dtype dt, const void* X, const void* Y, const void* W, void* Z,
            int64_t n, const fx_launch* cfg, void* stream);

/* Z = a*X % Y + exp(-W), with a rounded to the compute type. FP dtypes. */
int fx_axy_expw(fx_dtype dt, double a, const void* X, const void* Y, const void* W,
                void* Z, int64_t n, const fx_launch* cfg, void* stream);

/* *d_out = accu(X % Y) = sum_i X[i]*Y[i], as FP64 (FP dtypes) or, for
 * FX_U32, the full u64 sum stored in d_out's 8 bytes.  Per-thread sums are
 * compensated (Neumaier) in the compute type and combined in FP64 in a fixed
 * order by the last block to finish.  ws: fx_workspace_bytes(FX_R_ACCU). */
int fx_accu_xy(fx_dtype dt, const void* X, const void* Y, int64_t n, void* d_out,
               void* ws, size_t ws_bytes, const fx_launch* cfg, void* stream);

/* dot(X, Y): the same value as fx_accu_xy (identical kernel and order). */
int fx_dot(fx_dtype dt, const void* X, const void* Y, int64_t n, void* d_out,
           void* ws, size_t ws_bytes, const fx_launch* cfg, void* stream);

/* Z = (X + Y) % exp(-abs(W)) / (1 + X % X), element-wise over `shape`.
 * FP dtypes. */
int fx_c2_z(fx_dtype dt, const void* X, const void* Y, const void* W, void* Z,
            fx_shape shape, const fx_launch* cfg, void* stream);

/* out[c] = sum_r E(r, c) for the C2 expression E: 1 x n_cols, written in the
 * accumulator dtype (float for F32/BF16/F16, double for F64).
 * ws: fx_workspace_bytes(FX_R_COLSUM). */
int fx_c2_colsum(fx_dtype dt, const void* X, const void* Y, const void* W, void* out,
                 fx_shape shape, void* ws, size_t ws_bytes, const fx_launch* cfg,
                 void* stream);

/* out[r] = sum_c E(r, c) for the C2 expression E: n_rows x 1, accumulator
 * dtype.  ws: fx_workspace_bytes(FX_R_ROWSUM). */
int fx_c2_rowsum(fx_dtype dt, const void* X, const void* Y, const void* W, void* out,
                 fx_shape shape, void* ws, size_t ws_bytes, const fx_launch* cfg,
                 void* stream);

/* *d_out = norm_fro(X - Y) = sqrt(sum (X - Y)^2) as FP64.
 * ws: fx_workspace_bytes(FX_R_NORM). */
int fx_norm_fro_diff(fx_dtype dt, const void* X, const void* Y, fx_shape shape,
                     double* d_out, void* ws, size_t ws_bytes, const fx_launch* cfg,
                     void* stream);

/* out[c] = sum_r X(r, c) * Y(r, c): sum(X % Y, 0), accumulator dtype. */
int fx_colsum_xy(fx_dtype dt, const void* X, const void* Y, void* out, fx_shape shape,
                 void* ws, size_t ws_bytes, const fx_launch* cfg, void* stream);

/* The paper's element-wise benchmark expressions (Sec. 4) that need no
 * transposed, submatrix or diagonal views.  Capital letters are matrices,
 * beta and alpha scalars; % is the Schur product. */
typedef enum {
  FX_PAPER_ADD2 = 1,    /* Z = X + Y                       inputs {X, Y}        */
  FX_PAPER_ADD4 = 2,    /* Z = A + B + C + D               inputs {A, B, C, D}  */
  FX_PAPER_RELU = 3,    /* Z = X % (X > 0)                 inputs {X}           */
  FX_PAPER_SIGMOID = 4, /* Z = 1 / (1 + exp(-X))           inputs {X}           */
  FX_PAPER_SWISH = 5,   /* Z = X / (1 + exp(-beta * X))    inputs {X}; s[0]=beta */
  FX_PAPER_GELU = 6,    /* Z = (X / 2) % (1 + tanh(sqrt(2/pi) * (X + alpha * pow(X, 3))))
                           inputs {X}; s[0]=alpha; sqrt(2/pi) rounded to the compute type */
  FX_PAPER_EXPR3 = 7    /* Z = 1 / (X % conv_to<fmat>::from(Y) + log(log(X + 2) % W))
                           inputs {X, Y, W}; Y is stored as FP64 and converted */
} fx_paper_expr_id;

/* One of the expressions above, fused into one kernel.  dt: FX_F32 or
 * FX_BF16 (Y of EXPR3 is always FP64).  scalars may be NULL when unused.
 * Scalars are rounded to the compute type. */
int fx_paper_expr(int which, fx_dtype dt, const void* const* inputs, const double* scalars,
                  void* Z, fx_shape shape, const fx_launch* cfg, void* stream);

/* Z = A1 + A2 + ... + An (1 <= n <= 16), added left to right: the add-N
 * family of the paper's bandwidth experiment (Sec. 4), one fused kernel
 * reading each input once.  dt: FX_F32 or FX_BF16. */
int fx_addn(fx_dtype dt, const void* const* inputs, int32_t n, void* Z, fx_shape shape,
            const fx_launch* cfg, void* stream);

/* The paper's expressions over strided views (Sec. 4; Sec. 3 gives the
 * transposed access, row and column swapped).  Inputs are m x n column-major
 * matrices (leading dimension m, the `shape` argument); the result Z is dense:
 *   FX_PAPER_ADDSUB2, _ADDSUB4: Z = sum of the centre submatrices (half the
 *     rows and columns, from row (m - m/2)/2 and column (n - n/2)/2) of
 *     2 or 4 inputs; Z is m/2 x n/2.
 *   FX_PAPER_EXPR1: Z = 2 * (X.t() + Y) + 2 * (X + Y.t()); m == n; Z m x m.
 *   FX_PAPER_EXPR2: Z = a * A + (B + C).t() + log(pow(D, 2)); m == n;
 *     s[0] = a; Z m x m.
 *   FX_PAPER_DIAGSUM: Z = (X.diag(-1) + X.diag(1)) % (Y.diag(-1) + Y.diag(1));
 *     Z is a column of the length the two diagonals share,
 *     min(min(m - 1, n), min(m, n - 1)) (m - 1 for a square matrix).
 * Transposed operands are staged through LDS tiles so that every HBM read
 * stays coalesced.  dt: FX_F32, FX_F64 or FX_BF16.  A non-square input for
 * EXPR1/EXPR2 gives FX_E_SHAPE.  Z may not overlap an input read through a
 * transposed, offset or diagonal view (FX_E_ARG, checked before anything is
 * enqueued); only EXPR2's A and D, read in place, may be Z itself. */
typedef enum {
  FX_PAPER_ADDSUB2 = 16,
  FX_PAPER_ADDSUB4 = 17,
  FX_PAPER_EXPR1 = 18,
  FX_PAPER_EXPR2 = 19,
  FX_PAPER_DIAGSUM = 20
} fx_paper_view_id;

/* Result shape of a view expression over m x n inputs (FX_E_SHAPE if the
 * inputs do not fit the expression). */
int fx_paper_view_shape(int which, fx_shape shape, fx_shape* out);
int fx_paper_view_expr(int which, fx_dtype dt, const void* const* inputs, const double* scalars,
                       void* Z, fx_shape shape, void* stream);

/* ---- unfused baseline: one kernel per operator ---------------------------
 * The same skeletons and launch configurations as the fused calls, but each
 * operator writes a full temporary, as toolkits without fusion do (Sec. 4). */

/* out = op(A), op in NEG/ABS/EXP/SQRT/LOG/TANH; floating-point dtypes only.
 * Each is the device function that the fused expressions inline. */
int fx_op_unary(int op, fx_dtype dt, const void* A, void* out, int64_t n,
                const fx_launch* cfg, void* stream);

/* out = A op B, op in ADD/SUB/SCHUR/DIV (FP) or ADD/SUB/SCHUR/XOR (U32). */
int fx_op_binary(int op, fx_dtype dt, const void* A, const void* B, void* out,
                 int64_t n, const fx_launch* cfg, void* stream);

/* out = scalar op with k (FX_OP_S*), k rounded to the compute type
 * (for U32 it must be an integer in [0, 2^32); SPOW is floating point only). */
int fx_op_scalar(int op, fx_dtype dt, const void* A, double k, void* out, int64_t n,
                 const fx_launch* cfg, void* stream);

/* A reduction of materialised arrays: ACCU/COLSUM/ROWSUM/NORM of A, or DOT
 * of A and B.  Output as for the fused calls (FP64 scalar, or accumulator
 * dtype vector). */
int fx_reduce(int kind, fx_dtype dt, const void* A, const void* B, fx_shape shape,
              void* out, void* ws, size_t ws_bytes, const fx_launch* cfg, void* stream);

/* Bytes of temporaries that fx_unfused(expr) needs. */
size_t fx_unfused_tmp_bytes(int expr, fx_dtype dt, fx_shape shape);

/* The workload expression `expr` (FX_EXPR_*) evaluated one operator at a
 * time with caller-provided temporaries `tmp` (fx_unfused_tmp_bytes bytes),
 * enqueuing one fx_op_* / fx_reduce kernel per AST node.  inputs = {X, Y, W}
 * as the expression needs; `a` is the scalar of FX_EXPR_AXY_EXPW. */
int fx_unfused(int expr, fx_dtype dt, const void* const* inputs, double a, void* out,
               fx_shape shape, void* tmp, size_t tmp_bytes, void* ws, size_t ws_bytes,
               const fx_launch* cfg, void* stream);

/* ---- run-time expression tapes ------------------------------------------
 * For trees only known at run time (they cannot be C++ types).  The tree is
 * compiled on the host into a short accumulator program that one kernel
 * interprets per element; the element loop and the reductions are the same
 * skeletons as the fused calls, so a tape is also read once and written
 * once.  Operators: FX_OP_ADD/SUB/SCHUR/DIV (binary), FX_OP_NEG/ABS/EXP/SQRT
 * (unary), FX_OP_LEAF and FX_OP_CONST (leaves).  Floating-point dtypes. */

/* One node.  Nodes are listed children first and the last node is the root;
 * a node may be the operand of several later nodes (a DAG is accepted). */
typedef struct {
  int32_t op;    /* FX_OP_* above */
  int32_t a, b;  /* operand node indices (< this node's index); -1 if unused */
  int32_t input; /* FX_OP_LEAF: which input array (0..3) */
  double value;  /* FX_OP_CONST: the constant, rounded to the compute type */
} fx_node;

/* Structural features of a compiled tape (also the cost model's inputs). */
typedef struct {
  int32_t n_nodes, n_inputs, depth, n_instructions, n_slots, n_consts;
  int32_t op_count[8]; /* add, sub, schur, div, neg, abs, exp, sqrt */
} fx_tape_info;

typedef struct fx_tape fx_tape;

/* Compile nodes[0..n_nodes) into *out (library-owned; fx_tape_destroy frees
 * it).  Limits: 4 inputs, 128 instructions, 16 slots counting the inputs
 * (FX_E_UNSUPPORTED beyond them); malformed trees give FX_E_ARG. */
int fx_tape_create(const fx_node* nodes, int32_t n_nodes, fx_tape** out);
void fx_tape_destroy(fx_tape* t);
int fx_tape_describe(const fx_tape* t, fx_tape_info* out);

/* The instructions of a compiled tape, for inspection and host-side
 * checking.  The machine has one accumulator `acc` and slots s[0..16);
 * input q is preloaded in s[q] and the result is acc after the last
 * instruction.  y is s[slot] for the _S forms and imm for the _I forms. */
typedef enum {
  FX_TI_LD = 0,  /* acc = s[slot] */
  FX_TI_LDI,     /* acc = imm */
  FX_TI_ST,      /* s[slot] = acc */
  FX_TI_ADD_S, FX_TI_ADD_I,   /* acc = acc + y */
  FX_TI_SUB_S, FX_TI_SUB_I,   /* acc = acc - y */
  FX_TI_RSUB_S, FX_TI_RSUB_I, /* acc = y - acc */
  FX_TI_MUL_S, FX_TI_MUL_I,   /* acc = acc * y (element-wise) */
  FX_TI_DIV_S, FX_TI_DIV_I,   /* acc = acc / y */
  FX_TI_RDIV_S, FX_TI_RDIV_I, /* acc = y / acc */
  FX_TI_NEG, FX_TI_ABS, FX_TI_EXP, FX_TI_SQRT, /* acc = f(acc) */
  FX_TI_STLD,   /* s[slot] = acc, then acc = s[slot2] */
  /* modifier bits or-ed into the opcode of an instruction that reads acc,
   * applied in this order before the operation: acc = s[slot2] (a load
   * folded into its consumer), acc = |acc|, acc = -acc (abs and neg nodes
   * are folded into their consumer this way) */
  FX_TI_ABS_IN = 0x100,
  FX_TI_NEG_IN = 0x200,
  FX_TI_LD_IN = 0x400
} fx_tape_opcode;

/* Copy up to `cap` instructions of t into op[] (opcode | modifier bits),
 * slot[], slot2[] and imm[] (any may be NULL when cap is 0); returns the
 * instruction count, or a negative fx_status for a NULL tape. */
int32_t fx_tape_program(const fx_tape* t, uint16_t* op, uint8_t* slot, uint8_t* slot2, double* imm,
                        int32_t cap);

/* Evaluate tape t over inputs[0..n_inputs) (n_inputs >= the tape's inputs,
 * all of storage dtype dt and shape `shape`).  kind 0: element-wise, `out`
 * has the storage dtype; FX_R_ACCU / FX_R_NORM: one double; FX_R_COLSUM /
 * FX_R_ROWSUM: accumulator dtype vector.  ws as for the fused reductions
 * (fx_workspace_bytes of the same kind, which covers both the library's and
 * the interpreter's defaults).  Fields of cfg left at 0 take the
 * interpreter's own defaults, chosen on the autotuner's training trees:
 * element-wise 64 threads, EPT 1, 16-byte vectors, one tile per block (256
 * threads, EPT 2 for 4- and 8-byte types from 2^20 elements on);
 * accu / norm 512 threads, EPT 2 (1 for half types), 2 blocks per CU;
 * column sums 256 threads, EPT 2 (1 for half types), one block per column
 * when there are at least as many columns as CUs; row sums 256 threads,
 * EPT 2, one row per thread, 64 column chunks.  The split default applies
 * only when all of cfg is 0 (or cfg is NULL); then a model attached with
 * fx_tape_set_model chooses instead.  Tapes are compiled for EPT 1, 2 and 4
 * and for vectors of one element, 8 or 16 bytes: other explicit values give
 * FX_E_UNSUPPORTED. */
int fx_tape_eval(const fx_tape* t, fx_dtype dt, const void* const* inputs, int32_t n_inputs,
                 fx_shape shape, int kind, void* out, void* ws, size_t ws_bytes,
                 const fx_launch* cfg, void* stream);

/* For callers that cannot allocate device memory (code under stream or graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as fx_tape_eval, same kernels and same bits for the same
 * launch, with the reductions' workspace taken from a static device array
 * of the library (16 MiB, one per GPU, held until the process ends) instead
 * of a caller's.  The caller still passes inputs and outputs.  The launch is
 * cfg, or the interpreter's defaults for fields left at 0; a model attached
 * with fx_tape_set_model is not consulted.  A reduction whose
 * fx_workspace_bytes exceeds 16 MiB gives FX_E_WORKSPACE before anything is
 * enqueued.  The first call on a device looks the array's address up and
 * clears it with a kernel on `stream`; every call leaves its finish counters
 * at zero.  No call allocates: no hipMalloc, hipFree or allocating library
 * routine.  All calls on one GPU share the array, so calls that may overlap
 * on one GPU (different streams, or other host threads) race and must be
 * serialised by the caller. */
int fx_tape_eval_static(const fx_tape* t, fx_dtype dt, const void* const* inputs, int32_t n_inputs,
                        fx_shape shape, int kind, void* out, const fx_launch* cfg, void* stream);

/* ---- run-time source mode -------------------------------------------------
 * The paper's own mechanism (Sec. 3): the kernel source of an expression is
 * generated, compiled through the driver at first use and reused.  Here a
 * tree (the fx_node list of the tapes) and a result kind become the HIP
 * source of one fused kernel, compiled with hipRTC for gfx950 with the
 * library's flags and cached per process by its text.  The compiled kernel
 * reads each input once (and writes once, element-wise), like a
 * compile-time expression, without the interpreter's per-instruction cost;
 * its reductions follow the fused ones (compensated per-thread sums, FP64
 * block and cross-block combine, single-pass finish).  FP32, FP64, BF16 and
 * FP16 storage; the launch configuration is the library default of the kind
 * and storage type. */
typedef struct fx_rtc fx_rtc;

/* Generate and compile (or find in the cache) the kernel of nodes[0..n_nodes)
 * for storage dtype dt and result kind (0: element-wise; FX_R_ACCU,
 * FX_R_NORM, FX_R_COLSUM, FX_R_ROWSUM).  Synchronous; needs no device.
 * Compilation errors give FX_E_HIP with the compiler log in fx_last_error;
 * another dtype gives FX_E_DTYPE, another kind FX_E_ARG. */
int fx_rtc_create(const fx_node* nodes, int32_t n_nodes, fx_dtype dt, int kind, fx_rtc** out);
void fx_rtc_destroy(fx_rtc* r);
/* The generated source (NUL-terminated, truncated to cap - 1); *len = its
 * full length. */
int fx_rtc_source(const fx_rtc* r, char* buf, size_t cap, size_t* len);
/* Milliseconds spent compiling at creation (0: found in the cache). */
double fx_rtc_compile_ms(const fx_rtc* r);
/* Evaluate r over inputs[0..n_inputs) (n_inputs >= the tree's inputs, all of
 * the storage dtype and column-major shape `shape`, 16-byte aligned).  Kind
 * 0: out has the storage dtype and shape's size (16-byte aligned; exact
 * aliasing with an input is allowed); FX_R_ACCU / FX_R_NORM: one double;
 * FX_R_COLSUM / FX_R_ROWSUM: n_cols / n_rows values of the accumulator dtype
 * (double for FP64 storage, float otherwise).  ws as for the fused
 * reductions: fx_workspace_bytes(kind, dt, shape, NULL) bytes, zeroed once.
 * Loads the module on the current device at its first use; enqueues one
 * kernel on `stream`.  An empty result is a no-op; accu and norm of an empty
 * shape write 0, dimension sums over an empty dimension write zeros. */
int fx_rtc_eval(fx_rtc* r, const void* const* inputs, int32_t n_inputs, fx_shape shape, void* out,
                void* ws, size_t ws_bytes, void* stream);

/* ---- kernels generated as source from expression types -------------------
 * The paper's mechanism itself (Sec. 3): the library's workload expressions
 * (FX_EXPR_*), the same C++ expression types that instantiate the fused
 * entry points above, are walked at compile time and each becomes the full
 * source text of one kernel, a string constant built during compilation and
 * embedded in libfx.so.  At first use the driver (hipRTC) compiles it for the
 * device; the code object is kept for the process (Sec. 4: that first
 * compilation is the only overhead).  Every leaf occurrence is a kernel
 * argument of its own and every scalar of the expression a run-time argument,
 * as in the paper's generated kernels; loops, loads and reductions are the
 * fused skeletons written as text (default launch configuration).
 *
 * fx_source_eval: evaluate expression `expr` over inputs {X, Y, W} (as the
 * expression needs; `a` is the scalar of FX_EXPR_AXY_EXPW) of storage dtype
 * dt and shape `shape`: Z (element-wise), one double (accu, norm_fro) or the
 * column / row sums in the accumulator dtype, as fx_unfused() defines them;
 * ws as for the fused calls.  Every array must be 16-byte aligned (FX_E_ARG
 * otherwise).  FP dtypes; FX_U32 for FX_EXPR_C1_Z only.  The first call for
 * an (expr, dt) compiles, which takes a while and needs hipRTC. */
int fx_source_eval(int expr, fx_dtype dt, const void* const* inputs, double a, void* out,
                   fx_shape shape, void* ws, size_t ws_bytes, void* stream);
/* The generated text of (expr, dt): *len = its length; up to cap - 1 bytes
 * and a terminating NUL are copied to buf (either may be NULL / 0). */
int fx_source_text(int expr, fx_dtype dt, char* buf, size_t cap, size_t* len);
/* Compile (expr, dt)'s text now if that has not happened (no GPU needed);
 * *compile_ms (may be NULL) = milliseconds the compilation took. */
int fx_source_prepare(int expr, fx_dtype dt, double* compile_ms);

/* ---- batches: thousands of uneven expressions in one launch -------------
 * Every expression of a batch is a compiled tape over vectors.  The batch is
 * cut into fixed-size tiles (the tiles of one expression are consecutive);
 * one persistent kernel walks the tile table and runs each tile's program,
 * and the last tile of a reducing expression to finish adds its tile
 * partials in tile order (FP64), so each result is independent of the other
 * expressions and of their order in the batch.  The launch can be captured
 * once in a HIP graph and replayed. */

typedef struct {
  const fx_tape* tape;      /* compiled tree (not retained after create) */
  const void* inputs[4];    /* device inputs, n elements each, as the tape reads */
  void* out;                /* kind 0: n elements of the storage dtype;
                               FX_R_ACCU: one double */
  int64_t n;                /* elements (a vector of length n) */
  int32_t kind;             /* 0 (element-wise) or FX_R_ACCU */
  int32_t reserved;
} fx_batch_item;

typedef struct {
  int32_t count, block, ept, vec_bytes, grid;
  int64_t n_tiles, tile_elems;
  int64_t bytes; /* algorithmic bytes: inputs read once + element-wise outputs */
} fx_batch_info;

typedef struct fx_batch fx_batch;

/* Build a batch (synchronous: allocates and uploads its device tables, owned
 * by the batch).  cfg: block / ept / vec_bytes as elsewhere (0 = 512 threads
 * for 4- and 8-byte storage, 256 for half storage; 16-byte vectors; and as
 * many vectors per thread as fill one interpreter pass: 2 for FP32 and FP64
 * storage, 1 for half storage), split = grid of the persistent kernel (0 =
 * as many blocks as the device holds at once); tile_elems: elements per tile
 * (0 = 16 block passes: 65536 for FP32, 32768 for FP64 and half storage with
 * the default block; rounded up to whole block passes).  Tiles are handed out from a work queue, costliest first.  Item
 * pointers must stay valid while the batch is used. */
int fx_batch_create(const fx_batch_item* items, int32_t count, fx_dtype dt,
                    const fx_launch* cfg, int64_t tile_elems, fx_batch** out);

/* Enqueue the whole batch as one kernel launch on `stream`. */
int fx_batch_launch(fx_batch* b, void* stream);

/* First call: capture the launch on `stream` into a HIP graph and launch it;
 * later calls: replay the graph on `stream` (one hipGraphLaunch). */
int fx_batch_graph(fx_batch* b, void* stream);

/* The same work as count separate launches, one fx_tape_eval per item with
 * the library's default configuration (the comparison point of the
 * persistent launch).  Reducing items use workspaces owned by the batch. */
int fx_batch_launch_each(fx_batch* b, void* stream);

int fx_batch_describe(const fx_batch* b, fx_batch_info* out);

/* Frees the batch's device tables and graph (synchronises its last stream). */
void fx_batch_destroy(fx_batch* b);

/* ---- autotuning -----------------------------------------------------------
 * The timing core of the exhaustive autotuner and the learned cost model
 * that replaces it.  Neither appears in the paper; they choose the launch
 * configuration (block, EPT, vector width, split) the kernels above take. */

/* Time tape t, run exactly as fx_tape_eval(t, dt, inputs, n_inputs, shape,
 * kind, out, ws, ...) would run it, under each of cfgs[0..n_cfgs): `warmup`
 * untimed launches, then `reps` launches each bracketed by HIP events on
 * `stream` (an all-zero configuration is the library defaults, even with a
 * model attached to t).  ms[c*reps + r] receives the times in milliseconds; a
 * configuration that is not compiled or does not fit (FX_E_UNSUPPORTED,
 * FX_E_CONFIG, FX_E_WORKSPACE) gets NaN and the sweep goes on.  ws must hold
 * the largest workspace among the configurations.  Synchronous. */
int fx_tune_time(const fx_tape* t, fx_dtype dt, const void* const* inputs, int32_t n_inputs,
                 fx_shape shape, int kind, void* out, void* ws, size_t ws_bytes,
                 const fx_launch* cfgs, int32_t n_cfgs, int32_t warmup, int32_t reps,
                 float* ms, void* stream);

/* The exhaustive autotuner's configuration grid for a tape of result kind
 * `kind` (0 or FX_R_*) and storage dtype dt: block {64, 128, 256, 512} x EPT
 * {1, 2, 4} x vector {one element, 8 bytes, 16 bytes} x four split values of
 * the kind (element-wise 0, 2, 8, 32 blocks per CU; accu / norm 1, 2, 4, 8
 * blocks per CU; column sums 0, 1, 4, 16 chunks per column; row sums 0, 16,
 * 64, 256 column chunks; 0 = the library's choice), then the default (all 0).
 * Writes the 145 configurations to out[0..cap) and returns their count; with
 * out NULL or cap too small, only the count.  Negative fx_status on a bad
 * kind or dtype. */
int32_t fx_tune_grid(int kind, fx_dtype dt, fx_launch* out, int32_t cap);

/* Exhaustive autotuning: time tape t (arguments as for fx_tape_eval) under
 * every configuration of fx_tune_grid, each `warmup` untimed launches and
 * then the median of `reps` timed ones, and return the fastest in *best
 * and its median time in *best_ms.  The default configuration is timed but
 * never chosen.  Configurations whose workspace exceeds ws_bytes, or that
 * are not compiled, are skipped; FX_E_UNSUPPORTED if none runs.
 *
 * db_path (may be NULL): a timing database, one JSON object per line, that
 * the search appends its item to: "key" (a hash of the program with shape,
 * dtype and kind), "dtype", "reduce" (null for element-wise), "shape",
 * "cus", "features" (the 25 of fx_tape_features), "ms" (every grid
 * configuration's median in grid order, null where it did not run),
 * "best" (grid index), "best_ms", "default_ms", "mode" ("native") and
 * "tune_seconds".  The learned model trains on such lines.  FX_E_ARG if
 * the file cannot be opened or written (the search's results are still
 * returned).  Synchronous. */
int fx_autotune(const fx_tape* t, fx_dtype dt, const void* const* inputs, int32_t n_inputs,
                fx_shape shape, int kind, void* out, void* ws, size_t ws_bytes, int32_t warmup,
                int32_t reps, fx_launch* best, float* best_ms, const char* db_path,
                void* stream);

/* The learned cost model: a two-layer perceptron (standardised features ->
 * hidden ReLU layer -> one softmax head per launch knob), trained on the
 * autotuner's best configurations with softmax cross-entropy and Adam, by
 * hand-written FP32 kernels (no matrix cores).  Parameters: one flat FP32
 * array W1 [hidden x F] row-major, b1 [hidden], W2 [C x hidden], b2 [C],
 * C = sum of head sizes. */
typedef struct fx_model fx_model;

/* F <= 64 features, hidden <= 256, up to 8 heads of >= 2 classes each
 * (C <= 64).  Parameters start at zero: set them with fx_model_set. */
int fx_model_create(int32_t n_features, int32_t hidden, const int32_t* head_sizes,
                    int32_t n_heads, fx_model** out);
int32_t fx_model_num_params(const fx_model* m);

/* Host arrays (any may be NULL to keep the current values, trained ones
 * included): parameters, feature means and standard deviations (> 0).  New
 * parameters wait for queued training steps, then replace them and reset
 * Adam.  Synchronous. */
int fx_model_set(fx_model* m, const float* params, const float* mean, const float* stdv);
/* Copy parameters / standardisation to host arrays (synchronous). */
int fx_model_get(fx_model* m, float* params, float* mean, float* stdv);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on a device batch: X [batch x F]
 * row-major FP32, labels [batch x n_heads] int32 class indices.  *d_loss
 * (device, may be NULL) gets the mean cross-entropy before the update.
 * Gradients are summed over the batch in row order (deterministic). */
int fx_model_train_step(fx_model* m, const float* d_X, const int32_t* d_labels, int32_t batch,
                        float lr, float* d_loss, void* stream);

/* Train for `epochs` passes over the n device rows d_X [n x F] / d_labels
 * [n x n_heads] in mini-batches of `batch` rows (the last of an epoch may be
 * shorter), one fx_model_train_step each.  Epoch e visits the rows in the
 * order perm[e*n .. e*n + n): a HOST int32 array, each epoch a permutation
 * of 0..n-1 (checked: FX_E_ARG otherwise); NULL visits them in order.
 * d_losses (device FP32 [epochs], may be NULL) gets each epoch's last
 * mini-batch loss.  Waits for the stream's earlier work and the copy of
 * perm, then enqueues the steps on `stream` and returns.  Calls on one
 * model must not overlap. */
int fx_model_train(fx_model* m, const float* d_X, const int32_t* d_labels, int32_t n,
                   int32_t epochs, int32_t batch, float lr, const int32_t* perm,
                   float* d_losses, void* stream);

/* The gradient of the mean cross-entropy (no update) into d_grad [params]. */
int fx_model_grad(fx_model* m, const float* d_X, const int32_t* d_labels, int32_t batch,
                  float* d_grad, float* d_loss, void* stream);

/* Inference on a device batch: logits [batch x C] and/or per-head argmax
 * [batch x n_heads] (either may be NULL, not both). */
int fx_model_forward(const fx_model* m, const float* d_X, int32_t batch, float* d_logits,
                     int32_t* d_choice, void* stream);

/* Host twin of the inference kernel for one feature row: the same FP32
 * fused multiply-add arithmetic in the same order, on the host.  Uses the
 * current parameters: after training steps it first waits for the device and
 * copies them back once (a synchronisation); otherwise no GPU is involved. */
int fx_model_choose(const fx_model* m, const float* features, int32_t* choice);

void fx_model_destroy(fx_model* m);

/* The model's 25 input features for tape t evaluated with storage dtype dt,
 * shape `shape` and result kind `kind` (0 or FX_R_ACCU / COLSUM / ROWSUM /
 * NORM), in training order: 8 operator counts (add, sub, schur, div, neg,
 * abs, exp, sqrt); constants, depth, instructions, slots, inputs; 1 for
 * 2-byte storage; log2 of size, rows and columns (those of an n x 1 shape
 * for element-wise results and full reductions, which see the data as one
 * flat vector); the kind one-hot
 * (element-wise, accu, column sums, row sums, norm); bytes per element
 * (inputs, plus the output if element-wise); div + exp + sqrt count; log2
 * of the bytes moved.  Writes them to out[0..cap) and returns 25 (only the
 * count with out NULL or cap < 25); negative fx_status on bad arguments.
 * Host only. */
int32_t fx_tape_features(const fx_tape* t, fx_dtype dt, fx_shape shape, int kind, float* out,
                         int32_t cap);

/* Load a model file written by the Python driver's save ("FXM1": int32
 * n_features, hidden, n_heads, head sizes; float means, standard
 * deviations; int32 parameter count; float parameters) into a new model
 * (device memory; fx_model_destroy frees it).  FX_E_ARG if the file is
 * missing or malformed. */
int fx_model_load(const char* path, fx_model** out);

/* The launch configuration the model picks for one feature row: its four
 * heads (block 4, EPT 3, vector 3, split 4 classes) mapped onto the
 * autotuner's grid for `kind` and dt (fx_tune_grid), on the host. */
int fx_model_predict(const fx_model* m, const float* features, int kind, fx_dtype dt,
                     fx_launch* out);

/* Attach model m to tape t (NULL detaches).  From then on, fx_tape_eval
 * calls on t that leave the launch configuration to the library (cfg NULL
 * or all zero) run the model's pick for their dtype, shape and kind
 * (fx_tape_features, then fx_model_predict, on the host; the last pick is
 * cached in the tape until the dtype, shape or kind changes or the model is
 * trained or set again).  A pick whose workspace exceeds the call's ws_bytes
 * falls back to the defaults.  Explicit configurations, fx_tune_time and
 * fx_autotune are unaffected.  m must stay alive while attached. */
int fx_tape_set_model(fx_tape* t, const fx_model* m);

/* ---- measurement kernels ------------------------------------------------- */

/* dst[i] = src[i] for `bytes` bytes (16-byte aligned, multiple of 16): the
 * achievable-bandwidth ceiling (Sec. 4 measures it with a copy benchmark). */
int fx_bw_copy(const void* src, void* dst, size_t bytes, const fx_launch* cfg,
               void* stream);

/* Streams `bytes` bytes of src into a per-block sum written to sink (one
 * double per block; sink holds at least `split` doubles): read ceiling. */
int fx_bw_read(const void* src, size_t bytes, double* sink, const fx_launch* cfg,
               void* stream);

/* dst[i] = value for `bytes` bytes: write ceiling and cache flushing. */
int fx_bw_write(void* dst, size_t bytes, uint32_t value, const fx_launch* cfg,
                void* stream);

/* dst = a + b + c over `bytes` bytes per array (u32 lanes, wrapping; every
 * pointer 16-byte aligned, bytes a multiple of 16): the ceiling of a kernel
 * that reads three streams for each one it writes.  flags: 1 = streaming
 * (nontemporal) stores.  cfg: block, EPT (vectors in flight per array and
 * thread) and grid as for element-wise calls. */
int fx_bw_triad(const void* a, const void* b, const void* c, void* dst, size_t bytes, int flags,
                const fx_launch* cfg, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FX_H */
