/*
 * saturator.h -- C ABI of the equality-saturation path of libstencil.so:
 * pointwise multi-statement kernels ("programs") over a 3-D grid, rewritten
 * by an e-graph and generated as HIP for gfx950.
 *
 * This is the paper's own method (arXiv 2306.13002) applied at kernel
 * generation time: the loop body is put into single-assignment form and
 * loaded into one e-graph (Sec. "E-Graph Creation"), saturated with the rule
 * set of Table tab:rule -- FMA1..FMA3, COMM-ADD, COMM-MUL, ASSOC-ADD1/2,
 * ASSOC-MUL1/2 -- plus constant folding (Sec. "Rewriting Rules"), under the
 * limits of Sec. Experimental Methodology (10 000 e-nodes, 10 iterations, 10 s); the
 * cheapest equal program is extracted under the cost model of Sec. "Cost
 * Model" (constant 0, input variable 1, arithmetic 10, memory access 100,
 * common e-classes counted once); temporaries are inserted and, in the bulk
 * forms, every load is moved ahead of the first statement in ascending
 * (array, offset) order (Sec. "Code Generation", "Bulk Load").
 *
 * A program is an ordered list of statements over one padded grid
 * geometry.  Statement s assigns either an output array at the current
 * point, out[o](i,j,k) = expr, or a local scalar that later statements
 * read.  Expressions are given in postfix form (sat_insn below) over
 *   - loads  in[a](i+dx, j+dy, k+dz)  of FP64 input arrays,
 *   - scalar FP64 parameters (values passed at run time),
 *   - FP64 constants,
 *   - +, -, *, unary - ; FMA(A, B, C) = A + B*C is produced by the rules only.
 * Every array (inputs and outputs) has the padded layout of stencil.h:
 * element (x,y,z) at base + z*pitch_z + y*pitch_y + x, interior point
 * (i,j,k) at (i+r, j+r, k+r), r = radius >= max |offset|.  Outputs are
 * written at interior points only; inputs are never written.  Outputs must
 * not overlap inputs or each other (checked on the host from the base
 * pointers and the padded span; a program that needs in-place updates is
 * outside this interface).
 *
 * Forms (sat_form) -- the paper's ablation versions (Sec. Evaluation):
 *   SAT_PLAIN     the statements as written: every operand loaded where it
 *                 appears, products and sums rounded in the written order;
 *   SAT_CSE       one e-graph without rewrite rules: each distinct load and
 *                 subexpression computed once, temporaries placed right
 *                 before their first use;
 *   SAT_CSE_SAT   CSE after equality saturation (rules + extraction);
 *   SAT_CSE_BULK  CSE with every load hoisted to the start (bulk load);
 *   SAT_ACCSAT    saturation and bulk load together (the paper's default);
 *   SAT_ACCSAT_Z  ACCSAT's arithmetic with the loads reused along z: a
 *                 thread walks `zblock` planes of its (i, j) column; each
 *                 load enters a register window of its (array, dx, dy)
 *                 column one plane ahead and is reused while its z offset
 *                 moves through the window (the MI355X counterpart of the
 *                 stencil kernels' register queues).  Bit-identical to
 *                 SAT_ACCSAT.
 * SAT_PLAIN and SAT_CSE evaluate exactly the written operations and are
 * bitwise reproducible against a plain FP64 evaluation; the saturated forms
 * reassociate and fuse (each fma rounds once).
 *
 * Errors, streams and ownership follow stencil.h: status codes with
 * stencil_last_error(); arrays are caller-owned DEVICE pointers; the plan
 * owns its compiled module only.
 */
#ifndef SATURATOR_H
#define SATURATOR_H

#include <stdint.h>

#include "stencil.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sat_plan_s *sat_plan_t;

typedef enum {
    SAT_OP_CONST = 1, /* push consts[a] */
    SAT_OP_PARAM = 2, /* push params[a] */
    SAT_OP_LOAD = 3,  /* push in[a](i+b, j+c, k+d) */
    SAT_OP_ADD = 4,   /* pop y, pop x, push x + y */
    SAT_OP_SUB = 5,   /* pop y, pop x, push x - y */
    SAT_OP_MUL = 6,   /* pop y, pop x, push x * y */
    SAT_OP_NEG = 7,   /* pop x, push -x */
    SAT_OP_STORE = 8, /* pop x: out[a](i,j,k) = x; ends a statement (stack must then be empty) */
    SAT_OP_SET = 9,   /* pop x: local scalar a = x; ends a statement */
    SAT_OP_GET = 10   /* push local scalar a (must have been SET before) */
} sat_op;

typedef struct {
    int32_t op;          /* sat_op */
    int32_t a, b, c, d;  /* operands, see sat_op; unused ones 0 */
} sat_insn;

typedef struct {
    uint32_t struct_size;  /* = sizeof(sat_program_desc) */
    int32_t n_inputs;      /* 1..128 input arrays */
    int32_t n_outputs;     /* 1..128 output arrays */
    int32_t n_params;      /* 0..64 scalar parameters */
    int32_t n_locals;      /* 0..256 local scalars */
    int32_t n_insns;       /* 1..65536 */
    const sat_insn *insns; /* HOST array, copied */
    int32_t n_consts;
    const double *consts;  /* HOST array, copied */
    int32_t radius;        /* halo width of every array, 0..8, >= every |offset| */
    int64_t n[3];          /* interior extents x, y, z, each >= 1 */
    int64_t pitch_y, pitch_z; /* elements; 0 = dense */
} sat_program_desc;

typedef enum { SAT_PLAIN = 0, SAT_CSE = 1, SAT_CSE_SAT = 2, SAT_CSE_BULK = 3, SAT_ACCSAT = 4, SAT_ACCSAT_Z = 5 } sat_form;

/* Extraction: SAT_EXTRACT_GREEDY = bottom-up tree cost, then a DAG-cost local
 * search (common e-classes counted once); SAT_EXTRACT_EXACT = exhaustive
 * minimum DAG cost, offered only for e-graphs with at most 2^22 selections
 * (E_UNSUPPORTED otherwise; meant for checking the greedy extraction). */
typedef enum { SAT_EXTRACT_GREEDY = 0, SAT_EXTRACT_EXACT = 1 } sat_extract;

typedef struct {
    int32_t enodes, eclasses;  /* e-graph size after saturation */
    int32_t iterations;        /* rewrite iterations run */
    int32_t saturated;         /* 1 if the last iteration added nothing */
    double cost_input;         /* cost-model cost of the program as written (DAG, CSE applied) */
    double cost_extracted;     /* cost of the extracted program */
    int32_t loads, ops, fmas;  /* extracted program: distinct loads, arithmetic ops, of which FMA */
    double saturate_ms, extract_ms;
} sat_stats;

/* Rewrite and generate (host only, no GPU needed).  Writes the generated HIP
 * source (kernel "sat_kernel_<form>", e.g. sat_kernel_accsat) to src[0..src_len) and the extracted program
 * as single-assignment text to ssa[0..ssa_len), both NUL-terminated; either
 * buffer may be NULL.  SSA lines:  "v<N> = <op> <args>"  with op one of
 * const <hexfloat> | param <p> | load <a> <dx> <dy> <dz> | add | sub | mul |
 * neg | fma (fma A B C = A + B*C), args "v<M>"; then "store <o> v<N>" or
 * "set <l> v<N>" per statement in order.  E_INVAL if a buffer is too small
 * (the message gives the size needed). */
stencil_status sat_generate(const sat_program_desc *d, int32_t form, int32_t extract, int32_t tile_x, int32_t tile_y,
                            int32_t zblock, char *src, int64_t src_len, char *ssa, int64_t ssa_len, sat_stats *stats);

/* Rewrite, generate and compile (hipRTC) the program for one form; one
 * thread per interior (i, j) column, blocks of tile_x * tile_y threads (0 =
 * 64 x 4) over x and y, each thread evaluating `zblock` consecutive planes
 * of its column (0 = 1 plane; 32 for SAT_ACCSAT_Z).  With zblock > 1 the
 * non-streaming forms issue every load again at each plane, and the planes
 * shared with the previous one come from the caches; results do not depend
 * on zblock. */
stencil_status sat_plan(const sat_program_desc *d, int32_t form, int32_t tile_x, int32_t tile_y, int32_t zblock,
                        sat_plan_t *out);

/* Run the program once over the interior.  inputs: n_inputs device
 * pointers; outputs: n_outputs device pointers; params: n_params HOST
 * doubles (may be NULL if n_params == 0); stream: hipStream_t or NULL.
 * Asynchronous. */
stencil_status sat_run(sat_plan_t p, const void *const *inputs, void *const *outputs, const double *params,
                       void *stream);

/* Compiled-kernel resources of the plan, as the HIP runtime reports them:
 * registers per lane, private (spill) bytes per lane, static LDS bytes. */
stencil_status sat_plan_info(sat_plan_t p, int32_t *regs, int32_t *private_bytes, int32_t *lds_bytes);

/* Event timing of sat_run (HIP events on the run's stream): while enabled,
 * every sat_run is bracketed by events; read returns the milliseconds of the
 * last profiled run (synchronizing with it) and runs = 1.  E_STATE if no
 * run was profiled. */
stencil_status sat_profile_enable(sat_plan_t p, int32_t enable);
stencil_status sat_profile_read(sat_plan_t p, double *run_ms, int32_t *runs);

stencil_status sat_destroy(sat_plan_t p); /* NULL ok */

#ifdef __cplusplus
}
#endif

#endif /* SATURATOR_H */
