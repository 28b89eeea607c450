/*
 * qlg.h -- C ABI of libqlg, the MI355X (gfx950) spin-2 quantum-lattice-gas step.
 *
 * The method is the unitary QLG algorithm for the spin-2 Gross-Pitaevskii
 * equation of Taylor, Smith and Yepez (arXiv:1907.12834):
 *   - equation of motion: Sec. II, eq. (eomspin2) with the spin-2 matrices
 *     f_x, f_y, f_z printed there, couplings g0 (density), g1 (spin F.f),
 *     g2 (singlet pair);
 *   - encoding: two qubit amplitudes (a_m, b_m) per m_f level, psi = a + b
 *     (Sec. III "Local quantum entanglement": 10 qubits per site);
 *   - step: I'_q = S_q C S_q^T C, plain split psi(t+tau) = I'_1 I'_1 I'_2 I'_2 U psi(t)
 *     and the interleaved split I'_1 U^{1/4} I'_1 U^{1/4} I'_2 U^{1/4} I'_2 U^{1/4}
 *     (Lie product n = 4 in 1D, n = 8 in 2D, n = 12 in 3D, the axes in the order
 *     z, y, x) of Sec. VII "Operator interleaving";
 *   - lattice scaling x -> a x, t -> a^2 t (Sec. VII "Scaling"): one step
 *     advances physical time eps^2 on a lattice of spacing eps.
 * The definitions of C, S and U that the paper defers to its references are
 * fixed by the readings documented with the repository: C = sqrt(SWAP) with
 * entries (1 -+ i)/2, S_q shifts qubit q by one site along +axis, and U is the
 * per-site frozen-field unitary exp(-i th g0 n) exp(-i th g1 F.f)
 * (I + (exp(-i th g2 n/5) - 1) v v^H / n), v_m = (-1)^m conj(psi_{-m}).
 *
 * Conventions for every call:
 *   - Pointers named *_dev are device pointers on the current HIP device;
 *     *_host are host pointers.  The library never frees caller memory.
 *   - Calls return a qlg_status.  Argument, shape and dtype errors are detected
 *     on the host before any launch and leave the context unchanged.  A failed
 *     HIP launch or copy returns QLG_ERR_DEVICE and puts the context into an
 *     error state in which every later call except qlg_destroy and
 *     qlg_last_error returns QLG_ERR_STATE.
 *   - Work is enqueued on the caller's stream given at qlg_init (hipStream_t,
 *     passed as void*; NULL is the default stream).  Calls that return host
 *     data (qlg_observables, qlg_objective_grad, qlg_adjoint_step) synchronise
 *     that stream; the others are asynchronous.
 *   - No C++ exception crosses this interface.
 *
 * Field layout (the canonical layout for psi_dev / qubits_dev arguments):
 *   complex numbers are interleaved (re, im), float for QLG_C64 and double for
 *   QLG_C128.  Instances follow one another; within instance i,
 *     psi[m][z][y][x]        m index 0..4 <-> m_f = 2, 1, 0, -1, -2, x fastest;
 *     qubits[q][m][z][y][x]  q = 0 for a (the paper's qubit 1), 1 for b (qubit 2).
 *   nz == 1 for 1D and 2D instances, ny == 1 for 1D instances.
 */
#ifndef QLG_H
#define QLG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QLG_OK = 0,
  QLG_ERR_ARG = 1,      /* NULL pointer, bad enum, non-finite coupling, buffer too small */
  QLG_ERR_SHAPE = 2,    /* ndim not 1..3, extent < 1, lattice too large, call not for this ndim */
  QLG_ERR_DTYPE = 3,    /* dtype not QLG_C64 / QLG_C128 */
  QLG_ERR_DEVICE = 4,   /* a HIP call failed; message in qlg_last_error */
  QLG_ERR_OOM = 5,      /* the library's host-side context allocation failed */
  QLG_ERR_STATE = 6,    /* context is in an error state, or call out of order */
  QLG_ERR_NUMERIC = 7   /* non-finite values, or qubit norm drift above threshold */
} qlg_status;

typedef enum { QLG_C64 = 0, QLG_C128 = 1 } qlg_dtype;

typedef enum {
  QLG_SPLIT_INTERLEAVED = 0, /* U^{1/(4d)} before every I' (Sec. VII, Lie product n = 4d) */
  QLG_SPLIT_PLAIN = 1        /* one U, then all I' (Sec. VII, the non-interleaved step) */
} qlg_split;

typedef struct qlg_params {
  int32_t ndim;          /* 1, 2 or 3 */
  int32_t dtype;         /* qlg_dtype */
  int32_t split;         /* qlg_split */
  int32_t nbatch;        /* >= 1 independent lattices; they may differ in size */
  const int64_t* nx;     /* [nbatch] x extents (host memory, copied at qlg_init) */
  const int64_t* ny;     /* [nbatch] y extents, or NULL for ndim == 1 */
  const int64_t* nz;     /* [nbatch] z extents, or NULL for ndim < 3 */
  double g0, g1, g2;     /* couplings of eq. (eomspin2), shared by all instances */
  double eps;            /* lattice spacing: one step = physical time eps^2; norms use eps^ndim */
} qlg_params;

typedef struct qlg_obs {
  double norm_q;         /* eps^d sum (|a|^2 + |b|^2): conserved exactly by the method */
  double norm_psi;       /* eps^d sum |a + b|^2 */
  double pop[5];         /* eps^d sum |psi_m|^2, m = 2..-2 */
  double energy;         /* eps^d sum [ sum_axis |psi(x+e)-psi(x)|^2/eps^2
                                        + (g0 n^2 + g1 |F|^2 + g2 |sigma|^2/5)/2 ] */
  double overlap_re;     /* eps^d <psi_t | psi_{t-1}> over the last step of the last qlg_step */
  double overlap_im;
  double e_overlap_re;   /* i (<psi_t|psi_t> - <psi_t|psi_{t-1}>) / <psi_t|psi_t>, Sec. IV
                            eq. (disecrete_energy); ~ E eps^2 for an eigenstate */
  double e_overlap_im;
  int64_t step;          /* steps taken since the last qlg_set_psi / qlg_set_qubits */
  int32_t has_overlap;   /* 1 if overlap_* refer to the last step, else 0 */
  int32_t reserved;
} qlg_obs;

/* Launch plan of the fused step; chosen by qlg_autotune or set by the caller. */
typedef struct qlg_tuning {
  int32_t steps_per_pass; /* 1D: steps fused per HBM pass, 4 S halo sites per side of each
                             tile (1..7 with 64-site tiles, 1..3 with the 32-site tiles of
                             qubit_split 2); 2D and 3D: must be 1 */
  int32_t tile_rows;      /* 2D and 3D: rows per streaming tile (8..256); 1D: ignored.
                             A 3D step is two HBM passes: the four z substeps streaming
                             along z, then the y and x substeps streaming along y, both
                             in bands of tile_rows */
  int32_t use_graph;      /* 1: replay qlg_step's launches from a captured hipGraph */
  int32_t qubit_split;    /* 1D: where the two qubit amplitudes (a_m, b_m) of a site live:
                             0 = one lane holds both (64-site tiles, steps_per_pass 1..7);
                             1 = two wavefronts, a on one and b on the other (64-site
                             tiles, steps_per_pass 1..7); 2 = two neighbouring lanes of
                             one wavefront (32-site tiles, steps_per_pass 1..3).  1 and 2
                             spread a lattice too small to fill the chip over twice the
                             lanes.  2D and 3D: 0 = the four y (3D: also z) substeps of a
                             pass in one launch; 1 = in two launches, qubit b's two then qubit
                             a's two (with the x substeps): half the LDS per wavefront, twice
                             the HBM round trips (the state between the launches is the true
                             state; both forms give the same numbers) */
} qlg_tuning;

typedef struct qlg_ctx qlg_ctx;

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t qlg_version(void);

/* Bytes the caller must provide for a lattice described by *params:
 *   state_bytes:   two copies (ping-pong) of all qubit planes, padded;
 *   scratch_bytes: reduction partials for observables and overlaps, and the
 *                  device tables of the launch geometry (instance descriptors,
 *                  tile and chunk maps).
 * Errors: QLG_ERR_ARG / SHAPE / DTYPE as for qlg_init. */
qlg_status qlg_query_sizes(const qlg_params* params, size_t* state_bytes, size_t* scratch_bytes);

/* Create a context over caller-owned device buffers.  state_dev and
 * scratch_dev must be 256-byte aligned and at least the sizes reported by
 * qlg_query_sizes.  hip_stream is a hipStream_t (or NULL).  The state is
 * undefined until qlg_set_psi or qlg_set_qubits.  The library allocates no
 * device memory: its tables live in scratch_dev.  It owns only the host
 * context and, once used, its captured graphs and timing events. */
qlg_status qlg_init(const qlg_params* params, void* state_dev, size_t state_bytes,
                    void* scratch_dev, size_t scratch_bytes, void* hip_stream, qlg_ctx** out);

/* qlg_init for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the caller
 * passes no scratch buffer.  The context's scratch (the scratch_bytes of
 * qlg_query_sizes: reduction partials and device tables) is a fixed array of
 * QLG_STATIC_SCRATCH_BYTES in the library's own device memory, one per GPU,
 * held until the process ends; this call allocates no device memory.  The
 * caller still provides state_dev (as for qlg_init).  One such context per GPU
 * at a time: QLG_ERR_STATE while another context made by this call lives on
 * the current device (qlg_destroy releases the array after synchronising the
 * context's stream); QLG_ERR_ARG when the lattice's scratch_bytes exceed
 * QLG_STATIC_SCRATCH_BYTES, or as for qlg_init.  The array keeps what the
 * previous context left in it; no kernel reads a value of it that the same
 * context has not written first.  Every other call behaves as on a context
 * made by qlg_init. */
#define QLG_STATIC_SCRATCH_BYTES (16u << 20)
qlg_status qlg_init_static(const qlg_params* params, void* state_dev, size_t state_bytes,
                           void* hip_stream, qlg_ctx** out);

/* Load psi (canonical layout) and encode a = b = psi / 2.  Resets the step counter. */
qlg_status qlg_set_psi(qlg_ctx* ctx, const void* psi_dev);
/* Decode psi = a + b into psi_dev (canonical layout). */
qlg_status qlg_get_psi(qlg_ctx* ctx, void* psi_dev);
/* Load / store both qubit amplitudes (canonical qubits layout). */
qlg_status qlg_set_qubits(qlg_ctx* ctx, const void* qubits_dev);
qlg_status qlg_get_qubits(qlg_ctx* ctx, void* qubits_dev);

/* External and chemical potential (Sec. II, "Additional terms"): the equation of
 * motion of every component gains (V(x) + mu) psi_m, so each self-interaction U
 * gains the per-site phase exp(-i theta (V(x) + mu)) and the energy of qlg_obs
 * gains eps^d sum (V + mu) n.  V_dev: device memory owned by the caller, FP64,
 * 8-byte aligned, in the canonical scalar layout of qlg_fields (nbatch * sites
 * doubles), or NULL for no potential; the library keeps the pointer, and every
 * later qlg_step and observables call reads it, so it must stay allocated until
 * the potential is replaced or the context destroyed (its values may change
 * between calls).  mu: finite, else QLG_ERR_ARG.  qlg_set_potential(ctx, NULL, 0)
 * returns to the plain equation.  The adjoint entry points differentiate the
 * run with the potential in place, V and mu being constants (no derivative with
 * respect to them); the energy objective includes its (V + mu) n term.
 * Host-side only; drops the captured step graphs. */
qlg_status qlg_set_potential(qlg_ctx* ctx, const double* V_dev, double mu);

/* Per-site diagnostic fields of the current state (Sec. III, eq. (cmap)), in
 * FP64, each in the canonical scalar layout: the instances back to back, each
 * [ny][nx] row-major (x fastest), nbatch * sites doubles in all:
 *   n_dev:      density n = sum_m |psi_m|^2;
 *   f_par_dev:  F_par = F_z = sum_m m |psi_m|^2;
 *   f_perp_dev: F_perp = sqrt(F_x^2 + F_y^2);
 *   a00_dev:    |A00| = |2 psi_2 psi_-2 - 2 psi_1 psi_-1 + psi_0^2| / sqrt(5),
 *               the singlet-pair amplitude.
 * psi = a + b is formed in the context's dtype (the value qlg_get_psi returns)
 * and then promoted to FP64.  Device buffers owned by the caller, 8-byte
 * aligned; a NULL output is not written, but not all four may be NULL
 * (QLG_ERR_ARG).  Asynchronous on the context's stream. */
qlg_status qlg_fields(qlg_ctx* ctx, double* n_dev, double* f_par_dev, double* f_perp_dev, double* a00_dev);

/* Lattice vorticity of hyperfine component m_index (0..4 for m = 2..-2) of a
 * 2D or 3D state (Sec. VI, "Calculating quantum vorticity on a lattice"), periodic:
 * the phase S = arg psi_m (0 where psi_m is exactly zero) gives velocities by
 * central differences, v_x(x, y) = w(S(x+1, y) - S(x-1, y)) / 2 and v_y
 * likewise, each difference w(.) reduced to (-pi, pi]; then
 *   omega_dev[x, y] = (v_y(x+1, y) - v_y(x-1, y) - v_x(x, y+1) + v_x(x, y-1)) / 2
 * (FP64), and winding_dev[x, y] (int32) is the winding number of the plaquette
 * (x, y) -> (x+1, y) -> (x+1, y+1) -> (x, y+1): the sum of its four wrapped
 * phase differences over 2 pi: +1 where the phase of psi_m rises by 2 pi
 * counter-clockwise (x right, y up) around the plaquette.
 * Both use the canonical scalar layout of qlg_fields; either may be NULL, not
 * both (QLG_ERR_ARG).  On a 3D lattice (which the paper names as future work)
 * the same is done in every family of lattice planes: omega_dev and winding_dev
 * then hold three such arrays one after the other (3 x the total site count),
 * for the plaquettes normal to x, y and z, circulated y -> z, z -> x and x -> y
 * (right-handed about the normal), omega being the curl component along that
 * normal.  QLG_ERR_SHAPE for a 1D context, QLG_ERR_ARG for m_index outside
 * 0..4.  Asynchronous on the context's stream. */
qlg_status qlg_vorticity(qlg_ctx* ctx, int32_t m_index, double* omega_dev, int32_t* winding_dev);

/* Vortex cores of component m_index of a 2D state, for tracking them through a
 * run (Sec. VI follows every core of every channel over time): the plaquettes
 * whose winding number, as qlg_vorticity defines it, is non-zero, listed in
 * the order (instance, y, x) as cores_dev[k] = {instance, y, x, winding}
 * (int32 x 4; (y, x) is the plaquette's lower-left corner).  On a 3D lattice
 * the plaquettes of the three plane families are listed, in the order (family,
 * instance, z, y, x), as cores_dev[k] = {instance, family, z, y, x, winding}
 * (int32 x 6; family 0, 1, 2 = normal to x, y, z as in qlg_vorticity; (z, y, x)
 * is the plaquette's first corner).  At most capacity entries are written;
 * count_dev[0] (device int64) receives the number of cores, which may exceed
 * capacity (call again with a larger buffer).  winding_dev (device, int32 in
 * the canonical scalar layout: nbatch * sites in 2D, 3 x that in 3D) is filled
 * with the winding field on the way.  The order is deterministic (no
 * atomics).  QLG_ERR_SHAPE for a 1D lattice; QLG_ERR_ARG for m_index outside
 * 0..4, NULL winding_dev or count_dev, capacity < 0, or capacity > 0 with NULL
 * cores_dev.  Asynchronous on the context's stream. */
qlg_status qlg_find_vortices(qlg_ctx* ctx, int32_t m_index, int32_t* winding_dev, int32_t* cores_dev,
                             int64_t capacity, int64_t* count_dev);

/* Advance every instance by nsteps >= 0 QLG steps (Sec. VII), asynchronously. */
qlg_status qlg_step(qlg_ctx* ctx, int64_t nsteps);

/* Norms, populations, energy (Sec. II energy functional on the lattice) and,
 * once a qlg_step call has run since the last set, the overlap energy of the
 * last step (Sec. IV), per instance, into out_host[nbatch].  Synchronises the
 * stream.  Returns QLG_ERR_NUMERIC (after filling out_host) if any value is
 * non-finite or |norm_q / norm_q(at set) - 1| exceeds 1e-4 (C64) or 1e-10 (C128). */
qlg_status qlg_observables(qlg_ctx* ctx, qlg_obs* out_host);

/* Observables without a host round trip, for diagnostics every k steps of a
 * long run.  qlg_record_observables enqueues the reductions of the current
 * state into rec_dev (device memory owned by the caller, at least
 * QLG_RECORD_DOUBLES * nbatch doubles, 8-byte aligned) and returns at once;
 * the record holds the FP64 sums, the step count and the reference norm, so it
 * can be decoded at any later time.  qlg_decode_records turns nrec consecutive
 * records (rec_host[nrec][nbatch][QLG_RECORD_DOUBLES], host memory) into
 * out_host[nrec][nbatch] with exactly the values and checks of qlg_observables
 * (QLG_ERR_NUMERIC if any record fails them).  Both are host-side only apart
 * from the kernels the first enqueues. */
#define QLG_RECORD_DOUBLES 16
qlg_status qlg_record_observables(qlg_ctx* ctx, double* rec_dev);
qlg_status qlg_decode_records(qlg_ctx* ctx, const double* rec_host, int64_t nrec, qlg_obs* out_host);

/* Plan control.  qlg_set_tuning returns QLG_ERR_ARG for a field out of the ranges
 * above (the context keeps its plan).  qlg_autotune times the candidate plans on the
 * context's own lattice without changing its state and keeps the fastest; among plans
 * within 2 % of the fastest it prefers fewer launches, then qubit_split 0, 1, 2, then
 * taller bands.  Chosen plans are kept for the process, keyed by device, dtype, ndim,
 * split, batched or not and the total site count rounded up to a power of two; a new
 * context with the same key starts from that plan.  When the environment variable
 * QLG_TUNE_CACHE names a file, qlg_autotune also appends the plan to it as a text line
 * "key steps_per_pass tile_rows use_graph qubit_split", and qlg_init takes the last
 * in-range line with its key from the file before the process's own record. */
qlg_status qlg_set_tuning(qlg_ctx* ctx, const qlg_tuning* tuning);
qlg_status qlg_get_tuning(const qlg_ctx* ctx, qlg_tuning* tuning);
qlg_status qlg_autotune(qlg_ctx* ctx);

/* Kernel timing.  qlg_set_timing(ctx, 1) starts (and resets) it: every
 * fused-step launch of later qlg_step calls is then dispatched with a pair of
 * HIP events that the dispatch packet itself stamps at kernel start and end
 * (no graph replay while timing; each qlg_step call synchronises the stream).
 * qlg_last_kernel_ms returns the average kernel time in milliseconds over all
 * launches timed since then, and their number (0 if none). */
qlg_status qlg_set_timing(qlg_ctx* ctx, int32_t enable);
qlg_status qlg_last_kernel_ms(qlg_ctx* ctx, double* ms_host, int64_t* launches_host);

/* ---------------------------------------------------------------------------
 * Adjoint (reverse-mode derivative of a final-state objective).
 *
 * Cotangents use the convention lambda = dL/dRe z + i dL/dIm z for every
 * complex amplitude z (so d|z|^2 has cotangent 2 z).  Adjoint vectors are
 * complex128 in the qubits layout, whatever the forward dtype; the
 * self-interaction Jacobian is evaluated in FP64.
 * ------------------------------------------------------------------------- */

/* Sizes for recording a forward run of nsteps with a checkpoint every
 * checkpoint_every steps (>= 1), and for the adjoint workspace.  The workspace
 * holds the input of every self-interaction of one checkpoint segment
 * (checkpoint_every x 4 ndim state copies for the interleaved split,
 * checkpoint_every copies for the plain split) twice, plus two state copies, two
 * complex128 cotangents and small reduction buffers: memory traded for
 * recomputation, so checkpoint_every bounds it.  The second set of segment inputs
 * comes last; it lets the reverse sweep recompute the next segment's inputs on a
 * second stream while it pulls the cotangent back through the current segment. */
qlg_status qlg_adjoint_query(const qlg_params* params, int64_t nsteps, int32_t checkpoint_every,
                             size_t* ckpt_bytes, size_t* work_bytes);

/* Run nsteps forward from the current state, storing the state at steps
 * 0, K, 2K, ... (K = checkpoint_every) into ckpt_dev. */
qlg_status qlg_forward_record(qlg_ctx* ctx, int64_t nsteps, int32_t checkpoint_every,
                              void* ckpt_dev, size_t ckpt_bytes);

/* Objective of the current state and its cotangent lambda (complex128 qubits layout):
 *   kind 0: energy E of qlg_obs (per instance, summed over instances);
 *   kind 1: fidelity |<target|psi>|^2 with target_dev in the canonical psi layout
 *           (forward dtype), summed over instances.
 * value_host[0] receives L; dg_host[3] (may be NULL) receives the explicit
 * dL/d(g0, g1, g2).  Synchronises the stream. */
qlg_status qlg_objective_grad(qlg_ctx* ctx, int32_t kind, const void* target_dev,
                              void* lambda_dev, double* value_host, double* dg_host);

/* Pull lambda back through the nsteps recorded by qlg_forward_record
 * (same nsteps and checkpoint_every): on entry lambda_dev holds dL/d(state at
 * the end), on exit dL/d(state at the start).  dg_host[3] is incremented by
 * dL/d(g0, g1, g2) accumulated over the steps.  work_dev holds work_bytes from
 * qlg_adjoint_query, or at least that less the second set of segment inputs
 * (checkpoint_every x 4 ndim state copies, checkpoint_every for the plain split;
 * QLG_ERR_ARG below it), in which case the segments are recomputed and pulled back
 * one after the other on the context's stream.  With the whole workspace the
 * context makes, on first use, a second stream of default priority (released by
 * qlg_destroy) for the recompute, ordered against its stream by events; the
 * results are the same bit for bit.  The context's current state is left at the
 * end state of the recorded run.  Synchronises the stream. */
qlg_status qlg_adjoint_step(qlg_ctx* ctx, int64_t nsteps, int32_t checkpoint_every,
                            const void* ckpt_dev, void* lambda_dev, void* work_dev,
                            size_t work_bytes, double* dg_host);

/* Adjoint of qlg_set_psi, the encoding a = b = psi / 2 (Sec. III, two qubits
 * per m_f level): from the cotangent of both qubits lambda_dev (complex128,
 * canonical qubits layout, as qlg_adjoint_step leaves it) writes the cotangent
 * of psi, dpsi_dev = (lambda_a + lambda_b) / 2 (complex128, canonical psi
 * layout, the same convention).  Device buffers owned by the caller, 16-byte
 * aligned, not overlapping; QLG_ERR_ARG for NULL or misaligned pointers.
 * Asynchronous on the context's stream. */
qlg_status qlg_set_psi_adjoint(qlg_ctx* ctx, const void* lambda_dev, void* dpsi_dev);

/* Fault injection, for tests of the error-state contract above: puts the context into the
 * state that a failed HIP launch or copy leaves, without touching the device — returns
 * QLG_ERR_DEVICE, after which every call on the context except qlg_destroy and
 * qlg_last_error returns QLG_ERR_STATE, and qlg_last_error names `reason` (may be NULL).
 * Enqueues nothing; other contexts are not affected.  QLG_ERR_ARG for a NULL context,
 * QLG_ERR_STATE if the context is already in the error state. */
qlg_status qlg_inject_device_error(qlg_ctx* ctx, const char* reason);

/* Human-readable status name, and the last error message of a context. */
const char* qlg_status_string(qlg_status status);
const char* qlg_last_error(const qlg_ctx* ctx);

/* Release the context (never the caller's buffers).  NULL is allowed. */
void qlg_destroy(qlg_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* QLG_H */
