/*
 * mpole -- multipole Poisson solve for Newtonian self-gravity on a
 * spherical-coordinate mesh, for one AMD Instinct MI355X (gfx950).
 *
 * The method is the one of GenASiS II, Sec. 2.2 ("Poisson Solver"): the
 * Green-function solution of the Poisson equation (Eq. IntPoisson) expanded
 * in multipoles (Eq. Multipole) with real angular kernels
 * A^c_lm = P~_l^m(cos th) cos m ph, A^s_lm = P~_l^m(cos th) sin m ph
 * (Eqs. AngularKernel_c/_s), discrete angular moments per radial shell
 * (Eq. AngularMomentsDiscrete), outward/inward radial integration of the
 * regular (r^l) and irregular (r^-(l+1)) radial moments at shell edges, and
 * the potential of Eq. Solution at cell centres.  Angular cells may be
 * merged into coarsening blocks (Sec. 2.1), per radial shell.
 *
 * Conventions fixed by this library where the paper leaves a choice:
 *   - modes: 0 <= m <= l <= lmax, a in {cos, sin}, without the identically
 *     zero A^s_l0, so nAM = (lmax+1)^2; mode index iAM = l*l for m = 0,
 *     l*l + 2m - 1 for (m, cos), l*l + 2m for (m, sin);
 *   - the source is S = 4 pi G rho (Sec. 3);
 *   - angular cell averages are solid-angle weighted, radial cell averages
 *     of r^l and r^-(l+1) are r^2 dr (volume) weighted;
 *   - edge moments are averaged to the shell centre (arithmetic mean of the
 *     two edges) before Eq. Solution is evaluated with cell-averaged kernels;
 *   - a shell whose inner edge is r = 0 has no irregular increment and no
 *     <r^-(l+1)> term for l >= 2 (the average diverges there);
 *   - a coarsening block is one cell of the solve: its density is the
 *     solid-angle weighted mean of its member cells, its kernels are the
 *     solid-angle weighted means of theirs, and its potential is written to
 *     every member cell.
 *
 * Layouts.  rho and phi are C-order [nr][ntheta][nphi] (phi fastest), FP64,
 * in device memory.  Moments are [shell or edge][iAM], FP64, device memory.
 * Everything crossing this interface is FP64; the precision mode only
 * changes how the two angular contractions are evaluated internally.
 *
 * Ownership.  The caller owns every device buffer, including the workspace
 * whose size mpole_plan_workspace_bytes() reports.  The library never
 * allocates or frees device memory.  A plan holds host metadata and
 * pointers into the bound workspace; one plan serves one stream at a time
 * (solves that overlap on one workspace race).
 *
 * Errors.  Every call returns an mpole_status, and mpole_last_error() (per
 * thread) describes a failure.  Every argument, size and state check of a
 * call runs before its first enqueue, so MPOLE_ERR_INVALID, _RANGE,
 * _WORKSPACE and _UNSUPPORTED mean that nothing was enqueued.
 * MPOLE_ERR_DEVICE means that a HIP call or kernel launch failed while the
 * call was enqueueing its work: the launches before it may already be on
 * the stream (a partial solve or table build), so the outputs, and after a
 * failed bind the tables, are undefined until a later call succeeds.
 * Faults inside already-enqueued kernels surface at the caller's next
 * stream synchronisation.  No call aborts or throws.
 */
#ifndef MPOLE_H
#define MPOLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPOLE_ABI_VERSION 2
#define MPOLE_LMAX_MAX 64
#define MPOLE_GRADIENT_MAX_NPHI ((1 << 28) - 1)   /* longest phi row of mpole_gradient / mpole_gravity_sources */

typedef enum {
  MPOLE_OK = 0,
  MPOLE_ERR_INVALID = 1,     /* bad argument: null pointer, bad size, non-monotone edges, ... */
  MPOLE_ERR_RANGE = 2,       /* r^(l+3) or r^(2-l) leaves [1e-290, 1e290] for a nonzero edge */
  MPOLE_ERR_WORKSPACE = 3,   /* workspace missing, too small or misaligned (256 B) */
  MPOLE_ERR_DEVICE = 4,      /* a HIP runtime call or kernel launch failed */
  MPOLE_ERR_UNSUPPORTED = 5  /* lmax above MPOLE_LMAX_MAX, unknown precision, ... */
} mpole_status;

typedef enum {
  MPOLE_FP64 = 0,            /* both contractions in FP64 (MFMA f64) */
  MPOLE_BF16X3 = 1,          /* both contractions as three-way split BF16 products, FP32 accumulation */
  MPOLE_FP16X2 = 2,          /* both contractions as two-way split FP16 products, per-shell scaling */
  MPOLE_FP64_SEPARABLE = 3,  /* FP64; each contraction as a phi transform and per-m theta transforms
                                (the cell-averaged kernels and solid angles factor in theta and phi;
                                the same sums reordered).  A batch of separable fields runs each
                                field's launches in turn; mpole_plan_copy_table has no table. */
  MPOLE_BF16X3_SEPARABLE = 4 /* the separable form with both phi transforms (the m >= 1 trig modes)
                                as three-way split BF16 products with FP32 accumulation, the density
                                and the theta-synthesis output split on the fly; the m = 0 mode, the
                                theta transforms and the radial sums stay FP64.  Batches and tables
                                as for MPOLE_FP64_SEPARABLE. */
} mpole_precision;

typedef struct mpole_plan_t *mpole_plan;

/*
 * Mesh descriptor (all pointers are HOST pointers; the plan copies them).
 *   nr, ntheta, nphi >= 1; 0 <= lmax <= MPOLE_LMAX_MAX.
 *   r_edges[nr+1]: strictly increasing, finite, r_edges[0] >= 0.
 *   theta_edges[ntheta+1]: strictly increasing within [0, pi].
 *   phi_edges[nphi+1]: strictly increasing, total span at most 2 pi.
 *   nclasses: 0 = no coarsening (every angular cell is its own block);
 *     otherwise shell_class[nr] in [0, nclasses) picks the class of each
 *     shell, and class_block[nclasses][ntheta*nphi] gives each angular cell
 *     (index j*nphi + k) its block id in that class; the ids of a class must
 *     be exactly 0..nblocks-1, each used at least once.
 *   G: gravitational constant (S = 4 pi G rho); must be finite.
 *   precision: an mpole_precision value.
 */
typedef struct {
  int32_t nr, ntheta, nphi, lmax;
  const double *r_edges;
  const double *theta_edges;
  const double *phi_edges;
  int32_t nclasses;
  const int32_t *shell_class;
  const int32_t *class_block;
  double G;
  int32_t precision;
} mpole_mesh;

/* ABI version of the loaded library (MPOLE_ABI_VERSION). */
int mpole_abi_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char *mpole_last_error(void);

/*
 * Validate a mesh and build a plan on the host (no device work, no HIP call).
 * Returns MPOLE_ERR_INVALID / _RANGE / _UNSUPPORTED for a bad mesh; *out is
 * set only on success.
 */
int mpole_plan_create(const mpole_mesh *mesh, mpole_plan *out);

/* Device workspace the plan needs, in bytes (0 for a null plan). */
size_t mpole_plan_workspace_bytes(mpole_plan plan);

/* Number of angular moments (lmax+1)^2 of a plan (0 for a null plan). */
int mpole_plan_nmodes(mpole_plan plan);

/*
 * 1 if the plan's dense contractions run folded over mirror pairs, else 0
 * (also for a null plan).  A mesh whose theta edges are symmetric about the
 * equator and whose coarsening blocks map onto blocks under theta -> pi -
 * theta has kernels that differ between a block and its mirror image only
 * by the sign (-1)^(l+m) (P~_l^m is even or odd in cos theta); the moment
 * contraction then runs over the sums (even l+m) and differences (odd l+m)
 * of the two blocks' sources, and the expansion over the even and odd mode
 * sums of one block of each pair, giving both blocks' potentials: the same
 * sums of Eqs. AngularMomentsDiscrete and Solution with about half the
 * multiply-adds.  Dense precisions only; the environment variable
 * MPOLE_FOLD=0 at plan creation turns it off.
 */
int mpole_plan_folded(mpole_plan plan);

/*
 * Bind a device workspace (256-byte aligned, at least
 * mpole_plan_workspace_bytes) and enqueue the one-time table construction
 * on hip_stream (a hipStream_t; NULL = default stream): Legendre cell
 * averages by composite Gauss-Legendre quadrature in FP64, phi-cell
 * averages, merged-block kernel tables, radial kernel integrals and, for
 * the split precisions, their split planes (Sec. 2.2: the angular and radial
 * kernels are averaged once, before any solve).  The workspace must stay
 * allocated while the plan is used.  Rebinding is allowed.  Returns after
 * the table construction has completed on hip_stream (the call
 * synchronises it).  The part of the workspace a solve uses for its
 * intermediates is filled with NaN bit patterns here; every solve writes it
 * before reading it.
 */
int mpole_plan_bind(mpole_plan plan, void *dev_workspace, size_t bytes, void *hip_stream);

/*
 * One solve on hip_stream; asynchronous, no allocation, no host sync.
 *   rho  [nr][ntheta][nphi] device, FP64 density (required).
 *   phi  [nr][ntheta][nphi] device, FP64 potential out (may be NULL).
 *   ang_moments [nr][nAM] device, angular moments of S = 4 pi G rho per
 *     shell, Eq. AngularMomentsDiscrete (may be NULL).
 *   interior [nr+1][nAM] device, regular radial moments at shell edges,
 *     edge 0 = 0, outward sums (may be NULL).
 *   exterior [nr+1][nAM] device, irregular radial moments at shell edges,
 *     edge nr = 0, inward sums (may be NULL).
 * Output buffers must not overlap each other or rho.
 */
int mpole_solve(mpole_plan plan, const double *rho, double *phi, double *ang_moments,
                double *interior, double *exterior, void *hip_stream);

/*
 * mpole_solve for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * arguments, kernels and results, but the solve's intermediates (packed
 * operands, split-K partials, moments, coefficients, edge sums) live in a
 * static device array of the library, 256 MiB on each device it runs on,
 * held until the process ends, instead of in the plan's workspace.  The
 * call allocates nothing, host or device, and records no timing events.
 * The plan must be bound (its tables stay in its workspace) on the device
 * that is current at the call.  Every static solve on a device shares that
 * device's array, which keeps the last solve's contents (each solve writes
 * what it reads first), so static solves that overlap on one device race;
 * serialise them (one stream, or events).
 * Errors: MPOLE_ERR_UNSUPPORTED when a solve of this plan needs more than
 * the array holds (checked first, also for an unbound plan),
 * MPOLE_ERR_WORKSPACE for an unbound plan, MPOLE_ERR_INVALID for a null rho
 * or another current device, MPOLE_ERR_DEVICE if the array could not be
 * located at bind or a launch fails.
 */
int mpole_solve_static(mpole_plan plan, const double *rho, double *phi, double *ang_moments,
                       double *interior, double *exterior, void *hip_stream);

/*
 * Copy the FP64 block-averaged kernel table of coarsening class cls
 * ([nblocks][nAM], row b = block b) to host memory, synchronously on
 * hip_stream.  *nblocks receives the block count (query with host_out =
 * NULL first).  For tests of the table construction.
 */
int mpole_plan_copy_table(mpole_plan plan, int32_t cls, double *host_out, int64_t *nblocks,
                          void *hip_stream);

/*
 * Per-phase device timing for profiling.  While enabled, every solve records
 * a pair of HIP events around each of its kernels on the solve's stream (host
 * event objects only; no device memory).  mpole_plan_phase_ms synchronises
 * the recorded events, writes the summed milliseconds and launch counts per
 * phase, and clears the record.  Phases: MPOLE_PHASE_PACK (density
 * streaming), _MOMENT (moment contraction), _REDUCE (split-K sum), _SCAN
 * (radial sums and coefficients), _SPLIT (coefficient split, split
 * precisions only), _EXPAND (expansion contraction and potential streaming),
 * _BCAST (the potential of merged blocks of banded coarsening classes copied
 * from each block's first cell to its other cells).
 */
enum {
  MPOLE_PHASE_PACK = 0, MPOLE_PHASE_MOMENT = 1, MPOLE_PHASE_REDUCE = 2, MPOLE_PHASE_SCAN = 3,
  MPOLE_PHASE_SPLIT = 4, MPOLE_PHASE_EXPAND = 5, MPOLE_PHASE_BCAST = 6, MPOLE_NPHASES = 7
};
int mpole_plan_set_timing(mpole_plan plan, int enable);
int mpole_plan_phase_ms(mpole_plan plan, double *total_ms, int64_t *launches);

/*
 * Algorithmic work of one solve of this plan: flops of the two angular
 * contractions counted on merged blocks (2 per block x shell x mode, each),
 * and the minimum HBM bytes of the solve (FP64 rho in, FP64 phi out, the
 * kernel tables read once).  Either pointer may be NULL.
 */
int mpole_plan_work(mpole_plan plan, double *moment_flops, double *expand_flops, double *min_bytes);

/*
 * Launch tuning of the two angular contractions (host only, before bind; the
 * choice changes how the same sums are tiled and split, not what they are):
 *   moment_wgs     workgroup target of the moment contraction, whose K (the
 *                  blocks of a shell) is split over about that many
 *                  workgroups; 0 = default (about one round of resident
 *                  workgroups).  Split precisions also cap each split at 2048
 *                  blocks, so their FP32 accumulation chains stay short.
 *   moment_tile_m  output tile height (rows = shells) of the moment
 *   expand_tile_m  and of the expansion contraction: 0 = default, 64, or 128
 *                  (128 only for the split precisions; FP64 tiles are 64).
 * mpole_plan_tune returns MPOLE_ERR_UNSUPPORTED for another tile height and
 * MPOLE_ERR_INVALID after bind; it changes mpole_plan_workspace_bytes.
 * mpole_plan_get_tuning reports the plan's current choice (moment_wgs = the
 * target in use).  mpole_plan_configure(plan, w) is mpole_plan_tune with
 * {w, 0, 0}; mpole_plan_moment_wgs reports the moment launch size.  These
 * are the knobs the package's autotuner searches.
 */
/*
 * Coordinate gradient of a potential on the plan's mesh, for the
 * gravitational source terms -rho grad Phi and -rho v . grad Phi of the
 * balance equations (Sec. 3; each derivative the simplest centred difference
 * over the two nearest neighbours).  Writes, on hip_stream, dPhi/dr,
 * dPhi/dtheta and dPhi/dphi at the cell centres (edge midpoints) as
 * (Phi(next) - Phi(previous)) / (x(next) - x(previous)); the first and last
 * shell and theta row use the cell itself for the missing neighbour
 * (one-sided); phi wraps around when phi_edges span 2 pi (to 1e-12),
 * otherwise it is one-sided too; a dimension with one cell gets 0.
 * phi (in) and d_r, d_theta, d_phi (out) are device [nr][ntheta][nphi] FP64
 * (phi fastest), owned by the caller; an output may be NULL (not written).
 * The plan must be bound.  MPOLE_ERR_INVALID for a null plan or phi or an
 * unbound plan, MPOLE_ERR_UNSUPPORTED for nphi > MPOLE_GRADIENT_MAX_NPHI,
 * MPOLE_ERR_DEVICE for a launch failure.  Asynchronous, no allocation,
 * graph-capturable.
 */
int mpole_gradient(mpole_plan plan, const double *phi, double *d_r, double *d_theta, double *d_phi,
                   void *hip_stream);

/*
 * Gravitational sources of the balance equations (Sec. 3, the source vector
 * of the gravitational collapse problems), from the same centred
 * differences as mpole_gradient: the momentum covector source
 * s_i = -rho dPhi/dx^i for x = (r, theta, phi), and the energy source
 * s_energy = -rho v . grad Phi = -rho sum_i v^i dPhi/dx^i with v^i the
 * contravariant velocity components.  phi and rho (mass density, in) are
 * required; v_r, v_theta, v_phi (in) may be NULL (that component counts as
 * zero); s_r, s_theta, s_phi, s_energy (out) may be NULL (not written).
 * All are device [nr][ntheta][nphi] FP64 (phi fastest), owned by the caller;
 * outputs must not overlap the inputs.  One pass over the mesh.  The plan
 * must be bound.  MPOLE_ERR_INVALID for a null plan, phi or rho or an
 * unbound plan, MPOLE_ERR_UNSUPPORTED for nphi > MPOLE_GRADIENT_MAX_NPHI,
 * MPOLE_ERR_DEVICE for a launch failure.  Asynchronous on hip_stream, no
 * allocation, graph-capturable.
 */
int mpole_gravity_sources(mpole_plan plan, const double *phi, const double *rho, const double *v_r,
                          const double *v_theta, const double *v_phi, double *s_r, double *s_theta,
                          double *s_phi, double *s_energy, void *hip_stream);

/*
 * Coarsening operation of Sec. 2.3 on the plan's blocks: every cell of a
 * coarsening block receives the volume-weighted mean of the block,
 * sum_j V_j K_j / sum_j V_j over its member cells j (within a shell the
 * volumes are proportional to the solid angles); a block of one cell keeps
 * its value.  This is how the paper averages the Runge-Kutta updates of the
 * balanced densities; it is also the block mean the solve applies to its
 * density.  in (read) and out (written) are device [nr][ntheta][nphi] FP64,
 * owned by the caller; in == out (in place) is allowed, other overlap is
 * not.  The plan must be bound.  MPOLE_ERR_INVALID for a null plan, in or
 * out or an unbound plan, MPOLE_ERR_DEVICE for a launch failure.
 * Asynchronous on hip_stream, no allocation, graph-capturable.
 */
int mpole_coarsen(mpole_plan plan, const double *in, double *out, void *hip_stream);

/*
 * GenASiS spherical mesh with automatic angular coarsening (Sec. 2.1; the
 * mesh parameters of Sec. 3), built on the host (no HIP call).
 *
 * Radius: a core r < r_core of N_core shells of uniform width
 * dr_min = r_core / N_core, then shells growing by the factor (1 + 1/N_core)
 * each (dr proportional to r, so the polar/radial aspect ratio stays at its
 * value at r_core); N_core = N_theta / core_ratio to the nearest integer,
 * N_r = floor(r_radial * N_theta) (with a 1e-9 guard against the rounding of
 * the product).  theta: N_theta uniform cells on [0, pi]; phi: 2 N_theta
 * uniform cells on [0, 2 pi] (dphi = dtheta).  dims 2 has one phi cell and
 * dims 1 one theta cell as well.
 *
 * Coarsening: in each shell, angular cells narrower than the coarsening
 * width (dr_coarsen, or dr_min when 0) are grouped into aligned blocks of
 * 2, 4, 8, ... cells per dimension: the theta group is the smallest power of
 * two c with c r dtheta >= width, then the phi group of each theta block is
 * the smallest power of two c with c r sin(theta) dphi >= width for every
 * row of the block (its row nearest the axis decides), r and theta at cell
 * centres (coordinate midpoints); each group is capped at the largest power
 * of two dividing the cell count of its dimension.  A cell's coarsening
 * factors c_i (Sec. 2.3) are its block's group sizes.
 *
 * Output in the layout of mpole_mesh: shells with equal block patterns form
 * one class (numbered by first shell), block ids of a class are numbered by
 * first member cell (j * nphi + k), so the arrays feed mpole_plan_create
 * directly.
 */
typedef struct {
  int32_t dims;        /* 1, 2 or 3 */
  int32_t ntheta;      /* resolution parameter N_theta, 1..65536 */
  double r_core;       /* core radius, > 0 */
  double core_ratio;   /* N_theta / N_core, > 0; 0 = 32/25 (the paper's choice) */
  double r_radial;     /* N_r / N_theta, > 0 */
  double dr_coarsen;   /* coarsening width, >= 0; 0 = dr_min */
} mpole_genasis;

/*
 * Sizes of the GenASiS mesh: shells, theta and phi cells, core shells and
 * coarsening classes (any output may be NULL).  MPOLE_ERR_INVALID for bad
 * parameters (N_core or N_r outside 1..2^20 included), MPOLE_ERR_RANGE when
 * the outer radius overflows.
 */
int mpole_genasis_shape(const mpole_genasis *params, int32_t *nr, int32_t *ntheta, int32_t *nphi,
                        int32_t *ncore, int32_t *nclasses);

/*
 * Fill caller-owned HOST arrays sized by mpole_genasis_shape:
 * r_edges[nr+1], theta_edges[ntheta+1], phi_edges[nphi+1], shell_class[nr],
 * class_block[nclasses][ntheta*nphi]; optionally (NULL = skip) c_theta[nr]
 * (theta group of each shell) and c_phi[nr][ntheta] (phi group of the block
 * holding each row).  Errors as mpole_genasis_shape, plus MPOLE_ERR_INVALID
 * for a null required array; nothing is written on error.
 */
int mpole_genasis_build(const mpole_genasis *params, double *r_edges, double *theta_edges, double *phi_edges,
                        int32_t *shell_class, int32_t *class_block, int32_t *c_theta, int32_t *c_phi);

typedef struct {
  int32_t moment_wgs;
  int32_t moment_tile_m;
  int32_t expand_tile_m;
} mpole_tuning;
int mpole_plan_tune(mpole_plan plan, const mpole_tuning *tuning);
int mpole_plan_get_tuning(mpole_plan plan, mpole_tuning *tuning);
int mpole_plan_configure(mpole_plan plan, int32_t moment_wgs);
int mpole_plan_moment_wgs(mpole_plan plan);

/* Free the plan's host memory (the workspace stays the caller's). NULL is a no-op. */
int mpole_plan_destroy(mpole_plan plan);

/*
 * Batched solve of many independent fields with uneven meshes and lmax (one
 * plan per field, all with the same precision).  A batch solve enqueues no
 * host synchronisation, allocation or memset, so it can be captured in a HIP
 * graph and replayed.  It runs in one of two ways:
 *
 * MPOLE_LAUNCH_PERSISTENT (the default where it applies): ONE launch of a
 *   persistent kernel (plus a small reset kernel) does every phase of every
 *   field.  At bind the library reads which XCD (accelerator die, with its
 *   own L2 cache) each workgroup runs on, and lays out one work queue per
 *   XCD: whole fields, spread over the queues by their estimated work and
 *   ordered shortest first within a queue, each field as its phases in solve
 *   order, each phase as items (one or a group of workgroups of the phase's
 *   own kernel).  A workgroup takes the next item of its own XCD's queue,
 *   waits until the field's previous phase is complete, and runs the item
 *   with the same device code as the per-phase kernels, so results are
 *   bitwise those of MPOLE_LAUNCH_PHASES.  Small fields complete early (see
 *   mpole_batch_field_ms).  Every dependency wait is bounded: after
 *   wait_polls polls it sets an error word, skips its item and the launch
 *   ends normally; mpole_batch_check reports it.  A batch launches per phase
 *   instead when its fields are separable, when a field has coarsened blocks
 *   of more than 64 cells, when the XCD ids do not follow the round-robin
 *   dispatch of workgroups, or when the fields cannot be spread over the
 *   queues within 1.25 times the mean estimated queue work
 *   (mpole_batch_launch_note says which).
 * MPOLE_LAUNCH_PHASES: every phase of the solve is ONE kernel launch
 *   covering all fields (workgroups are assigned to fields by prefix sums), a
 *   fixed sequence of a few launches.  Separable fields
 *   (MPOLE_FP64_SEPARABLE, MPOLE_BF16X3_SEPARABLE) are solved one after
 *   another, each field's launches filling the device on their own.
 *
 * mpole_batch_create: nfields in [1, 4096] meshes (host descriptors, copied);
 *   MPOLE_ERR_INVALID if their precisions differ.
 * mpole_batch_tune: optional per-field launch tuning ([nfields], see
 *   mpole_plan_tune; a zero moment_wgs means the field's share of one round of
 *   resident workgroups), before bind.  mpole_batch_configure(batch, w) is
 *   mpole_batch_tune with {w[f], 0, 0} per field.
 * mpole_batch_bind: binds one device workspace (256-byte aligned) holding all
 *   fields' plans, builds every field's tables on hip_stream, and records the
 *   fields' device I/O pointers rho[f] ([nr][ntheta][nphi] FP64 in) and
 *   phi[f] (same shape, FP64 out); the two host arrays are copied.
 * mpole_batch_solve: one solve of every field on hip_stream (asynchronous).
 * mpole_batch_field_ms: after the caller has synchronised the stream, the
 *   time from the start of the last batch solve to the completion of each
 *   field's potential, in milliseconds (device wall clock), into ms[nfields].
 */
typedef struct mpole_batch_t *mpole_batch;
int mpole_batch_create(int32_t nfields, const mpole_mesh *meshes, mpole_batch *out);
int mpole_batch_tune(mpole_batch batch, const mpole_tuning *tunings);
int mpole_batch_configure(mpole_batch batch, const int32_t *moment_wgs);
/* Per-field launch tuning in use ([nfields]; moment_wgs = each field's target). */
int mpole_batch_get_tuning(mpole_batch batch, mpole_tuning *tunings);
size_t mpole_batch_workspace_bytes(mpole_batch batch);
int mpole_batch_bind(mpole_batch batch, void *dev_workspace, size_t bytes, const double *const *rho,
                     double *const *phi, void *hip_stream);
int mpole_batch_solve(mpole_batch batch, void *hip_stream);
int mpole_batch_field_ms(mpole_batch batch, double *ms);
int mpole_batch_destroy(mpole_batch batch);

#define MPOLE_LAUNCH_PHASES 0
#define MPOLE_LAUNCH_PERSISTENT 1
#define MPOLE_LAUNCH_PERSISTENT_FORCED 2   /* persistent also when the queues are unbalanced */
/*
 * mpole_batch_set_launch: the launch later solves use (MPOLE_LAUNCH_PHASES,
 *   MPOLE_LAUNCH_PERSISTENT where the batch allows it, see above, or
 *   MPOLE_LAUNCH_PERSISTENT_FORCED, which skips only the balance condition:
 *   a batch of fewer fields than XCDs then leaves XCDs idle) and the
 *   wait budget of the persistent launch in polls (0: the default, 2^22
 *   polls, seconds of waiting).  Any time; a captured graph
 *   keeps the launch it captured.  MPOLE_ERR_INVALID for a null batch or an
 *   unknown launch.
 * mpole_batch_launch: for a bound batch, the launch the next solve runs; -1
 *   for a null or unbound batch.
 * mpole_batch_launch_note: why a bound batch does not run the persistent
 *   launch under MPOLE_LAUNCH_PERSISTENT ("" when it does, and for a null or
 *   unbound batch); the string belongs to the batch.
 * mpole_batch_check: synchronises hip_stream and, if the last solve ran the
 *   persistent launch and one of its dependency waits gave up (its
 *   potentials are then undefined), returns MPOLE_ERR_DEVICE; MPOLE_OK
 *   otherwise.  MPOLE_ERR_WORKSPACE for an unbound batch.
 */
int mpole_batch_set_launch(mpole_batch batch, int32_t launch, uint32_t wait_polls);
int mpole_batch_launch(mpole_batch batch);
const char *mpole_batch_launch_note(mpole_batch batch);
int mpole_batch_check(mpole_batch batch, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MPOLE_H */
