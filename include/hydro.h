/* hydro.h -- C ABI of the MI355X patch-group Euler solver (libhydro.so).
 *
 * The library advances the patch groups of one AMR level with the
 * dimensionally unsplit MUSCL-Hancock scheme (MHM: PLM reconstruction with a
 * generalized minmod limiter, HLLC Riemann solver, conservative update) and
 * computes the per-patch CFL time-step, following Schive et al. 2018
 * (GAMER-2), Sec. 2.2 (hydrodynamic schemes, Riemann solvers, limiters,
 * boundary conditions), Sec. 2.6 Eq. 2 (CFL condition for MHM), Sec. 3.1 and
 * Sec. 3.4 (patch groups of 2x2x2 sibling 8^3 patches, ghost zones allocated
 * only for the groups being solved).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers named *_dev are DEVICE pointers (HIP device memory of the current
 * device); pointers named *_host are host memory.  The caller allocates and
 * frees every buffer; the library keeps no pointer after a call returns.
 *
 * Fields: 5 conserved variables per cell in this order: rho, m_x, m_y, m_z, E
 * (mass density, momentum density, total energy density).  Ideal gas,
 * p = (gamma-1) (E - |m|^2 / (2 rho)).  Cubic cells of width dx.
 *
 * Level storage ("group-major"): float array [G][5][16][16][16], x fastest;
 * group g = (gz*NGy + gy)*NGx + gx on an NGx x NGy x NGz lattice of groups.
 *
 * Padded groups: float array [G][5][P][P][P], P = 16 + 2*ghost, x fastest; the
 * group interior sits at offsets ghost..ghost+15 on each axis.  The MHM step
 * reads the inner 2 ghost layers only (the stencil of PLM + Hancock + HLLC),
 * so ghost >= 2; configurations of the paper's CTU/PPM kind carry 3.
 *
 * dtype: HYDRO_F64 (double) or HYDRO_F32 (float) for every state array of a
 * call.  Time-steps are always double.
 *
 * Scheme word: bits 0-7 scheme id (HYDRO_SCHEME_MHM_PLM_HLLC), bits 8-9 HLLC
 * wave-speed estimate (HYDRO_WAVESPEED_ROE: Einfeldt/Roe-averaged, default;
 * HYDRO_WAVESPEED_DAVIS), bit 10 HYDRO_FIRST_ORDER (zero slopes: Godunov with
 * HLLC).  theta is the generalized-minmod parameter, 1 <= theta <= 2.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = null stream).
 * Every call is asynchronous on it; argument errors are reported
 * synchronously by the return value and nothing is launched.
 *
 * Status: HYDRO_OK (0), HYDRO_UNPHYSICAL (1, only from hydro_check_unphysical),
 * or a negative error code; hydro_strerror() names it.  HYDRO_EDEVICE means a
 * HIP call failed; hydro_last_hip_error() returns it.
 *
 * Context: the entry points whose kernels come in several launch shapes
 * (level step, batched step, adjoint) take a hydro_ctx* first.  The context
 * holds the caller's shape selections (set explicitly or autotuned, the
 * latter keyed by dtype and level lattice), optionally loaded from and saved
 * to a tuning-cache JSON file, and the graphs captured through it; two
 * contexts in one process never see each other's selections.  NULL selects
 * the measured defaults.  A context is used by one thread at a time for
 * tuning; launches through one context from several threads are safe.
 *
 * Determinism: for the same inputs, arguments and device the outputs are
 * bitwise identical from run to run (no floating-point atomics).
 */
#ifndef HYDRO_H_
#define HYDRO_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HYDRO_OK 0
#define HYDRO_UNPHYSICAL 1   /* hydro_check_unphysical: >= 1 unphysical item was counted */
#define HYDRO_EINVAL (-1)    /* bad shape, ghost, dtype, null pointer, aliasing, dt/dx/gamma/theta */
#define HYDRO_EDEVICE (-2)   /* a HIP runtime call failed */
#define HYDRO_ENOTUNED (-3)  /* the context requires a tuned shape and has none for this call */
#define HYDRO_EIO (-4)       /* tuning cache unreadable, malformed or not writable */

/* Opaque solver context (launch-shape selections, tuning cache, graphs). */
typedef struct hydro_ctx hydro_ctx;

#define HYDRO_F64 0
#define HYDRO_F32 1

#define HYDRO_SCHEME_MHM_PLM_HLLC 1
#define HYDRO_WAVESPEED_ROE (0 << 8)
#define HYDRO_WAVESPEED_DAVIS (1 << 8)
#define HYDRO_FIRST_ORDER (1 << 10)
/* Further scheme-word fields (Sec. 2.2), accepted by hydro_advance_ext only:
 * bits 0-7 scheme id MHM (= HYDRO_SCHEME_MHM_PLM_HLLC) or CTU (6 Riemann
 * solves per cell); bits 11-12 slope limiter; bit 13 limit characteristic
 * instead of primitive variables; bit 14 PPM instead of PLM; bits 16-17
 * Riemann solver; bit 18 dual energy (a sixth field per cell). */
#define HYDRO_SCHEME_MHM 1
#define HYDRO_SCHEME_CTU 2
#define HYDRO_LIMITER_GMINMOD (0 << 11)
#define HYDRO_LIMITER_VANLEER (1 << 11)
#define HYDRO_LIMITER_VANALBADA (2 << 11)
#define HYDRO_LIMITER_HYBRID (3 << 11)
#define HYDRO_CHARACTERISTIC (1 << 13)
#define HYDRO_PPM (1 << 14)
#define HYDRO_RIEMANN_HLLC (0 << 16)
#define HYDRO_RIEMANN_ROE (1 << 16)
#define HYDRO_RIEMANN_HLLE (2 << 16)
#define HYDRO_DUAL_ENERGY (1 << 18)

#define HYDRO_BC_PERIODIC 0
#define HYDRO_BC_OUTFLOW 1

/* Context (the solver's launch configuration, Sec. 3.1: the GPU solver is
 * configured once and then advances patch groups call after call).
 *   hydro_ctx_create    *ctx receives a new context.  tune_cache_json_path
 *                       (host string, may be NULL): a file of tuned shapes,
 *                       {"version": 1, "entries": {"<key>": <shape>, ...}},
 *                       read now if it exists (HYDRO_EIO if malformed) and
 *                       rewritten after every autotune call.  Keys name the
 *                       kernel, dtype and lattice, e.g. "level/f64/cfl/16x16x16",
 *                       "adjoint/f32/24x24x24", "batched/f64/8x8x8+8x8x24".
 *   hydro_ctx_destroy   destroys the graphs still owned by ctx, frees ctx.
 *   hydro_ctx_save      writes the cache file now (HYDRO_OK if no path).
 *   hydro_ctx_set_require_tuned  on != 0: a launch with no tuned (or cached)
 *                       shape for its key and no explicit selection returns
 *                       HYDRO_ENOTUNED instead of using the default.
 *   hydro_ctx_num_tuned number of tuned entries held (>= 0).
 * Shape lookup of a launch: the tuned entry for its key, else the explicit
 * selection (hydro_set_*_variant), else the default. */
int hydro_ctx_create(hydro_ctx** ctx, const char* tune_cache_json_path);
int hydro_ctx_destroy(hydro_ctx* ctx);
int hydro_ctx_save(hydro_ctx* ctx);
int hydro_ctx_set_require_tuned(hydro_ctx* ctx, int32_t on);
int hydro_ctx_num_tuned(hydro_ctx* ctx);

/* hydro_check_unphysical -- waits for `stream`, reads the device int32
 * n_bad_dev that the steps add their unphysical counts to (Sec. 2.2: results
 * with rho <= 0 or p <= 0 are detected) and returns HYDRO_UNPHYSICAL if it is
 * positive, HYDRO_OK if not; *n_bad_host (optional) receives the count.
 * SYNCHRONOUS.  The counter is not reset. */
int hydro_check_unphysical(const int32_t* n_bad_dev, void* stream, int32_t* n_bad_host);

/* hydro_advance -- one MHM step of G padded patch groups (Sec. 2.2: MHM with
 * PLM on primitive variables, generalized minmod limiter, HLLC solver, and the
 * conservative flux-difference update).
 *   U_pad_dev  [G][5][P^3] input state with filled ghost zones (not modified)
 *   U_out_dev  [G][5][16^3] output interiors (level storage); must not overlap
 *              U_pad_dev
 *   n_groups   G >= 0 (0 launches nothing)
 *   ghost      2..16
 *   dt, dx     > 0; if dt_dev is non-NULL the step reads dt from that device
 *              double instead (lets a CFL time-step stay on the device)
 *   gamma > 1, scheme, theta in [1, 2]: see above
 *   n_bad_dev  optional device int32 (may be NULL): the kernel ADDS the
 *              number of unphysical items (HLLC faces whose two input states
 *              are not both rho > 0 and p > 0, plus updated cells with rho <= 0
 *              or p <= 0).  No floors or fallbacks are applied.
 */
int hydro_advance(const void* U_pad_dev, void* U_out_dev, int64_t n_groups, int32_t ghost,
                  int32_t dtype, double dt, double dx, double gamma, int32_t scheme,
                  double theta, const double* dt_dev, int32_t* n_bad_dev, void* stream);

/* hydro_branch_record -- hydro_advance (FP64 only, dt on the host, no
 * unphysical count) that also writes every group's branch record to
 * record_dev[G] (device uint32): each thread of the group hashes the code of
 * every decision the step's arithmetic takes -- the limiter case and the
 * argument attaining its minimum (first on ties), the first or second
 * argument of each wave-speed minimum / maximum, the HLLC region -- in its
 * own order, and the threads' hashes are combined by XOR.  Two steps whose
 * records agree took the same branches (up to a 2^-32 collision), so their
 * results lie on one smooth piece of the step: the check a finite-
 * difference test of the adjoint needs (Sec. 2.2 arithmetic; the record is a
 * diagnostic of this library, not of the paper).  The state written equals
 * hydro_advance's bit for bit.  HYDRO_EINVAL for FP32 or invalid arguments. */
int hydro_branch_record(const void* U_pad_dev, void* U_out_dev, int64_t n_groups, int32_t ghost, int32_t dtype,
                        double dt, double dx, double gamma, int32_t scheme, double theta, uint32_t* record_dev,
                        void* stream);

/* hydro_advance_ext -- one step of G padded groups with any scheme of
 * Sec. 2.2 that the scheme word names (hydro_advance's arguments and
 * semantics, plus a workspace):
 *   MHM: face values, then the conservative Hancock half step with the three
 *        axes' face-value flux differences, then a Riemann solve at every
 *        face, then the conservative update;
 *   CTU (Colella 1990, 6 Riemann solves per cell): face values and a half
 *        step with each axis' own flux difference; first Riemann solves at
 *        every face; each axis' states corrected by dt/(2dx) times the other
 *        two axes' first-solve flux differences; second solves; update.
 *   Face values: PLM (W0 -+ s/2) or PPM (Colella & Woodward 1984: fourth-
 *   order interface values from the limited slopes of the three nearest
 *   cells, then the monotonicity constraints), with slopes limited on
 *   primitive or characteristic variables (left/right eigenvectors of the
 *   primitive Euler system of the cell); limiters: generalized minmod
 *   (theta), van Leer (harmonic mean), van Albada, hybrid (the smaller of
 *   generalized minmod and van Leer).  Solvers: HLLC, HLLE (Einfeldt), Roe
 *   (no entropy fix; a face whose linearized intermediate states are
 *   unphysical takes the HLLC flux, the first step of the paper's procedure
 *   for unphysical results).
 *   Dual energy (HYDRO_DUAL_ENERGY, Sec. 2.2): every state array has 6
 *   fields, [G][6][P^3] in and [G][6][16^3] out, field 5 the entropy per
 *   unit volume s = p / rho^(gamma-1), advected as a passive scalar (s/rho
 *   reconstructed like a primitive variable; Riemann flux = mass flux times
 *   s/rho of the upwind side); after the update E = s rho^(gamma-1)/(gamma-1)
 *   + E_kin where E - E_kin < xi E_kin, else s is reset from E.  xi >= 0 (the
 *   paper's typical 1e-2); ignored without the bit.  Not with face_flux_dev.
 *   ghost       >= 2, and >= 3 with PPM
 *   work_dev    device scratch of work_bytes bytes, at least
 *               hydro_ext_workspace_bytes(1, ghost, dtype, scheme); groups are
 *               processed in chunks of as many groups as it holds (all at
 *               once with hydro_ext_workspace_bytes(G, ...)); must not overlap
 *               U_pad_dev or U_out_dev.  MHM + PLM words without dual
 *               energy (any limiter, primitive or characteristic variables,
 *               any solver or wave-speed option, second or first order) run
 *               in the fused per-group kernel of hydro_advance (the default
 *               word in its own specialized copy) and need no workspace
 *               (their hydro_ext_workspace_bytes is 0; work_dev may be NULL);
 *               CTU, PPM and dual energy run as a chain of kernels through it
 *   n_bad_dev   as for hydro_advance (faces with unphysical input states plus
 *               updated cells with rho <= 0 or p <= 0)
 *   face_flux_dev  optional [G][9][5][16][16] output: the fluxes the update
 *               used on the faces of the patch boundaries of every group (the
 *               flux registers of coarse-fine coupling): plane p = 3 axis + k
 *               holds that axis' faces at normal coordinate 8 k (the face
 *               between cells 8k-1 and 8k), entry [p][field][b][a] with a, b
 *               the transverse coordinates in the cyclic order (axis+1,
 *               axis+2); must not overlap the other buffers
 * hydro_ext_workspace_bytes returns the bytes for n_groups groups, or
 * HYDRO_EINVAL for an invalid scheme word / ghost / dtype. */
int64_t hydro_ext_workspace_bytes(int64_t n_groups, int32_t ghost, int32_t dtype, int32_t scheme);
int hydro_advance_ext(const void* U_pad_dev, void* U_out_dev, int64_t n_groups, int32_t ghost, int32_t dtype,
                      double dt, double dx, double gamma, int32_t scheme, double theta, double xi,
                      const double* dt_dev, int32_t* n_bad_dev, void* work_dev, int64_t work_bytes,
                      void* face_flux_dev, void* stream);

/* Procedure for unphysical results (Sec. 2.2: a cell whose update gives
 * rho <= 0 or p <= 0 is (ii) recomputed first-order in space and time,
 * dimensionally unsplit; (iii) if that fails, first-order and dimensionally
 * split; (iv)-(v) if that fails too, the whole level is recomputed with the
 * time-step reduced by a fixed ratio until nothing fails or a minimum
 * time-step is reached).  Step (i), the switch of Roe's solver to HLLC on a
 * face with an unphysical intermediate state, is part of the Roe solver.
 *
 * hydro_repair_unphysical -- steps (ii)-(iii) on a level after a step:
 *   level_in_dev   [G][5][16^3] the step's input level (not modified)
 *   level_out_dev  [G][5][16^3] the step's output; every cell with rho <= 0 or
 *                  p <= 0 is replaced by its first-order unsplit recomputation
 *                  from level_in_dev (Riemann fluxes of the scheme's solver on
 *                  the cell averages of its six faces, summed x, y, z), or, if
 *                  that is unphysical too, by its first-order split
 *                  recomputation (x, y, z sweeps over the 3x3x3 block around
 *                  it); neighbours beyond the level follow bc_host
 *   scheme         only the Riemann solver and wave-speed fields are used
 *   dt, dt_dev     the step's time-step (dt_dev: device double read instead)
 *   counts_dev     3 device int32, ADDED to: cells repaired unsplit, cells
 *                  repaired split, cells still unphysical
 *   Asynchronous on stream; level limits as hydro_advance_level.
 *
 * hydro_fallback_workspace_bytes -- device scratch hydro_advance_level_fallback
 *   needs for a level (256 B of counters; for scheme words other than the
 *   fused step's, also a padded copy with 3 ghosts and the
 *   hydro_advance_ext workspace), or HYDRO_EINVAL.
 *
 * hydro_advance_level_fallback -- steps (ii)-(v): one step of the level
 *   (hydro_advance_level for the default scheme word, else hydro_fill_ghosts
 *   + hydro_advance_ext), then, if the step counted unphysical items,
 *   hydro_repair_unphysical; while cells remain unphysical and dt * ratio >=
 *   dt_min, the level is recomputed from level_in_dev with dt *= ratio.
 *   ratio in (0, 1) (0.8 in the paper), dt_min >= 0.
 *   work_dev, work_bytes  at least hydro_fallback_workspace_bytes(...)
 *   info_host      4 doubles: the dt of the last attempt, the number of
 *                  retries, the cells repaired unsplit and split in it
 *   Returns HYDRO_OK (no cell left unphysical), HYDRO_UNPHYSICAL (cells still
 *   unphysical at the last dt allowed; level_out_dev holds that attempt) or
 *   an error.  SYNCHRONOUS: waits on `stream` after each attempt.
 */
int hydro_repair_unphysical(const void* level_in_dev, void* level_out_dev, int32_t ngx, int32_t ngy, int32_t ngz,
                            const int32_t* bc_host, int32_t dtype, double dt, double dx, double gamma, int32_t scheme,
                            const double* dt_dev, int32_t* counts_dev, void* stream);
int64_t hydro_fallback_workspace_bytes(int32_t ngx, int32_t ngy, int32_t ngz, int32_t dtype, int32_t scheme);
int hydro_advance_level_fallback(hydro_ctx* ctx, const void* level_in_dev, void* level_out_dev, int32_t ngx,
                                 int32_t ngy, int32_t ngz, const int32_t* bc_host, int32_t dtype, double dt,
                                 double dt_min, double ratio, double dx, double gamma, int32_t scheme, double theta,
                                 void* work_dev, int64_t work_bytes, double* info_host, void* stream);

/* Coarse-fine coupling of AMR levels (Sec. 2.1: patches of 8^3 cells,
 * refinement ratio 2, the 8 children of a coarse patch form one fine patch
 * group; levels advance in a W-cycle with dt_l = dt_0 / 2^l.  Sec. 2.2: after
 * a coarse level is synchronized with its children, coarse cells covered by
 * them are restricted and uncovered coarse cells at the coarse-fine
 * interface are corrected by the difference of coarse and fine fluxes.
 * Sec. 3.2: ghost zones of a fine group come from sibling groups or by
 * interpolation from the coarse level).
 *
 * A level is described by hydro_amr_level_t: its states, its group
 * positions on the level's group lattice (level l has n_0 * 2^l groups per
 * axis over the domain; a fine group at position p covers coarse patch p,
 * i.e. coarse cells 8p .. 8p+7 per axis) and the dense map of that lattice
 * (group index, or -1 where the level has no group), all device memory.
 * Level 0 covers the domain.  A fine level must be properly nested: the 27
 * coarse patches around the parent patch of every fine group exist on the
 * coarse level (the caller guarantees it; the Python binding checks it). */
typedef struct {
  void* U_dev;             /* [G][5][16^3] states of the level */
  const int32_t* pos_dev;  /* [G][3] group positions (x, y, z) */
  const int32_t* map_dev;  /* [n[2]][n[1]][n[0]] group index or -1 */
  int64_t n_groups;
  int32_t n[3];            /* group lattice of the level over the domain */
} hydro_amr_level_t;

/* hydro_amr_fill_ghosts -- padded groups [G][5][P^3] of level `fine`
 *   (P = 16 + 2 ghost, 0 <= ghost <= 16): a ghost cell is copied from the
 *   sibling group holding it, else interpolated from `coarse` (NULL only for
 *   level 0): time-linear between coarse_old_dev and coarse_new_dev (the
 *   coarse step's input and output, [G_c][5][16^3]) at weight a in [0, 1],
 *   space-conservative-linear (coarse value + minmod-limited slopes of the
 *   conserved variables times the +-1/4-cell offsets of the child, summed x,
 *   y, z).  bc_host: the domain's boundary conditions.
 * hydro_amr_flux_accumulate -- flux registers reg_dev [G_f][6][5][8][8]
 *   (sides x-, x+, y-, y+, z-, z+; field; the coarse face's transverse
 *   coordinates (b, a) in cyclic order) ADD weight * (1/4) * the sum of the
 *   2x2 fine faces over each coarse face, from face_flux_dev (the
 *   [G_f][9][5][16][16] output of hydro_advance_ext), on every side of a
 *   fine group with no sibling group across it (weight = dt_f / dt_c).
 * hydro_amr_restrict -- every coarse cell covered by a fine group becomes the
 *   mean of its 8 children (coarse->U_dev is written).
 * hydro_amr_fixup -- every uncovered coarse cell sharing a face with a fine
 *   group: U += dt_over_dx (R - F_c) if the face is its low face, -= if its
 *   high face, sides in the order x-, x+, y-, y+, z-, z+; F_c from
 *   coarse_face_flux_dev (the coarse step's hydro_advance_ext face fluxes),
 *   R from reg_dev.
 * All asynchronous on stream; dtype of every state / flux array. */
int hydro_amr_fill_ghosts(const hydro_amr_level_t* fine, const hydro_amr_level_t* coarse, const void* coarse_old_dev,
                          const void* coarse_new_dev, double a, const int32_t* bc_host, int32_t ghost, int32_t dtype,
                          void* U_pad_dev, void* stream);
int hydro_amr_flux_accumulate(const hydro_amr_level_t* fine, const void* face_flux_dev, double weight,
                              const int32_t* bc_host, int32_t dtype, void* reg_dev, void* stream);
int hydro_amr_restrict(const hydro_amr_level_t* fine, const hydro_amr_level_t* coarse, int32_t dtype, void* stream);
int hydro_amr_fixup(const hydro_amr_level_t* coarse, const hydro_amr_level_t* fine, const void* coarse_face_flux_dev,
                    const void* reg_dev, double dt_over_dx, const int32_t* bc_host, int32_t dtype, void* stream);

/* hydro_advance_level -- one MHM step of every patch group of a level, read
 * directly from level storage (Sec. 2.2 scheme; Sec. 3.4 ghost zones; Sec. 2.6
 * Eq. 2 for the optional CFL outputs).  Each cell the stencil reaches outside
 * a group (2 layers) is read from the neighbouring group with the index map
 * of hydro_fill_ghosts, so the result equals hydro_fill_ghosts followed by
 * hydro_advance, without the padded copy.
 *   level_dev       [G][5][16^3] input level, G = ngx*ngy*ngz (not modified);
 *                   every level entry point takes 1 <= ngx, ngy, ngz <= 2^26
 *                   and G < 2^31 - 8 (else HYDRO_EINVAL)
 *   level_out_dev   [G][5][16^3] output level; must not overlap level_dev
 *   bc_host         6 ints on the host (x-, x+, y-, y+, z-, z+), 0 periodic,
 *                   1 outflow
 *   dt, dt_dev, dx, gamma, scheme, theta, n_bad_dev: as for hydro_advance
 *   c_cfl           CFL safety factor, > 0 if any of the three outputs below
 *                   is requested
 *   dt_next_dev     optional device double: the minimum over all patches of
 *                   the Eq. 2 time-step of the OUTPUT state is folded in with
 *                   an (exact, order-independent) minimum; it must hold +inf
 *                   or a larger value when the step starts
 *   dt_patch_next_dev optional [G][8] double: per-patch Eq. 2 time-steps of
 *                   the output state (bit-identical to hydro_dt on it)
 *   dt_reset_dev    optional device double the step sets to +inf (before any
 *                   other use in the step); lets three buffers rotate over a
 *                   rollout (read dt from A, reduce into B, reset C); must
 *                   differ from dt_dev and dt_next_dev
 */
int hydro_advance_level(hydro_ctx* ctx, const void* level_dev, void* level_out_dev, int32_t ngx, int32_t ngy, int32_t ngz,
                        const int32_t* bc_host, int32_t dtype, double dt, double dx, double gamma, int32_t scheme,
                        double theta, const double* dt_dev, int32_t* n_bad_dev, double c_cfl, double* dt_next_dev,
                        double* dt_patch_next_dev, double* dt_reset_dev, void* stream);

/* Adjoint (vector-Jacobian product) of one MHM step -- the transpose of the
 * Jacobian of hydro_advance / hydro_advance_level with respect to its input
 * state, applied to a cotangent of its output, at the same scheme, dt, dx,
 * gamma and theta (dt fixed, not differentiated).  Recomputes the forward
 * intermediates from the input state.  Derivatives at non-smooth points:
 * limiter zero when the one-sided differences are not of one strict sign,
 * otherwise through the argument attaining the minimum (the first on ties);
 * min/max of wave speeds through the first argument unless the second is
 * strictly smaller/larger; HLLC through the branch the forward takes.
 * Deterministic: no floating-point atomics.
 *
 * hydro_adjoint_workspace_bytes -- bytes of scratch device memory the two
 *   adjoint calls need for n_groups groups (level != 0: the level form, which
 *   stages each group's reachable-cell cotangents before the gather; the
 *   padded form needs none and returns 0); the caller allocates it
 *   (HYDRO_EINVAL on bad arguments).
 *
 * hydro_advance_adjoint -- padded form.
 *   U_pad_dev   [G][5][P^3] the step's input (not modified)
 *   gU_out_dev  [G][5][16^3] cotangent of the step's output
 *   gU_pad_dev  [G][5][P^3] receives the cotangent of U_pad (zero on cells
 *               the step does not read)
 *   work_dev, work_bytes  scratch of at least
 *               hydro_adjoint_workspace_bytes(G, dtype, 0) bytes (may be NULL
 *               when that is 0)
 *   No two of U_pad_dev, gU_out_dev, gU_pad_dev, work_dev may overlap.
 *
 * hydro_advance_level_adjoint -- level form (adjoint of hydro_advance_level,
 *   including the ghost fill: cotangents of ghost copies are gathered back to
 *   the cells they copy, in a fixed order).
 *   level_dev        [G][5][16^3] the step's input level (not modified)
 *   g_level_out_dev  [G][5][16^3] cotangent of the step's output level
 *   g_level_in_dev   [G][5][16^3] receives the cotangent of the input level
 *   work_dev, work_bytes  at least hydro_adjoint_workspace_bytes(G, dtype, 1)
 *   dt_dev           optional device double read instead of dt
 *   Lattice limits: those of hydro_advance_level, and also every axis below
 *   2^19 groups and G < 2^28 - 1 (else HYDRO_EINVAL); the same for
 *   hydro_gather_ghost_adjoint.
 */
int64_t hydro_adjoint_workspace_bytes(int64_t n_groups, int32_t dtype, int32_t level);
int hydro_advance_adjoint(hydro_ctx* ctx, const void* U_pad_dev, const void* gU_out_dev, void* gU_pad_dev, int64_t n_groups,
                          int32_t ghost, int32_t dtype, double dt, double dx, double gamma, int32_t scheme,
                          double theta, void* work_dev, int64_t work_bytes, void* stream);
int hydro_advance_level_adjoint(hydro_ctx* ctx, const void* level_dev, const void* g_level_out_dev, void* g_level_in_dev, int32_t ngx,
                                int32_t ngy, int32_t ngz, const int32_t* bc_host, int32_t dtype, double dt, double dx,
                                double gamma, int32_t scheme, double theta, const double* dt_dev, void* work_dev,
                                int64_t work_bytes, void* stream);

/* Form of the two adjoint calls (per context and dtype); both give the same
 * cotangents up to the summation order of the limiter / flux terms:
 *   0  one fused z-march per group (face cotangents stay on chip);
 *   1  two z-marches per group with the face cotangents in the workspace
 *      (smaller LDS and register footprint: two workgroups per CU).
 * hydro_set_adjoint_variant returns HYDRO_EINVAL for other values;
 * hydro_get_adjoint_variant returns the current form. */
int hydro_set_adjoint_variant(hydro_ctx* ctx, int32_t dtype, int32_t variant);
int hydro_get_adjoint_variant(hydro_ctx* ctx, int32_t dtype);

/* hydro_autotune_adjoint -- time both adjoint forms of
 * hydro_advance_level_adjoint on the caller's level (same arguments as that
 * call, dt fixed internally; two passes of 1 untimed + `reps` timed launches
 * per form, 1 <= reps <= 1000, a form's time is the smaller of its two means),
 * record the faster in ctx (non-NULL) for `dtype` and this lattice and return
 * it (0 fused, 1 two kernels), or a negative status (nothing is recorded).  SYNCHRONOUS;
 * g_level_in_dev and the workspace are overwritten; times_ms_host, if not
 * NULL, receives the 2 times in milliseconds.  Results do not depend on the
 * form (within rounding of the 1e-12 parity bound; both are deterministic). */
int hydro_autotune_adjoint(hydro_ctx* ctx, const void* level_dev, const void* g_level_out_dev, void* g_level_in_dev, int32_t ngx,
                           int32_t ngy, int32_t ngz, const int32_t* bc_host, int32_t dtype, double dx, double gamma,
                           void* work_dev, int64_t work_bytes, int32_t reps, float* times_ms_host, void* stream);

/* One level of a batched launch (hydro_advance_batched).  Pointers are
 * device memory; bc holds the x-, x+, y-, y+, z-, z+ boundary conditions;
 * dt is this level's time-step (dt_l = dt_0 / 2^l in the W-cycle of Sec. 2.1)
 * unless dt_dev is non-NULL, in which case it is *dt_dev times dt_dev_scale
 * (0 is taken as 1; a power of two keeps it exact, e.g. 2^-l with dt_dev the
 * coarse dt_0); dx is this level's cell width.
 * CFL outputs of the state the launch writes for this level (Sec. 2.6 Eq. 2,
 * reduced in the same pass as in hydro_advance_level; all optional, NULL for
 * none; c_cfl > 0 when any is given):
 *   dt_patch_next_dev  [G_l][8] per-patch time-steps (bit-identical to
 *                      hydro_dt on the output)
 *   dt_next_dev        the level's minimum times dt_next_scale (0 is taken
 *                      as 1) is folded in with an exact, order-independent
 *                      minimum; it must hold +inf or a larger value when the
 *                      launch starts.  Levels may share it: with dt_next_scale
 *                      = 2^l every level folds the coarse step its state
 *                      allows, min_l 2^l dt_l
 *   dt_reset_dev       set to +inf at the start of the launch (before any
 *                      other use in it), so that three words can rotate over
 *                      coarse steps (read dt_0 from A, reduce into B, reset
 *                      C); must differ from every level's dt_dev and
 *                      dt_next_dev */
typedef struct {
  const void* level_dev;  /* [G_l][5][16^3] input level storage */
  void* level_out_dev;    /* [G_l][5][16^3] output level storage */
  int32_t ngx, ngy, ngz;  /* group lattice of the level (limits as hydro_advance_level) */
  int32_t bc[6];
  double dt;
  double dx;
  const double* dt_dev;
  double dt_dev_scale;
  double c_cfl;
  double dt_next_scale;
  double* dt_next_dev;
  double* dt_patch_next_dev;
  double* dt_reset_dev;
} hydro_level_t;

/* hydro_advance_batched -- one MHM step of every group of n_levels levels in
 * ONE persistent launch (Sec. 2.1: levels of an AMR hierarchy advance with
 * their own dt; here their groups are pooled).  Workgroups take (level, group)
 * items from a device work counter until all are done; results are
 * bit-identical to one hydro_advance_level call per level.
 *   levels_host  n_levels (1..8) entries in host memory; no output may overlap
 *                any input or another output
 *   dtype, gamma, scheme, theta, n_bad_dev: as for hydro_advance
 *   work_dev     HYDRO_BATCH_WORK_WORDS device uint32 owned by the caller:
 *                zero before the first call; every call leaves them zero
 *                again.  Launches sharing a work_dev must not run
 *                concurrently.
 *   grid         persistent workgroups (0: two per compute unit in FP64,
 *                four in FP32, capped at the item count)
 * Launch shapes (per context and dtype, HYDRO_BATCHED_VARIANTS of them):
 * bit 0 item order (0: level 0 first, 1: finest level first), bit 1
 * occupancy target, bits 2-3 work distribution (0: one queue; 1: one queue
 * per XCD, each serving one residue class of items mod 8, with stealing when
 * it runs dry; 2: static round-robin, workgroup b takes items b, b + grid,
 * ...; 3: one queue per XCD, each serving level by level one of 8
 * contiguous blocks of the level's groups in column-tile order (the range
 * the XCD-blocked column-tile level step gives that XCD), with stealing);
 * hydro_set_batched_variant / hydro_get_batched_variant select and read it,
 * hydro_autotune_batched times all of them on the given levels (two passes
 * of 1 untimed + `reps` timed launches per shape, a shape's time is the
 * smaller of its two means; SYNCHRONOUS; the outputs are overwritten;
 * times_ms_host receives HYDRO_BATCHED_VARIANTS floats) and records the
 * fastest in ctx (non-NULL) for these level lattices.
 */
#define HYDRO_BATCH_WORK_WORDS 16
#define HYDRO_BATCHED_VARIANTS 16
int hydro_advance_batched(hydro_ctx* ctx, const hydro_level_t* levels_host, int32_t n_levels, int32_t dtype, double gamma,
                          int32_t scheme, double theta, int32_t* n_bad_dev, uint32_t* work_dev, int32_t grid,
                          void* stream);
/* hydro_advance_batched_noalloc -- hydro_advance_batched for callers that
 * cannot allocate device memory (code under graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same launch and arguments
 * except work_dev.  The work counters live in the library's own array of
 * HYDRO_BATCH_WORK_WORDS uint32 (64 bytes) per device, held until the
 * process ends, and are cleared by a small kernel on `stream` before every
 * launch; nothing is allocated.  Limits: those of hydro_advance_batched (at
 * most 8 levels, fewer than 2^32 - 2^20 groups in all; HYDRO_EINVAL beyond).
 * Every call on one device shares that device's counters: calls that overlap
 * in time on one device (different streams, or host threads) race and must
 * not be issued. */
int hydro_advance_batched_noalloc(hydro_ctx* ctx, const hydro_level_t* levels_host, int32_t n_levels, int32_t dtype,
                                  double gamma, int32_t scheme, double theta, int32_t* n_bad_dev, int32_t grid,
                                  void* stream);
int hydro_set_batched_variant(hydro_ctx* ctx, int32_t dtype, int32_t variant);
int hydro_get_batched_variant(hydro_ctx* ctx, int32_t dtype);
int hydro_autotune_batched(hydro_ctx* ctx, const hydro_level_t* levels_host, int32_t n_levels, int32_t dtype, double gamma,
                           uint32_t* work_dev, int32_t reps, float* times_ms_host, void* stream);

/* Graph capture of a sequence of library calls (e.g. a level's substeps or
 * the stages of a coarse step), replayed without per-launch host overhead.
 *   hydro_graph_begin    start capturing `stream` (a non-NULL hipStream_t)
 *   hydro_graph_end      stop capturing, instantiate; *graph_exec receives an
 *                        opaque handle, owned by ctx (freed at the latest by
 *                        hydro_ctx_destroy) or, with ctx NULL, by the caller
 *   hydro_graph_launch   replay the captured work on `stream`
 *   hydro_graph_destroy  free a handle (with the ctx it was captured through;
 *                        HYDRO_EINVAL if that ctx does not own it)
 * Calls made between begin and end are recorded, not executed; kernel
 * arguments (pointers, dt values) are frozen at capture time, so buffers
 * must stay allocated while the graph is used.  The library records no
 * memset nodes. */
int hydro_graph_begin(void* stream);
int hydro_graph_end(hydro_ctx* ctx, void* stream, void** graph_exec);
int hydro_graph_launch(void* graph_exec, void* stream);
int hydro_graph_destroy(hydro_ctx* ctx, void* graph_exec);

/* hydro_dt -- per-patch CFL time-step, Sec. 2.6 Eq. 2 (the form for MHM):
 * dt_patch = (c_cfl * dx) / max over the patch's 8^3 cells of
 * (|u| + |v| + |w| + 3 c_s), c_s = sqrt(gamma p / rho), evaluated in double
 * precision for both dtypes (FP32 states are widened first).
 *   U_pad_dev       [G][5][P^3] (only interiors are read; ghost 0..16)
 *   dt_patch_dev    [G][8] double output; patch p = (pz*2 + py)*2 + px of a group
 *   dt_min_dev      optional device double (may be NULL): receives the minimum
 *                   over all patches (the level time-step); written, not
 *                   accumulated.
 */
int hydro_dt(const void* U_pad_dev, int64_t n_groups, int32_t ghost, int32_t dtype, double dx,
             double gamma, double c_cfl, double* dt_patch_dev, double* dt_min_dev, void* stream);

/* hydro_fill_ghosts -- build padded groups from level storage (Sec. 3.4: ghost
 * zones exist only for the groups being solved; Sec. 2.2 boundary conditions).
 * Every padded cell copies the level cell whose index along each axis is the
 * padded index mapped independently per axis: inside the domain unchanged,
 * beyond a periodic face wrapped, beyond an outflow face clamped to the
 * nearest interior cell.
 *   level_dev   [G][5][16^3], G = ngx*ngy*ngz
 *   U_pad_dev   [G][5][P^3] output, must not overlap level_dev
 *   ghost       0..16
 *   bc_host     6 ints on the host: x-, x+, y-, y+, z-, z+ faces
 */
int hydro_fill_ghosts(const void* level_dev, void* U_pad_dev, int32_t ngx, int32_t ngy, int32_t ngz,
                      int32_t ghost, int32_t dtype, const int32_t* bc_host, void* stream);

/* hydro_gather_ghost_adjoint -- the adjoint (transpose) of hydro_fill_ghosts:
 * every level cell receives the sum of the padded cotangents at all padded
 * positions that copy it (its own interior position and each ghost position
 * the fill maps to it), summed in a fixed order (deterministic).  With
 * hydro_advance_adjoint it gives the cotangent of the level state of a step
 * taken as hydro_fill_ghosts + hydro_advance (the reverse of Sec. 3.4's ghost
 * preparation; the adjoint itself is not in the paper).
 *   g_pad_dev    [G][5][P^3] padded cotangents, G = ngx*ngy*ngz (not modified)
 *   g_level_dev  [G][5][16^3] output (overwritten), must not overlap g_pad_dev
 *   ghost        0..16, as given to hydro_fill_ghosts
 *   bc_host      6 ints on the host, as given to hydro_fill_ghosts
 */
int hydro_gather_ghost_adjoint(const void* g_pad_dev, void* g_level_dev, int32_t ngx, int32_t ngy, int32_t ngz,
                               int32_t ghost, int32_t dtype, const int32_t* bc_host, void* stream);

/* Launch shapes of hydro_advance_level.  Every shape runs the same per-cell
 * arithmetic in the same order, so all give bit-identical results; they
 * differ in the register budget the compiler was given (occupancy, bit 1),
 * in the order groups are dealt to workgroups (bit 0: plain, or blocked so
 * that each of the 8 XCDs sweeps a contiguous range of groups and finds
 * neighbour-group halos in its own L2; bit 2: linear, or column-tile order --
 * tiles of about 64 groups' rows, each visited layer by layer upward in z,
 * so that a group's ghost planes in z are still cached from the group below
 * it), in the LDS layout of the plane tiles (bit 3: packed rows,
 * or rows padded by one element) and in the threads per workgroup (bit 4:
 * 256, one group per workgroup, or 512, two groups marched side by side
 * with their own LDS and shared barriers).  The choice is per context, per dtype and per kernel form
 * (with_cfl: the form that reduces the next CFL time-step, which needs more
 * registers and 4 KB more LDS per workgroup).  Setters need a context;
 * getters with ctx NULL return the default (6: XCD-blocked, column-tile,
 * low occupancy target).
 *   hydro_num_variants       number of shapes (>= 1)
 *   hydro_set_level_variant  select one (0 .. n-1) for one form; HYDRO_EINVAL otherwise
 *   hydro_get_level_variant  current selection for a dtype and form
 *   hydro_set_variant        select one for both forms
 *   hydro_get_variant        current selection of the CFL form
 *   hydro_variant_name       short description into buf[len] (host memory)
 */
int hydro_num_variants(void);
int hydro_set_level_variant(hydro_ctx* ctx, int32_t dtype, int32_t with_cfl, int32_t variant);
int hydro_get_level_variant(hydro_ctx* ctx, int32_t dtype, int32_t with_cfl);
int hydro_set_variant(hydro_ctx* ctx, int32_t dtype, int32_t variant);
int hydro_get_variant(hydro_ctx* ctx, int32_t dtype);
int hydro_variant_name(int32_t variant, char* buf, int32_t len);

/* hydro_autotune -- time every launch shape of hydro_advance_level on the
 * caller's level (two passes of 1 untimed + `reps` timed launches per shape,
 * HIP events on `stream`, 1 <= reps <= 1000; a shape's time is the smaller of
 * its two means), record the fastest in ctx (non-NULL) for `dtype` and this
 * lattice and return its index (>= 0), or a negative status (nothing is
 * recorded).  Shapes within 1.5% of the fastest count as ties, resolved
 * towards fewer HBM bytes per step: XCD-blocked before plain order,
 * column-tile before linear, low before high occupancy target, then the
 * lowest number (the timing relaunches one cached input, where a group
 * order's extra HBM reads hardly show).  Both kernel forms are timed and
 * tuned separately (without and
 * with the CFL epilogue; the returned index is the CFL form's).  SYNCHRONOUS:
 * waits on `stream`; allocates nothing on the device.  level_dev is read,
 * scratch_out_dev ([G][5][16^3]) is overwritten, cfl_scratch_dev receives the
 * CFL form's outputs: at least (3 + 8 G) doubles (cfl_scratch_bytes); no two
 * of the three may overlap.  times_ms_host, if not NULL, receives
 * 2 * hydro_num_variants() times in milliseconds (the form without CFL first).
 */
int hydro_autotune(hydro_ctx* ctx, const void* level_dev, void* scratch_out_dev, int32_t ngx, int32_t ngy,
                   int32_t ngz, const int32_t* bc_host, int32_t dtype, double dx, double gamma,
                   double* cfl_scratch_dev, int64_t cfl_scratch_bytes, int32_t reps, float* times_ms_host,
                   void* stream);

/* Name of a status code (static string). */
const char* hydro_strerror(int status);

/* hipError_t of the last failed HIP call made by the library on this thread. */
int hydro_last_hip_error(void);

/* Library ABI version (increases when an entry point changes). */
int hydro_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HYDRO_H_ */
