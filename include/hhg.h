/*
 * hhg.h -- C ABI of the MI355X Uzawa-multigrid Stokes solver.
 *
 * Method: all-at-once Uzawa multigrid (UMG) for the P1-P1 PSPG-stabilised
 * Stokes system in Laplace form on hierarchical hybrid grids (Gmeiner, Huber,
 * John, Ruede, Wohlmuth, arXiv:1511.02134): Section 2.1 (discretisation,
 * eq. linear-system), Section 3.3 (inexact Uzawa smoother, eq. Uzawa_smooth),
 * Section 3.5 (smoothers, V-cycle), Section 3.6 (stopping criterion) and
 * Section 3.7 (coarse-grid PMINRES).
 *
 * Conventions shared by every call
 * --------------------------------
 *  * Status: every call returns an hhg_status; nothing throws across the ABI.
 *    Arguments and meshes are validated on the host before any launch; a
 *    failed validation returns HHG_EINVAL and launches nothing.  The message
 *    of the last failure is returned by hhg_last_error (per context) or
 *    hhg_global_error (calls that have no context yet).
 *  * Memory: the caller owns all device memory.  hhg_plan reports the size of
 *    one device workspace; hhg_create carves every table and work vector out
 *    of it.  The library never allocates device memory.
 *  * Streams: `stream` is a hipStream_t (NULL = the default stream).  Every
 *    call only enqueues work on that stream unless it says it synchronises.
 *  * Levels: level l = 0..L holds the mesh refined R_l = l + 2 times (level 0
 *    is the paper's coarse grid T_0, the twice refined macro mesh); L = R - 2.
 *  * Vectors: a "vector" of level l is an array of 4 fields (u_x, u_y, u_z, p)
 *    of hhg_vec_len(ctx, l) values each, field-major, in the library's
 *    per-macro layout: every macro tetrahedron stores the full closure of its
 *    refined vertices (tetrahedral slab/row order, each row split into four
 *    sub-rows by i mod 4), so vertices on macro faces, edges and corners
 *    exist once per macro that contains them.  All calls keep those copies
 *    identical (the ghost exchange).  Vectors are double precision unless
 *    stated otherwise.  hhg_scatter / hhg_gather convert to and from nodal
 *    arrays in lattice order.
 *  * Nodal (lattice) order: node (X, Y, Z) of the level-l lattice, integer
 *    coordinates in units of 2^-R_l, has index X + nx*(Y + ny*Z) where
 *    nx, ny, nz are the lattice extents of the bounding box of the mesh.
 *    Lattice points that lie in no macro (a hole of the mesh) are not
 *    vertices: scatter ignores their values and gather writes 0 there.
 *  * Dirichlet data live in the Dirichlet velocity entries of the solution
 *    vector x and are never modified; the residual and K x vanish on those
 *    rows.  Pressure is an unknown at every vertex.
 */
#ifndef HHG_H
#define HHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hhg_ctx hhg_ctx;
typedef void* hhg_stream; /* hipStream_t */

/* Entries of the per-level arrays of hhg_solve_info; a hierarchy has at most
 * 9 levels, since n_refine <= 10. */
#define HHG_MAX_LEVELS 16

typedef enum {
    HHG_OK = 0,
    HHG_EINVAL = 1,   /* bad argument or malformed mesh; nothing was launched */
    HHG_ENOMEM = 2,   /* workspace too small */
    HHG_EDEVICE = 3,  /* a HIP runtime call failed */
    HHG_ENOCONV = 4,  /* solve stopped before the tolerance (info is filled) */
    HHG_ENAN = 5      /* NaN or Inf in a residual norm */
} hhg_status;

/* Macro mesh T_{-2} (Section 2.1).  All arrays are host memory, read during
 * the call only.  Requirements checked by hhg_plan / hhg_create:
 *   xyz [nv][3]   vertex coordinates on the integer lattice (the topology:
 *                 refinement, node numbering and colouring follow it);
 *   tet [nt][4]   vertex ids in Kuhn path order: tet[1]-tet[0], tet[2]-tet[1],
 *                 tet[3]-tet[2] are the three distinct positive unit vectors;
 *                 the tetrahedra are conforming (a face is shared by at most
 *                 two) and lie in the bounding box of xyz, which they tile
 *                 unless `phys` is given (then lattice points of the box may
 *                 lie in no macro: a hole, such as the inside of a shell);
 *   nu  [nt]      per-macro viscosity > 0 (NULL: all 1);
 *   face_bc [nt][4] tag of the face opposite vertex f: 0 interior (shared by
 *                 two macros), 1 Dirichlet velocity, 2 natural (do-nothing),
 *                 3 free-slip (Section 6.1): u . n = 0 at the face's vertices
 *                 (those on a Dirichlet face excepted) with the
 *                 mass-conservative normal n_i = <grad phi_i, 1> / |.|, zero
 *                 tangential stress.  The velocity rows of K x, the residual
 *                 and the right-hand side of such a vertex are projected onto
 *                 its tangent plane, and so are its smoothed values and
 *                 transferred corrections; hhg_solve projects x first.  Needs
 *                 the Laplace form, the colour ordering, the direct coarse
 *                 solver and krylov = 0; hhg_grad and hhg_adjoint_rhs reject
 *                 such meshes;
 *   phys [nv][3]  physical coordinates of the vertices (NULL: xyz; the
 *                 field was appended to the struct, callers must set it).  Every
 *                 macro carries its refinement affinely (Section 2.1: uniform
 *                 refinement splits a tetrahedron into 8 by its edge
 *                 midpoints), so its stencils are those of its own affine
 *                 image: general 15-point stencils for a_1 and c_l.  Each
 *                 macro must keep its orientation (positive volume when its
 *                 lattice image has one). */
typedef struct {
    int32_t nv;
    const double* xyz;
    int32_t nt;
    const int32_t* tet;
    const double* nu;
    const int8_t* face_bc;
    const double* phys;
} hhg_mesh;

/* Solver options (Section 3.5 and Table "settings", UMG column). */
typedef struct {
    int32_t nu1, nu2;     /* pre / post smoothing steps: V(nu1, nu2); default 3, 3 */
    int32_t cycle;        /* 0: V-cycle; 1: variable V-cycle (+2 steps per coarser level) */
    int32_t p_sweep;      /* 0: forward pressure sweep (paper); 1: forward + backward */
    double omega;         /* pressure under-relaxation; default 0.3 */
    int32_t precision;    /* 0: FP64 throughout; 1: FP32 cycles inside FP64 refinement */
    double coarse_rtol;   /* coarse PMINRES relative tolerance; default 1e-14 */
    int32_t coarse_maxit; /* coarse PMINRES iteration cap; default 500 */
    int32_t block_order;  /* workgroup -> tile order: 0 natural, 1 XCD-aware (default),
                             2 reversed (a schedule permutation used to test that
                             results do not depend on workgroup order) */
    int32_t coarse_prec;  /* pressure block of the coarse MINRES preconditioner:
                             0 exact Schur complement B A^-1 B^T + C (dense;
                             fewer iterations, each dearer), 1 lumped mass
                             weighted by 1/nu (the paper's choice, default) */
    int32_t coarse_solver; /* 0: exact, x0 = Z b0 with Z the inverse of the level-0
                              system bordered by the mass-weighted mean constraint
                              (formed on the device by hhg_create and
                              hhg_set_viscosity, Gauss-Jordan elimination; one
                              matrix-vector product per solve; default);
                              1: the block-diagonal preconditioned MINRES above.
                              Either way at most 16384 level-0 unknowns */
    int32_t krylov;       /* 1: reserve the ten finest-level vectors (4 fields each) of
                             hhg_pminres and hhg_scg; 0 (default): those calls return
                             HHG_EINVAL */
    int32_t graphs;       /* 1: hhg_solve captures the launches of one cycle and its
                             stopping test in a HIP graph on first use for an (x, b) pair
                             and replays it (at most four pairs kept; the capture records
                             launches without running them); 0 (default): plain launches
                             on the stream.  Results are bitwise identical either way */
    int32_t op;           /* velocity form (Section 2.1, eq. varform): 0 the Laplace form
                             a_1 = <nu grad u, grad v> (default); 1 the D form
                             a_2 = 2 <nu D(u), D(v)>, whose velocity block couples the
                             components: the velocity sweeps become point-block Gauss-Seidel
                             (3x3 centre block solved exactly, same colours and order), also
                             in the velocity multigrid of hhg_vel_cycle, hhg_pminres and
                             hhg_scg, and the viscosity gradient of hhg_grad takes the
                             coupled form.  The D form needs coarse_solver = 0 */
    int32_t ordering;     /* Gauss-Seidel order of the Uzawa smoother (Section 3.4):
                             0 (default) the global 4-colouring, colour (X+Y+Z) mod 4;
                             1 the hybrid order of HHG: primitive classes in the order
                             macro vertices, edges, faces, volumes; primitives of one
                             class decoupled (block Jacobi: a vertex reads the vertices
                             of other primitives of its class as they were when the
                             class started); inside a primitive the colours 0..3
                             (backward sweep 3..0, class order kept).  Laplace form,
                             without the Krylov vectors;
                             2 red-black: the parities of X+Y+Z (red: colours 0 and 2,
                             black: 1 and 3), one launch per parity.  Valid where a_1
                             and c_l couple only the six axis neighbours, whose
                             colours differ by one: meshes given without phys (with
                             phys every macro takes general 15-point stencils, and
                             the ordering is rejected).  Velocity sweep red, black, red (a second
                             black update in a row would change nothing); pressure
                             sweep red, black, then black, red when p_sweep = 1.
                             Laplace form, without the Krylov vectors */
} hhg_opts;

/* Result of hhg_solve. */
typedef struct {
    int32_t cycles;        /* cycles performed */
    int32_t status;        /* hhg_status of the solve */
    double r0;             /* ||f~ - K x_0||_2 (Section 3.6) */
    double r_final;        /* ||f~ - K x_k||_2 after the last cycle */
    double rel_res;        /* r_final / r0 */
    double rho_mean;       /* (r_final / r0)^(1/cycles) */
    double rho_max;        /* largest ||r_k|| / ||r_{k-1}|| */
    double t_solve_ms;     /* wall time of the cycles, hipEvent timed on the stream */
    double res_hist[256];  /* ||r_k||_2, k = 0..min(cycles, 255) */
    double n_op[4];        /* operator evaluations of A, B, C and M during the call,
                              weighted by level, sum_l 8^(l-L) n_op,l (Section 4.2,
                              eq. op_count); a colour sweep counts a quarter of its
                              operator, B and B^T count as B, the exact level-0
                              solves count nothing; the first Uzawa step of a level
                              in a cycle counts no B when f - B^T p is given (b on
                              levels whose iterate starts at 0; in the FP64 solve
                              on Kuhn macros in the Laplace form, the stopping
                              test's residual leaves it for the top level) */
    /* Phase times of hhg_solve in ms, summed over all cycles and levels, from
     * hipEvent pairs on the stream; 0 unless hhg_set_phase_timing(ctx, 1)
     * (the events cost a few microseconds each and disable graph replay):
     *   smooth    Uzawa smoothing steps on levels 1..L;
     *   transfer  restriction, zeroing of the coarse iterate, prolongation;
     *   coarse    the level-0 solve (with its residual and correction);
     *   residual  the residual before each restriction and the stopping test.
     * t_solve_ms minus their sum is the rest (projection, mixed-precision
     * scaling, event gaps). */
    double t_smooth_ms, t_transfer_ms, t_coarse_ms, t_residual_ms;
    /* The same event pairs by level (entries 0..L; the rest 0): level l's
     * smoothing, its residual, the restriction from it and the prolongation
     * into it, the zeroing of its iterate; level 0 the coarse solves.  They sum
     * to the four phase times. */
    double t_level_ms[HHG_MAX_LEVELS];
} hhg_solve_info;

/* Fills opts with the defaults above. */
void hhg_default_opts(hhg_opts* opts);

/* Validates the mesh and options and reports the device workspace size in
 * bytes for n_refine refinements (2 <= n_refine <= 10).  Host only. */
hhg_status hhg_plan(const hhg_mesh* mesh, int32_t n_refine, const hhg_opts* opts,
                    size_t* workspace_bytes);

/* Builds the hierarchy (levels 2..n_refine), stencils (one 15-point stencil
 * per macro and per interface primitive and level, from the P1 element
 * matrices of a_1, b, c_l and g_l, Section 2.1) and index tables, and uploads
 * them into d_workspace (device memory of at least hhg_plan's size,
 * 256-byte aligned).  Synchronises the device.  With d_workspace == NULL a
 * host-only context is built for inspection (hhg_node_info, counts); every
 * device call on it returns HHG_EINVAL. */
hhg_status hhg_create(const hhg_mesh* mesh, int32_t n_refine, const hhg_opts* opts,
                      void* d_workspace, size_t workspace_bytes, hhg_ctx** ctx);
void hhg_destroy(hhg_ctx* ctx);
const char* hhg_last_error(const hhg_ctx* ctx);
const char* hhg_global_error(void);

/* Sizes and geometry (host only). */
int32_t hhg_num_levels(const hhg_ctx* ctx);               /* L + 1 */
int64_t hhg_vec_len(const hhg_ctx* ctx, int32_t level);   /* values per field */
int64_t hhg_num_nodes(const hhg_ctx* ctx, int32_t level); /* lattice nodes */
int64_t hhg_num_dofs(const hhg_ctx* ctx, int32_t level);  /* 3*free velocity nodes + nodes
                                                             (vertices only, no hole points) */
int64_t hhg_num_interface(const hhg_ctx* ctx, int32_t level); /* vertices on macro faces */
/* Integer lattice coordinates [N][3] and velocity boundary flags [N] (either
 * may be NULL) of the level's lattice points in lattice order, into host
 * arrays (N = hhg_num_nodes): 1 Dirichlet, 2 free-slip, 0 otherwise (also at
 * the lattice points of a hole). */
hhg_status hhg_node_info(const hhg_ctx* ctx, int32_t level, int32_t* ijk, int8_t* dirichlet);

/* HHG primitive class (Section 3.4) of every lattice point of the level into
 * a host array [N] (lattice order): 0 on a macro vertex, 1 inside a macro
 * edge, 2 inside a macro face, 3 inside a macro, -1 at a point of a hole.
 * The hybrid ordering (opts.ordering = 1) sweeps the classes in this order. */
hhg_status hhg_primitive_classes(const hhg_ctx* ctx, int32_t level, int8_t* cls);

/* Lumped mass m_i = int phi_i of every node (lattice order) into a host
 * array [N]: the weights of the mean-zero pressure projection (0 at the
 * lattice points of a hole, which are not vertices). */
hhg_status hhg_mass_weights(const hhg_ctx* ctx, int32_t level, double* m);

/* Host-only self-check of the index tables: runs the kernels' index
 * arithmetic (tile decoding, row addressing, neighbour tables, transfer
 * addressing) on the CPU over every level and verifies that each access stays
 * inside the arrays and reaches the intended lattice vertex, that every
 * vertex is visited exactly once per sweep and that colour sweeps only touch
 * their colour.  Returns HHG_EINVAL with a message on the first violation. */
hhg_status hhg_check_layout(const hhg_ctx* ctx);

/* Layout conversion.  d_nodal: nfields arrays of N doubles (lattice order);
 * d_x: nfields arrays of hhg_vec_len doubles.  Scatter writes every copy of
 * every vertex; gather reads each vertex once.  1 <= nfields <= 4. */
hhg_status hhg_scatter(hhg_ctx* ctx, int32_t level, const double* d_nodal, int32_t nfields,
                       void* d_x, hhg_stream stream);
hhg_status hhg_gather(hhg_ctx* ctx, int32_t level, const void* d_x, int32_t nfields,
                      double* d_nodal, hhg_stream stream);
/* Ghost exchange (Section 3.4, Figure "ghost layer structure"): copies the
 * primary value of every interface vertex into all its other macro copies. */
hhg_status hhg_exchange(hhg_ctx* ctx, int32_t level, void* d_x, int32_t nfields,
                        hhg_stream stream);

/* Right-hand side of eq. (linear-system) on the finest level from the nodal
 * P1 interpolant of the forcing: d_rhs = (M f on free velocity rows,
 * g_l(I_h f) on pressure rows).  d_f: 3 fields in the internal layout. */
hhg_status hhg_rhs(hhg_ctx* ctx, const void* d_f, void* d_rhs, hhg_stream stream);
/* The same on level l (0..L), from the forcing interpolated at that level's
 * vertices (3 fields, internal layout of level l); the right-hand sides of
 * full multigrid. */
hhg_status hhg_rhs_level(hhg_ctx* ctx, int32_t level, const void* d_f, void* d_rhs,
                         hhg_stream stream);

/* y = K x (eq. linear-system) on level l: rows of free velocity nodes and all
 * pressure rows; Dirichlet velocity rows of y are 0.  x must not alias y. */
hhg_status hhg_apply(hhg_ctx* ctx, int32_t level, const void* d_x, void* d_y,
                     hhg_stream stream);
/* r = b - K x on level l.  If h_norm is not NULL the call synchronises the
 * stream and stores ||r||_2 (free velocity rows and all pressure rows). */
hhg_status hhg_residual(hhg_ctx* ctx, int32_t level, const void* d_x, const void* d_b,
                        void* d_r, double* h_norm, hhg_stream stream);
/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the residual of
 * hhg_residual, r = b - K x on level l, with ||r||_2 (free velocity rows and
 * all pressure rows) written to the device scalar *d_norm instead of host
 * memory.  It allocates nothing, records no event and never synchronises:
 * its per-block partial sums live in a static device array of the library
 * (8 MiB, 2^20 doubles, one per GPU, held until the process ends); levels
 * needing more partial sums than that (beyond about 9 refinements of the
 * unit cube) return HHG_EINVAL.  Every call on one GPU shares that array, so
 * calls that overlap in time on one GPU (on different streams or host
 * threads) race; calls ordered on one stream do not.  The context's device
 * must be the current device (HHG_EINVAL otherwise); r must not alias x or
 * b.  Results equal hhg_residual's bit for bit. */
hhg_status hhg_residual_noalloc(hhg_ctx* ctx, int32_t level, const void* d_x, const void* d_b,
                                void* d_r, double* d_norm, hhg_stream stream);

/* `steps` inexact Uzawa smoothing steps (eq. Uzawa_smooth) in place on x:
 * symmetric 4-colour Gauss-Seidel on the velocity, then the pressure sweep
 * on C with relaxation omega.  Colour of vertex (X,Y,Z) = (X+Y+Z) mod 4. */
hhg_status hhg_smooth(hhg_ctx* ctx, int32_t level, void* d_x, const void* d_b, int32_t steps,
                      hhg_stream stream);
/* Restriction of a level-l residual to the right-hand side of level l-1
 * (transpose of P1 interpolation, velocity Dirichlet rows zeroed), and
 * interpolation of a level-(l-1) correction added to a level-l vector. */
hhg_status hhg_restrict(hhg_ctx* ctx, int32_t level, const void* d_r_fine, void* d_b_coarse,
                        hhg_stream stream);
hhg_status hhg_prolong_add(hhg_ctx* ctx, int32_t level, const void* d_e_coarse,
                           void* d_x_fine, hhg_stream stream);
/* Level-0 solve (Section 3.7), x0 = K_0^-1 b0 with the pressure of zero mean
 * when it has a null space (b0 is first made consistent by removing its
 * component along the constant pressure, the Lagrange multiplier of the mean
 * constraint).  opts.coarse_solver 0: one product with the precomputed
 * inverse of the bordered system (exact up to rounding; iters = 1,
 * relres = 0).  1: block-diagonal preconditioned MINRES on the whole coarse
 * Stokes system, preconditioner diag(A_0^-1, S_0^-1) with S_0 the exact Schur
 * complement or the lumped 1/nu-weighted mass (opts.coarse_prec), run to
 * opts.coarse_rtol, then projected to zero mean.  iters / relres (host, may
 * be NULL) synchronise the stream. */
hhg_status hhg_coarse_solve(hhg_ctx* ctx, const void* d_b0, void* d_x0, int32_t* iters,
                            double* relres, hhg_stream stream);
/* Pressure projection to zero mean, p -= (sum m_i p_i)/(sum m_i) with
 * m_i = int phi_i; no-op when a natural boundary removes the null space. */
hhg_status hhg_project(hhg_ctx* ctx, int32_t level, void* d_x, hhg_stream stream);

/* One solver iteration on the finest level: a V(nu1,nu2) (or variable) cycle
 * followed by the mean-zero projection.  In mixed precision the cycle runs
 * in FP32 on the FP64 residual scaled by its norm (iterative refinement). */
hhg_status hhg_vcycle(hhg_ctx* ctx, void* d_x, const void* d_b, hhg_stream stream);
/* Full multigrid (Section 5, Figure "FMG"): d_x[l], d_b[l] (host arrays of
 * L+1 device pointers, internal layout of level l) hold on input the
 * Dirichlet values of level l in x's boundary velocity slots and the level's
 * right-hand side.  Level 0 is solved exactly (from those Dirichlet values);
 * then, for l = 1..L, x_l = P x_(l-1) on every slot but the Dirichlet
 * velocity ones, followed by `cycles` V-cycles whose top level is l (in the
 * variable cycle, level k below the top smooths 2 (l - k) more steps), each
 * followed by the mean-zero projection.  Every other slot of the d_x[l] is
 * overwritten; x_L is the result.  FP64 only (opts.precision 0): HHG_EINVAL
 * otherwise, and for cycles outside 1..16 or aliasing pointers. */
hhg_status hhg_fmg(hhg_ctx* ctx, void* const* d_x, const void* const* d_b, int32_t cycles,
                   hhg_stream stream);
/* Cycles from x until ||b - K x||_2 <= rtol ||b - K x_0||_2 (Section 3.6) or
 * max_cycles (<= 255).  Synchronises once per cycle (an 8-byte readback).
 * Returns HHG_ENOCONV if the tolerance was not met, HHG_ENAN on a non-finite
 * norm; info (may be NULL) is filled in every case. */
hhg_status hhg_solve(hhg_ctx* ctx, void* d_x, const void* d_b, double rtol, int32_t max_cycles,
                     hhg_solve_info* info, hhg_stream stream);

/* One multigrid cycle for the velocity block alone, A u_k = b_k (k = 0..2),
 * on the finest level (Sections 3.1, 3.2; Table "settings", SCG and PMINRES
 * columns): V(nu1, nu2) with forward colour Gauss-Seidel (colours 0,1,2,3) in
 * the pre-smoothing and backward (3,2,1,0) in the post-smoothing steps, the
 * A-residual restricted by the transpose of P1 interpolation, A_0 inverted
 * exactly on level 0 (the D form: point-block sweeps, the coupled A_2
 * residual and level-0 block).  Fields 0..2 of d_x are updated in place (their
 * Dirichlet entries are kept), field 3 is not touched; d_b fields 0..2 are
 * read (their Dirichlet rows are ignored).  0 <= nu1, nu2 <= 64, nu1 + nu2 > 0;
 * EINVAL on aliasing.  FP64. */
hhg_status hhg_vel_cycle(hhg_ctx* ctx, int32_t nu1, int32_t nu2, void* d_x, const void* d_b,
                         hhg_stream stream);

/* Block-diagonal preconditioned MINRES on K x = b (Section 3.2, eq.
 * precond_block_diag): Ahat^-1 one velocity V(nu, nu) cycle as in
 * hhg_vel_cycle (nu = 1 in Table "settings"), Shat^-1 the inverse of the
 * lumped pressure mass weighted by 1/nu_T (sum over the tetrahedra around a
 * vertex of |T| / (4 nu_T)).  x carries the Dirichlet velocity values.  The
 * Euclidean residual norm of the stopping test (Section 3.6) is carried by
 * its recurrence; iterations stop when it falls to rtol ||b - K x_0||_2, or
 * after maxit iterations (rtol = 0: exactly maxit).  The pressure is
 * projected to zero mean at the end when it is only defined up to a
 * constant.  info->cycles counts iterations, res_hist the residual after
 * each.  Needs krylov = 1 at creation; FP64; synchronises once per iteration.
 * HHG_ENOCONV if the tolerance was not met (x holds the last iterate). */
hhg_status hhg_pminres(hhg_ctx* ctx, void* d_x, const void* d_b, double rtol, int32_t maxit,
                       int32_t nu, hhg_solve_info* info, hhg_stream stream);

/* Schur-complement CG (Section 3.1, Algorithm 1).  Every outer iteration runs
 * n_A velocity V(nu, nu) cycles for A u = f - B^T p from the current u, then
 * n_S steps of CG on S p = B A^-1 f - g, S = B A^-1 B^T + C, preconditioned
 * by the weighted lumped mass of hhg_pminres, from the current p with the
 * residual B u - C p - g; inside CG every A^-1 is n_I cycles from zero.  The
 * pressure is projected to zero mean (when needed) and the stopping test
 * ||b - K x||_2 <= rtol ||b - K x_0||_2 evaluated after every outer
 * iteration (rtol = 0: exactly max_outer <= 255 of them).  Table "settings":
 * n_A = n_S = 3, n_I = 1, nu = 3.  Needs krylov = 1; FP64; synchronises once
 * per outer iteration. */
hhg_status hhg_scg(hhg_ctx* ctx, void* d_x, const void* d_b, double rtol, int32_t max_outer,
                   int32_t n_A, int32_t n_S, int32_t n_I, int32_t nu, hhg_solve_info* info,
                   hhg_stream stream);

/* Adjoint gradients of J = 1/2 ||u - u_obs||^2 (not in the paper): given the
 * forward solution x (with its Dirichlet values), the adjoint solution lambda
 * of K lambda = (u - u_obs, 0) and the forcing f (3 fields, internal layout;
 * NULL means f = 0), writes dJ/dnu_e for every macro into d_dJ_dnu [nt] and
 * dJ/df (3 fields, internal layout) into d_dJ_df (may be NULL). */
hhg_status hhg_grad(hhg_ctx* ctx, const void* d_x, const void* d_lambda, const void* d_f,
                    double* d_dJ_dnu, void* d_dJ_df, hhg_stream stream);

/* Right-hand side of the adjoint system of J (not in the paper; K is
 * symmetric, eq. linear-system): d_rhs = (dJ/du with its velocity Dirichlet
 * rows zeroed, Pi^T dJ/dp) on the finest level, where Pi p = p - m (m.p) /
 * sum(m) is the mean-zero pressure projection (Section 2.1, L^2_0; m_i =
 * int phi_i) and Pi^T q = q - m (sum_i q_i) / sum(m) its transpose.  When a
 * natural boundary removes the pressure null space, Pi is the identity.
 * d_g: 4 fields (dJ/du_x, dJ/du_y, dJ/du_z, dJ/dp) in the internal layout of
 * the finest level (every copy of a vertex equal, as hhg_scatter writes
 * them); d_rhs: 4 fields, every slot written.  EINVAL if they alias. */
hhg_status hhg_adjoint_rhs(hhg_ctx* ctx, const void* d_g, void* d_rhs, hhg_stream stream);

/* Replaces the per-macro viscosity (host array [nt], > 0) and rebuilds every
 * viscosity-dependent table (stencils, level-0 system, the pressure
 * preconditioner of hhg_pminres and hhg_scg).  Synchronises the device
 * before and after the upload, so work queued on any stream finishes with
 * the old tables. */
hhg_status hhg_set_viscosity(hhg_ctx* ctx, const double* nu);

/* Per-kernel-class timing.  When enabled, the launches of the classes below
 * on the finest level are bracketed by hipEvents on their stream: the
 * velocity colour sweeps of one smoothing step, which run back to back, by
 * one pair around all of them; every other launch by a pair of its own.
 * hhg_kernel_time synchronises and returns the number of timed launches,
 * their summed duration in ms and the algorithmic bytes they moved. */
enum {
    HHG_K_VEL = 0,     /* velocity colour sweep, finest level */
    HHG_K_PRES = 1,    /* pressure colour sweep, finest level */
    HHG_K_APPLY = 2,   /* B^T p / B u / residual passes, finest level (the
                          fused f - B^T p pass excepted) */
    HHG_K_RU = 3,      /* f - B^T p with its fused colour-0 or red velocity
                          update, finest level */
    HHG_K_NCLASS = 4
};
hhg_status hhg_set_timing(hhg_ctx* ctx, int32_t on);
/* Phase timers of hhg_solve (the t_*_ms fields of hhg_solve_info): on = 1
 * brackets every phase of every cycle by a hipEvent pair, on = 0 (default)
 * records nothing.  Host only. */
hhg_status hhg_set_phase_timing(hhg_ctx* ctx, int32_t on);
hhg_status hhg_kernel_time(hhg_ctx* ctx, int32_t kclass, int64_t* launches, double* ms,
                           double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* HHG_H */
