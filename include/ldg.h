/* ldg.h -- C ABI of the MI355X (gfx950) matrix-free LDG residual / Jacobian-vector
 * product library and its Newton-GMRES solvers.
 *
 * The operator is the local discontinuous Galerkin discretization of the
 * parametrized first-order system of Section 2.1 (Eq. 1a: q + grad u = 0;
 * Eq. 1b: m du/dt + div f(u,q) = s with m = 1), discretized as Section 2.2
 * states (LDG in space with user numerical traces/fluxes; implicit time
 * stepping), and solved by the matrix-free Newton-GMRES method of Section 3.3
 * (Jacobian-vector products by automatic differentiation or finite differences,
 * tensor-product sum factorization for the residual).
 *
 * Conventions shared by every call:
 *  - Meshes are quadrilaterals (nd = 2) or hexahedra (nd = 3) with multilinear
 *    maps; corners are numbered lexicographically (bit k of the corner index set
 *    <=> upper side in reference direction k).  Two elements that share a face
 *    must see it as opposite sides of the same reference direction with the same
 *    tangential orientation (structured-like topology); other meshes are rejected
 *    with LDG_EUNSUPPORTED.
 *  - The basis is the Lagrange basis on the (p+1)^nd tensor Gauss-Legendre nodes;
 *    volume and face integrals use nq1d Gauss-Legendre points per direction.
 *    nq1d = p+1 (collocated) is the general path; nq1d > p+1 is accepted only for
 *    the Poisson model with constant kappa on affine meshes, where the collocated
 *    rule integrates every solution-dependent term exactly and the data terms
 *    (source, boundary data) are integrated with the nq1d rule.
 *  - Degrees of freedom are element-major, then variable, then node with the
 *    first reference direction fastest: u[E][ncu][(p+1)^nd].  q = -grad u (Eq. 1a)
 *    is stored as q[E][ncu][nd][(p+1)^nd].
 *  - Boundary faces are numbered element-major, local-face-minor; local faces
 *    are (-xi, +xi, -eta, +eta, -zeta, +zeta).  Face points are the tensor
 *    Gauss-Legendre points of the two tangential directions, lower direction
 *    fastest.
 *  - Vector arguments are HIP device pointers owned by the caller, unless marked
 *    HOST.  Work is enqueued on the caller's stream (NULL = default stream); the
 *    operator calls never synchronize; the solvers synchronize on scalars to test
 *    convergence.  Handles are created/destroyed by the library and are not
 *    thread-safe.
 *  - Every call returns an ldg_status; on error, ldg_last_error() returns a
 *    thread-local message and outputs are unspecified, except that the solvers
 *    leave their last iterate in x / u and fill their stats.
 */
#ifndef LDG_H
#define LDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LDG_OK = 0,
  LDG_EINVAL = 1,        /* bad argument (null pointer, size, inconsistent model) */
  LDG_EUNSUPPORTED = 2,  /* valid but not implemented combination                 */
  LDG_EDEVICE = 3,       /* HIP runtime error                                     */
  LDG_ENOMEM = 4,        /* device allocation failed                              */
  LDG_ENOCONV = 5,       /* solver stopped without reaching its tolerance         */
  LDG_EBREAKDOWN = 6     /* non-finite value met inside a solver                  */
} ldg_status;

/* Precision of the Jacobian-vector product / operator evaluation.  Inputs and
 * outputs stay FP64; the mode sets the arithmetic and the storage of the
 * intermediates (q, face values). */
typedef enum {
  LDG_FP64 = 0,
  LDG_FP32 = 1,
  LDG_BF16_MFMA = 2,   /* derivative/test contractions on MFMA, bf16 operands, fp32 accumulation */
  LDG_FP16_MFMA = 3,   /* same with fp16 operands                                              */
  LDG_JVP_FD = 4,      /* finite-difference JVP: (R(u + eps v) - R(u)) / eps in FP64             */
  LDG_BF16 = 5,        /* storage only (block-Jacobi factors): bf16 codes, FP64 arithmetic       */
  LDG_FP16 = 6         /* storage only (block-Jacobi factors): fp16 codes, FP64 arithmetic       */
} ldg_precision;

/* Built-in PDE models (Section 2.1 classes): diffusion (Poisson/heat,
 * convection-diffusion, compressible Navier-Stokes) and convection (Euler).
 *   POISSON  f = kappa0 * kappa(x) q, s = src - lambda u;  mu = [kappa0, tau, lambda];
 *            aux = [kappa(x)] (optional, naux = 0 means kappa(x) = 1)
 *   CONVDIFF f = kappa0 kappa(x) q + b(x) u, s = src;     mu = [kappa0, tau]; aux = [kappa, b_1..b_nd]
 *   EULER    inviscid flux of (rho, rho v, rho E);         mu = [gamma]
 *   NS       inviscid - viscous flux (Stokes hypothesis, heat flux mu*gamma/Pr grad e),
 *            mu = [gamma, Re, Pr, tau]
 * Interior numerical flux: 1/2 (f- + f+).n + sigma (u- - u+) with
 *   sigma = tau kappa0 {kappa} (Poisson), + 1/2 max|b.n| (convection-diffusion),
 *   sigma = 1/2 max(|v.n| + c) (Euler), + tau / Re (NS);
 * numerical trace uhat = (u- + u+)/2.  tau is the interior-penalty parameter
 * chosen by the caller (the tests use (p+1)^2 / h). */
typedef enum {
  LDG_MODEL_POISSON = 0,
  LDG_MODEL_CONVDIFF = 1,
  LDG_MODEL_EULER = 2,
  LDG_MODEL_NS = 3,
  LDG_MODEL_USER = 4   /* physics from a source compiled at run time (ldg_model_create_user) */
} ldg_model_kind;

/* Boundary condition per boundary tag.
 *   DIRICHLET: uhat = g, u+ = g, q+ = q- in the interior flux formula
 *   NEUMANN:   uhat = u-, Fhat = h (normal flux data)
 *   EXTRAP:    uhat = u-, Fhat = f(u-, q-).n
 * Periodicity is a property of the mesh (matched faces), not a tag. */
typedef enum { LDG_BC_DIRICHLET = 0, LDG_BC_NEUMANN = 1, LDG_BC_EXTRAP = 2 } ldg_bc_kind;

typedef struct ldg_mesh_s* ldg_mesh;
typedef struct ldg_model_s* ldg_model;
typedef struct ldg_precond_s* ldg_precond;
typedef struct ldg_mlp_s* ldg_mlp;

/* Text of the last non-OK status on this thread (empty if none). */
const char* ldg_last_error(void);

/* ---------------------------------------------------------------- mesh ---- */
/* Mesh set-up (runs once, on the host, then uploads): connectivity, periodic
 * matching, boundary-face list and tags, distance-2 element colouring (used to
 * probe Jacobian diagonal blocks), multilinear geometry.  Section 3.2 (mesh
 * module for simple geometries).
 *   nd in {2,3}; p in [1,5]; nq1d >= p+1 (the operator kernels exist for quads with
 *             p <= 4 and hexes with p <= 3: ldg_model_create rejects other orders)
 *   vert      HOST [nvert][nd]
 *   elem_vert HOST [nelem][2^nd], lexicographic corners
 *   period    HOST [nd], >0 marks a periodic direction of that length (vertices
 *             on the two periodic ends must be the same vertex ids), 0 = none
 *   face_tag  HOST [nelem][2nd] tag of each boundary face (ignored for
 *             interior faces), or NULL = tag 0 everywhere
 * Errors: LDG_EINVAL (sizes, degenerate element, face shared by >2 elements),
 * LDG_EUNSUPPORTED (inconsistent face orientation, nq1d > p+1 on a non-affine
 * mesh is only rejected later at model creation). */
ldg_status ldg_mesh_create(int nd, int p, int nq1d, int64_t nvert, const double* vert, int64_t nelem,
                           const int64_t* elem_vert, const double* period, const int32_t* face_tag,
                           ldg_mesh* out);

/* info HOST [8] = {nelem, nodes per element, volume quadrature points per
 * element, points per face, boundary faces, colours, affine (0/1), nd}. */
ldg_status ldg_mesh_info(ldg_mesh mesh, int64_t* info);

/* HOST outputs (any may be NULL): node coordinates [E][nn][nd], volume
 * quadrature points [E][nqv][nd], boundary-face quadrature points
 * [nbf][nqf][nd], boundary faces as (element, local face) [nbf][2]. */
ldg_status ldg_mesh_points(ldg_mesh mesh, double* xnode, double* xquad, double* xbface, int64_t* bface);
ldg_status ldg_mesh_destroy(ldg_mesh mesh);

/* ---------------------------------------------------------------- model --- */
typedef struct {
  int kind;                 /* ldg_model_kind                                    */
  int ncu;                  /* 1 (Poisson, conv.-diff.) or nd+2 (Euler, NS)      */
  int nmu;                  /* <= 8                                              */
  const double* mu;         /* HOST [nmu] parameters (see ldg_model_kind)        */
  int naux;                 /* nodal coefficient fields                          */
  const double* aux;        /* DEVICE [E][naux][nn] or NULL                      */
  const double* src;        /* DEVICE [E][ncu][nqv] source at quadrature points  */
  const double* bdata;      /* DEVICE [nbf][ncu][nqf] boundary data or NULL      */
  int nbc;                  /* <= 8 tags                                         */
  const int32_t* bc_kind;   /* HOST [nbc] ldg_bc_kind per tag                    */
} ldg_model_desc;

/* Binds a model to a mesh.  The aux/src/bdata arrays are read during this call
 * (data terms of linear models are integrated once here) and, for the nonlinear
 * models, kept by pointer: they must stay valid while the model is used.
 * Errors: LDG_EINVAL (ncu, nmu, tags), LDG_EUNSUPPORTED (see nq1d above; no
 * compiled kernel for this (nd, p, model)). */
ldg_status ldg_model_create(ldg_mesh mesh, const ldg_model_desc* desc, void* stream, ldg_model* out);
ldg_status ldg_model_destroy(ldg_model model);

/* Model with run-time compiled physics.  The paper generates the flux, source
 * and boundary code of each PDE from its description (Section 3); here the
 * caller passes the pointwise physics as C++ source, compiled with hipRTC for
 * gfx950 together with the library's operator kernels for this mesh's element
 * type and order (one-off, a few seconds).  The source defines
 *
 *   struct LdgUser {
 *     static constexpr int NCU = ...;      conserved variables (= desc->ncu)
 *     static constexpr bool HASQ = ...;    the flux depends on q = -grad u (= has_q)
 *     static constexpr int NAUX = ...;     aux fields read (upper bound of desc->naux)
 *     template <int D, class V, class R> __device__ static void
 *       flux(const double* mu, int naux, const V* u, const V (*q)[D], const R* a, V (*f)[D]);
 *     template <int D, class V, class R> __device__ static void
 *       numflux(const double* mu, int naux, const V* uL, const V (*qL)[D], const R* aL,
 *               const V* uR, const V (*qR)[D], const R* aR, const R* n, V* Fh);
 *   };
 *
 * R is double or float; V is R or the dual number ldg::Dl<R> (value and
 * tangent), so the same source yields exact Jacobian-vector products.  Helpers
 * from the library's device header are in scope (ldg::VT<V>::mk, vsqrt, vabs,
 * vmax).  f is the physical flux [NCU][D] (R = -(f, grad phi) + <Fh, phi> -
 * (src, phi)), Fh the numerical flux along the unit normal n (interior faces,
 * Dirichlet faces with uR = g, qR = qL); Neumann and extrapolation tags behave
 * as for the built-in models.  A source may also define the state-dependent
 * source s(u, q) of Eq. 1b, which enters the residual as -(s, phi) beside the
 * data field desc->src:
 *
 *     static constexpr bool SOURCE = true;
 *     template <int D, class V, class R> __device__ static void
 *       source(const double* mu, int naux, const V* u, const V (*q)[D], const R* a, V* s);
 *
 * (s: [NCU] at one point), and the outside state of its Dirichlet-kind faces
 * (e.g. a slip wall):
 *
 *     static constexpr bool BOU = true;
 *     template <int D, class V, class R> __device__ static void
 *       bou(const double* mu, int naux, int tag, const V* uL, const V (*qL)[D],
 *           const R* aL, const R* n, V* ub);
 *
 * ub arrives holding the tag's data g (zero without boundary data) and leaves
 * holding uR for numflux; the outside gradient there is qR = qL, and the
 * gradient equation's boundary trace stays uhat = g.  desc->kind must be
 * LDG_MODEL_USER.  The model is nonlinear: JVPs need u.
 * Errors: LDG_EINVAL with the compiler's log in ldg_last_error() when the
 * source does not compile; otherwise as ldg_model_create. */
ldg_status ldg_model_create_user(ldg_mesh mesh, const ldg_model_desc* desc, const char* physics_source, int has_q,
                                 void* stream, ldg_model* out);

/* Compiles a physics source as ldg_model_create_user would for (nd, p, ncu,
 * has_q), on the host only (no device needed): LDG_OK, or LDG_EINVAL with the
 * compiler's log in ldg_last_error(). */
ldg_status ldg_user_physics_check(const char* physics_source, int nd, int p, int ncu, int has_q);

/* Implicit time wrapper (the configurations use BDF1/BDF2; DIRK stages have the
 * same form): G(u) = a0 M u - M (c1 r1 + c2 r2) + R(u).  r1, r2 are DEVICE
 * [E][ncu][nn] or NULL.  A NULL ldg_time* means steady: G = R. */
typedef struct {
  double a0;
  const double* r1;
  double c1;
  const double* r2;
  double c2;
} ldg_time;

/* The ODE that the paper couples to the PDE (Eq. 1c): alpha dw/dt + beta w =
 * s_w(u), with w (nw components) at the element nodes, DEVICE [E][nw][nn].  A
 * physics source defines it by
 *
 *     static constexpr int NW = ...;       in [1, 8]
 *     __device__ static void ode_source(const double* mu, int naux, const double* u,
 *                                       const double* a, double* sw);
 *
 * (u: the NCU state values at one node, a: its aux values, sw: [NW]; FP64).
 * w does not enter the PDE, so the ODE is advanced after each implicit stage of
 * the PDE, from that stage's state.  ldg_ode_size: nw, 0 when the model has no
 * ODE (all built-in models).  ldg_ode_stage: one implicit stage with the time
 * wrapper t, whose r1, r2 are here w-vectors [E][nw][nn] (or NULL):
 *     w = (alpha (c1 r1 + c2 r2) + s_w(u)) / (alpha a0 + beta)   at every node,
 * u the stage's PDE state [E][ncu][nn].  w may alias r1 or r2 (each node reads
 * them before it writes); it must not alias u.  Errors: LDG_EINVAL (null
 * arguments, t NULL, alpha a0 + beta = 0), LDG_EUNSUPPORTED (no ODE). */
ldg_status ldg_ode_size(ldg_model model, int* nw);
ldg_status ldg_ode_stage(ldg_model model, const ldg_time* t, double alpha, double beta, const double* u, double* w,
                         void* stream);

/* ------------------------------------------------------------- operator --- */
/* G(u) (Eq. 1a-1b discretized, with the time wrapper) and optionally
 * q_out = q(u).  prec: LDG_FP64 or LDG_FP32 (others -> LDG_EINVAL). */
ldg_status ldg_residual(ldg_model model, const ldg_time* t, const double* u, double* G, double* q_out,
                        ldg_precision prec, void* stream);

/* Jv = dG/du(u) v, exact forward-mode tangent (Section 3.3: JVP by automatic
 * differentiation) in the requested precision, or a one-sided finite
 * difference with prec = LDG_JVP_FD.  For the linear models u is not read
 * (may be NULL).  u, v, Jv: DEVICE [E][ncu][nn]; Jv must not alias u or v. */
ldg_status ldg_jvp(ldg_model model, const ldg_time* t, const double* u, const double* v, double* Jv,
                   ldg_precision prec, void* stream);

/* The same product with q(u) cached, as the solvers evaluate it (Section 3.3:
 * inside Newton-GMRES every product of one linear solve shares the
 * linearization point u, so q(u) = -grad u of Eq. 1a is formed once).
 * ldg_jvp_prepare computes q(u) into the model's cache for prec (LDG_FP64 or
 * LDG_FP32; a no-op for models without q); ldg_jvp_prepared then evaluates
 * J(u) v like ldg_jvp without recomputing it.  The cache is keyed by the
 * pointer u and the precision: the caller must not change u's contents in
 * between, and ldg_jvp, ldg_gmres_solve, ldg_newton_solve and the block-Jacobi
 * builds on the same model replace the cache.  Errors: LDG_EINVAL when q of
 * this u is not cached in this precision. */
ldg_status ldg_jvp_prepare(ldg_model model, const double* u, ldg_precision prec, void* stream);
ldg_status ldg_jvp_prepared(ldg_model model, const ldg_time* t, const double* u, const double* v, double* Jv,
                            ldg_precision prec, void* stream);

/* The same product with FP32 state: u and v in FP32 storage, FP32 arithmetic and
 * intermediates (the LDG_FP32 mode), Jv in FP64 (it feeds FP64 orthogonalization).
 * Halves the bytes of the input vectors; q(u) is formed from the FP32 state.  For
 * the library's own models (run-time physics: LDG_EUNSUPPORTED).  u, v: DEVICE
 * float [E][ncu][nn]; Jv: DEVICE double, must not alias u or v. */
ldg_status ldg_jvp_state32(ldg_model model, const ldg_time* t, const float* u, const float* v, double* Jv,
                           void* stream);

/* ------------------------------------------------------- preconditioners --- */
/* Exact diagonal blocks dG_K/du_K of the Jacobian at u_lin, by probing with the
 * distance-2 element colouring (one JVP per colour and local unknown), written
 * to blocks: DEVICE [E][nb][nb] row-major, nb = ncu*nn (per_variable = 0) or
 * [E][ncu][nn][nn] (per_variable = 1: the variable-diagonal sub-blocks).  For
 * the library's own models the probing products of one colour run up to 16 seed
 * columns per launch; their vectors (at most 1 GiB) are allocated by the model
 * at its first block build and kept until it is destroyed (LDG_ENOMEM when that
 * allocation fails). */
ldg_status ldg_jacobian_blocks(ldg_model model, const ldg_time* t, const double* u_lin, int per_variable,
                               double* blocks, void* stream);

/* Block-Jacobi preconditioner: the blocks above, inverted by Gauss-Jordan
 * elimination with partial pivoting, stored in FP64, FP32, BF16 or FP16
 * (factor_prec; with any storage below FP64 the probing JVPs run in FP32).  The
 * 16-bit forms store each row of B_K^{-1} divided by a power of two >= its
 * largest magnitude (so every code lies in (-1, 1) and the scaling is exact)
 * and apply in FP64 arithmetic.  Apply: z_K = B_K^{-1} r_K.  Other factor_prec
 * values: LDG_EINVAL. */
ldg_status ldg_precond_block_jacobi(ldg_model model, const ldg_time* t, const double* u_lin, int per_variable,
                                    ldg_precision factor_prec, void* stream, ldg_precond* out);
ldg_status ldg_precond_apply(ldg_precond pc, const double* r, double* z, void* stream);
ldg_status ldg_precond_destroy(ldg_precond pc);

/* ------------------------------------------------- learned preconditioner - */
/* Element-patch MLP (3 layers, ReLU): y = W3 relu(W2 relu(W1 x + b1) + b2) + b3,
 * FP32 master weights, GEMMs on MFMA with bf16 operands and fp32 accumulation
 * (use_bf16 = 1) or in FP32 (use_bf16 = 0).  The network is the learned right
 * preconditioner of flexible GMRES (with block-Jacobi as fallback); it is
 * trained on (residual, correction) pairs the solver generates. */
ldg_status ldg_mlp_create(int in_dim, int width, int out_dim, int nlayers, int use_bf16, ldg_mlp* out);
ldg_status ldg_mlp_destroy(ldg_mlp net);
/* HOST float [nparams], packed W1 b1 W2 b2 W3 b3, W row-major [out][in];
 * nparams = width*in + width + width*width + width + out*width + out.
 * set_params also resets the Adam state. */
ldg_status ldg_mlp_set_params(ldg_mlp net, const float* host_params);
ldg_status ldg_mlp_get_params(ldg_mlp net, float* host_params, float* host_grads);
/* Y[B][out] = net(X[B][in]); DEVICE float arrays. */
ldg_status ldg_mlp_forward(ldg_mlp net, const float* X, int64_t B, float* Y, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): ldg_mlp_forward with
 * the same kernels and the same result, but its hidden activations live in a
 * fixed 32 MiB device array of the library (8,388,608 floats, one per GPU, held
 * until the process ends) instead of the network's lazily grown work buffers.
 * Needs 2 * B * width <= 8,388,608 (B <= 16384 at width 256), else LDG_EINVAL;
 * calls no hipMalloc / hipFree.  Every call on one GPU shares that array, so
 * calls that overlap on one GPU (other streams, other threads) race; calls
 * queued on one stream are ordered.  X, Y: DEVICE float [B][in], [B][out]. */
ldg_status ldg_mlp_forward_noalloc(ldg_mlp net, const float* X, int64_t B, float* Y, void* stream);
/* One step on the mean squared error (1/(B out)) sum (net(X) - Y)^2: forward,
 * backward into the gradient buffer, then Adam (beta 0.9/0.999, eps 1e-8) with
 * learning rate lr when lr > 0.  The loss goes to HOST *loss_host (synchronizes). */
ldg_status ldg_mlp_train_step(ldg_mlp net, const float* X, const float* Y, int64_t B, float lr, float* loss_host,
                              void* stream);
/* Training step of the linear form (ldg_precond_mlp with composite = 2): the
 * network reads the coefficient features X[b][5 nn : 20 nn] of each sample (the
 * layout of ldg_mlp_gather_patches; in_dim = 15 nn) and its output, viewed as
 * the row-major matrix A_b [nn][5 nn] (out_dim = 5 nn^2), multiplies the
 * residual patch X[b][0 : 5 nn]: loss (1/(B nn)) sum (A_b X[b][0:5nn] - Y[b])^2,
 * gradients by the chain rule through the bilinear product, then Adam as
 * ldg_mlp_train_step.  X, Y DEVICE float; loss to HOST *loss_host (synchronizes).
 * EINVAL when the network's sizes are not (15 nn, width, 5 nn^2). */
ldg_status ldg_mlp_train_step_bilinear(ldg_mlp net, const float* X, const float* Y, int64_t B, float lr,
                                       float* loss_host, void* stream);
/* Patch features of the listed elements (elem_idx DEVICE int32 [B], or NULL =
 * all elements in order) of a 2D scalar model: the element and its four face
 * neighbours (-x, +x, -y, +y; zeros outside the domain) give
 * X[B][20 nn] = [r/s (5 nn) | log kappa (5 nn) | b_x/100, b_y/100 per patch element (10 nn)],
 * s = ||r on the patch||_2 + 1e-300 (S[B], DEVICE double, optional), and when
 * e_target is given Y[B][nn] = e on the element / s. */
ldg_status ldg_mlp_gather_patches(ldg_model model, const double* r, const double* e_target, const int32_t* elem_idx,
                                  int64_t B, float* X, float* Y, double* S, void* stream);
/* Learned right preconditioner (the learned-preconditioner pattern of the
 * Newton-Krylov solver, Section 3.3, with block-Jacobi as its base), in one of
 * three forms:
 *  composite = 0: z = s N(patches(r) / s)              (net: 20 nn -> nn)
 *  composite = 1: z = B^-1 r + s N(patches(r) / s)     (net: 20 nn -> nn)
 *  composite = 2: z = B^-1 (r + A_K patch(r)_K), the linear form: the network
 *                 maps the coefficient features of element K's patch (15 nn,
 *                 the layout of ldg_mlp_gather_patches after its residual part)
 *                 to the matrix A_K [nn][5 nn] (5 nn^2 outputs), evaluated for
 *                 every element here, once (on the null stream, synchronized);
 *                 later changes of the network's parameters need a new
 *                 preconditioner.  Needs aux = [kappa, b_x, b_y].
 * Forms 1 and 2 need the block-Jacobi fallback_bj.  EINVAL when the network's
 * sizes do not match the form.  Inside ldg_gmres_solve it is replaced by
 * fallback_bj for the rest of the solve when its output is non-finite or the
 * residual drops by less than 1% over opts.watch_window iterations
 * (stats.fell_back = 1).  The handles must outlive it. */
ldg_status ldg_precond_mlp(ldg_model model, ldg_mlp net, ldg_precond fallback_bj, int composite, ldg_precond* out);

/* ---------------------------------------------------------------- solvers - */
typedef struct {
  int restart;            /* Krylov basis size m                                  */
  int maxit;              /* total iteration cap                                  */
  int flexible;           /* 1 = FGMRES (store Z), 0 = right-preconditioned GMRES */
  double rtol, atol;      /* stop when |g_{j+1}| <= max(rtol ||r0||, atol)        */
  ldg_precision jvp_prec; /* precision of the Jacobian-vector products            */
  ldg_precond pc;         /* NULL = no preconditioner                             */
  int inject_fault;       /* test hook: 1 = poison the preconditioner output with NaN */
  int orth;               /* 0 = CGS2 (three streaming sweeps over the basis), 1 = modified Gram-Schmidt,
                             2 = CGS2 with the re-orthogonalization delayed to the next step (two sweeps) */
  int state32;            /* 1 = FP32 state: the preconditioned vectors z_j and the linearization point are
                             stored in FP32 and the products read them in FP32 (as ldg_jvp_state32); the
                             basis V, Gram-Schmidt, Givens and the true residual stay FP64.  Needs
                             jvp_prec = LDG_FP32, orth = 2 and a block-Jacobi preconditioner or none */
  int watch_window;       /* learned preconditioner (ldg_precond_mlp): it is replaced by its block-Jacobi
                             fallback when the residual estimate falls by less than 1% over this many
                             consecutive iterations; 0 = one restart cycle (restart iterations), < 0 = no
                             stagnation watch (a non-finite output still falls back) */
  double* record_v;       /* training-data hook, NULL = off: DEVICE [record_max][n] each; step i (counted over
                             restarts) stores the vector v_i it hands to the preconditioner in record_v[i]
                             and the product J z_i of the preconditioner's output z_i in record_jz[i], for
                             i < record_max.  With block-Jacobi (z_i = B^-1 v_i) the residual J z_i has the
                             exact correction z_i, with B z_i = v_i.  Not with state32; ldg_newton_solve
                             ignores it in its inner solves */
  double* record_jz;
  int record_max;
} ldg_gmres_opts;

typedef struct {
  int iters, restarts, fell_back;
  double res0, res_est, res_true;          /* ||b - J x0||, Givens estimate, true ||b - J x|| */
  double t_jvp, t_pc, t_orth, t_total;     /* seconds per phase: the preconditioner, JVP and
                                              orthogonalization times are measured on every
                                              8th Arnoldi step and scaled to all steps;
                                              t_total is the wall time of the call       */
} ldg_gmres_stats;

/* Solves J(u_lin) x = b by restarted (F)GMRES with classical Gram-Schmidt and
 * one re-orthogonalization pass (CGS2, or modified Gram-Schmidt with orth = 1)
 * in FP64, Givens rotations in FP64 on the device.  x holds the initial guess on
 * entry and the solution on exit.
 * Returns LDG_ENOCONV if maxit is reached, LDG_EBREAKDOWN on a non-finite
 * value. */
ldg_status ldg_gmres_solve(ldg_model model, const ldg_time* t, const double* u_lin, const double* b, double* x,
                           const ldg_gmres_opts* opts, ldg_gmres_stats* stats, void* stream);

typedef struct {
  int maxit;             /* Newton iteration cap                                       */
  double rtol, atol;     /* stop when ||G(u_k)|| <= max(rtol ||G(u_0)||, atol)          */
  double eta;            /* linear solve relative tolerance (forcing term)              */
  int bj_refresh;        /* rebuild the block-Jacobi preconditioner: 0 never, 1 at every
                            iterate, 2 at the first iterate only (lagged)               */
  int bj_per_variable;   /* for bj_refresh                                              */
  ldg_precision bj_prec; /* storage precision of the refreshed blocks                   */
  ldg_gmres_opts lin;    /* inner solver options (rtol is replaced by eta)              */
} ldg_newton_opts;

typedef struct {
  int iters, gmres_iters;
  double res0, res_final, seconds;
  int lin_status;
  double t_jvp, t_pc, t_orth;   /* seconds per phase, summed over the inner solves */
} ldg_newton_stats;

/* Newton's method on G(u) = 0 (Section 3.3), FP64 residual, u updated in place. */
ldg_status ldg_newton_solve(ldg_model model, const ldg_time* t, double* u, const ldg_newton_opts* opts,
                            ldg_newton_stats* stats, void* stream);

/* ------------------------------------------------------------- utilities -- */
/* Device vector helpers used by the Python binding and the solvers:
 * y = a x + b y, and the squared 2-norm of x written to HOST *out (synchronizes). */
ldg_status ldg_axpby(int64_t n, double a, const double* x, double b, double* y, void* stream);
ldg_status ldg_norm2(int64_t n, const double* x, double* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LDG_H */
