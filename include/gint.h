/*
 * gint.h -- C ABI of the MI355X (gfx950) real-space grid-integration library.
 *
 * The library evaluates, on one GPU, the three uniform-mesh integrals of
 * NAO-based DFT / RT-TDDFT described in Sec. 3.3.1 ("Uniform Grid
 * Integration for Usual Quantities") of arXiv:2603.21835, at the Gamma point:
 *
 *   H_mu,nu   = dV sum_g phit_mu(r_g) V(r_g) phit_nu(r_g)        (H^loc equation)
 *   rho(r_g)  = sum_{mu,nu} D_mu,nu phit_mu(r_g) phit_nu(r_g)     (rho(r_g) equation)
 *   dE/dR_I   for E = dV sum_g W(r_g) rho(r_g)                   (F^{loc,Pulay} equation,
 *                                                                 returned as the gradient,
 *                                                                 i.e. minus the force)
 *
 * where phit_mu is the numerical atomic orbital f_{l zeta}(r) Y_lm(r^) of
 * Sec. 2.1 folded over all lattice images (the k = 0 case of the lattice sums
 * of the rho(r_g) and H(k) equations), f is the clamped cubic spline through
 * the caller's radial table, Y_lm are real spherical harmonics (no
 * Condon-Shortley phase), r_g = sum_i (n_i/N_i) a_i and dV = |det A|/(N1 N2 N3).
 *
 * Units: Hartree atomic units (bohr, Ha).  All caller-visible floating-point
 * data is FP64 in every precision mode.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Orbital order: atoms in input order; within an atom the species' radials
 *    sorted by l (stable, so radials of equal l keep their order = zeta),
 *    then m = -l..l.  gint_norb() gives the total.
 *  - Mesh arrays (V, W, rho) are N1*N2*N3 doubles, C order (index
 *    (n1*N2 + n2)*N3 + n3, n3 fastest).  Matrices (H, D) are norb*norb
 *    doubles, row-major.
 *  - Ownership: pointers marked "device" are caller-owned device memory
 *    (e.g. torch.Tensor.data_ptr()); the library never frees or keeps them
 *    beyond the call.  Host pointers are read during the call only.  The
 *    plan owns its spline tables, binning lists and work buffers.
 *  - Streams: every call enqueues its kernels on the plan's HIP stream and
 *    returns without waiting, except where stated (plan creation and
 *    gint_plan_set_positions read back list sizes and synchronise the stream).
 *  - Errors: invalid arguments are detected on the host before anything is
 *    enqueued and return GINT_EINVAL with outputs untouched.  A failed HIP
 *    call returns GINT_EDEVICE; asynchronous device errors surface on the
 *    next call or on gint_plan_sync.  No C++ exception crosses this ABI.
 *    gint_last_error() returns a message for the calling thread's last
 *    failure.
 *  - Outputs are overwritten, not accumulated.
 *  - A plan is not thread-safe; distinct plans may be used concurrently on
 *    distinct streams.
 *  - Limits: l <= 2, at most 16 orbitals per atom, 1 <= natom <= 16384,
 *    radial tables with nr >= 4 knots, N1*N2*N3 < 2^31.
 */
#ifndef GINT_H
#define GINT_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GINT_OK = 0,
    GINT_EINVAL = 1,       /* invalid argument (nothing enqueued)          */
    GINT_ENOMEM = 2,       /* device or host allocation failed             */
    GINT_EDEVICE = 3,      /* no usable gfx950 device, or a HIP call failed */
    GINT_EUNSUPPORTED = 4, /* valid but not supported (e.g. l > 2)         */
    GINT_ESTATE = 5        /* plan destroyed, corrupted or not ready       */
} gint_status;

/* Arithmetic of the contractions.  Inputs/outputs stay FP64 in all modes;
   the cross-batch reductions and the final dot products are FP64 in all
   modes.  The 16-bit modes apply to H; rho and the force then run as in
   GINT_FP32, except in GINT_FP16_SPLIT, where gint_rho_force, gint_force and
   gint_H_rho_force also contract T = (D + D^T) phi as FP16 hi/lo products
   (gint_build_rho keeps FP32).  Split modes write each operand as hi + lo
   (both 16-bit) and sum hi.hi + hi.lo + lo.hi on the matrix cores (3
   products).  FP16 operands are scaled by 2^8, so the scaled values must stay
   inside the FP16 range: |D_mu,nu + D_nu,mu|, |phi| and |w|^(1/2) |phi| below
   255; larger values overflow to infinity (practical density matrices and
   normalised orbitals are of order one). */
typedef enum {
    GINT_FP64 = 0,       /* FP64 orbitals, FP64 MFMA                          */
    GINT_FP32 = 1,       /* FP32 orbitals, FP32 MFMA (FP32 within a batch)     */
    GINT_BF16 = 2,       /* H: BF16 operands, FP32 accumulation, one product   */
    GINT_FP16 = 3,       /* H: FP16 operands (scaled), FP32 accumulation       */
    GINT_BF16_SPLIT = 4, /* H: BF16 hi/lo operands, 3 products                 */
    GINT_FP16_SPLIT = 5  /* H and T: FP16 hi/lo operands (scaled), 3 products  */
} gint_precision;

/* One radial function, tabulated on the host at r_i = i*dr, i < nr; its
 * cutoff is rc = (nr-1)*dr and f = 0 for r >= rc.  dfdr_0 and dfdr_rc are the
 * end slopes of the clamped cubic spline (Sec. 2.1 NAO radial; the radial
 * derivative is taken from the spline, Sec. 2.3 Pulay-force remark). */
typedef struct {
    int l;
    int nr;
    double dr;
    const double *f; /* host, nr doubles */
    double dfdr_0;
    double dfdr_rc;
} gint_radial;

typedef struct {
    int nradial;
    const gint_radial *radial; /* host, nradial entries */
} gint_species;

/* Work counts of the current geometry, for throughput reporting. */
typedef struct {
    long long ngrid;       /* N1*N2*N3                                           */
    long long nbatch;      /* mesh batches                                       */
    long long nentry;      /* (batch, atom) pairs after binning                  */
    long long npair;       /* active atom-group pairs                            */
    double sum_ng;         /* sum over mesh points of supported orbitals n_g     */
    double sum_ng2;        /* sum over mesh points of n_g^2                      */
    int batch[3];          /* batch shape in mesh points                         */
    int nslab;             /* batch ranges the H path is split into              */
    long long nblock;      /* H atom-pair block partials over all batches         */
    int mno;               /* block partial edge (most orbitals of one atom)      */
    int partial_bytes;     /* bytes per block partial element (8 FP64, 4 else)    */
    long long nblock_hr;   /* block partials of the unfolded atom images (H(R)),
                              -1 before the first gint_build_HR / gint_HR_lattice
                              call of the current geometry                      */
} gint_work;

typedef struct gint_plan_s *gint_plan;

/* Create a plan: geometry, mesh and basis (the GintInfo role of Fig. 2:
 * mesh division into batches and batch/atom neighbour lists).
 *   lattice          host, 9 doubles, rows a1, a2, a3 (bohr), det != 0
 *   grid             host, 3 ints N1, N2, N3 >= 1
 *   species          host, nspecies entries (see limits above)
 *   species_of_atom  host, natom ints in [0, nspecies)
 *   positions        host, natom*3 doubles, cartesian (any image)
 *   prec             arithmetic of the contractions
 *   hip_stream       hipStream_t to enqueue on (NULL = default stream)
 *   out              receives the plan (unchanged on error)
 * Batches start as 4x4x2 mesh points; an FP64 or FP32 plan whose atoms are
 * too many for the LDS of a 32-point batch starts with 2x2x4 instead
 * (gint_work reports the shape).  Synchronises the stream (list sizes are
 * read back). */
gint_status gint_plan_create(const double lattice[9], const int grid[3], int nspecies,
                             const gint_species *species, int natom, const int *species_of_atom,
                             const double *positions, gint_precision prec, void *hip_stream,
                             gint_plan *out);

/* Move the atoms (host, natom*3 doubles) and rebuild the binning lists on
 * the GPU.  Synchronises the stream once. */
gint_status gint_plan_set_positions(gint_plan plan, const double *positions);

/* Batch shape (mesh points per batch along each axis; product 16 or 32) and
 * the device-memory budget (bytes) of the H path's per-batch block partials
 * (0 = automatic: min(64 GiB, a third of free memory)); a smaller budget
 * splits H into more batch ranges.  Rebuilds the lists; synchronises the
 * stream. */
gint_status gint_plan_tune(gint_plan plan, const int batch[3], long long h_budget_bytes);

/* Change the stream subsequent calls enqueue on. */
gint_status gint_plan_set_stream(gint_plan plan, void *hip_stream);

/* H^loc of Sec. 3.3.1 (Gamma point, images folded):
 *   V_dev  device, N1*N2*N3 doubles (Ha)
 *   H_dev  device, norb*norb doubles, row-major, overwritten; exactly
 *          symmetric (each pair is computed once and mirrored). */
gint_status gint_build_H(gint_plan plan, const double *V_dev, double *H_dev);

/* As gint_build_H with the per-point weight given directly:
 * H_mu,nu = sum_g w_g phit_mu phit_nu (no dV factor).  This is the
 * derivative of sum_g w_g rho_g with respect to D. */
gint_status gint_build_H_weighted(gint_plan plan, const double *w_dev, double *H_dev);

/* Moving-basis matrix of Sec. 2.3 (Ehrenfest dynamics, D_K equation) at the
 * Gamma point, on the mesh, with an optional weight W:
 *   DK_c,mu,nu = < phit_mu | W | d phit_nu / d tau_K >_c,  K = atom of nu,
 *              = -dV sum_g W_g phit_mu(r_g) d/dr_c phit_nu(r_g),  c = x, y, z
 * (an orbital depends on its centre tau_K only through r - tau_K; at k = 0
 * the lattice sum of the D_K equation folds the orbital).  D_K,mu,nu is zero
 * unless nu is on K, so one array holds every D_K.  With W = 1 the mesh
 * overlap S_grid (gint_build_H_weighted with w = dV) has the derivatives
 *   dS_mu,nu / dtau_K = DK[.][nu][mu] (mu on K) + DK[.][mu][nu] (nu on K),
 * and P_mu,nu = -i sum_K tau_dot_K . D_K,mu,nu is the P matrix of the TDKS
 * equation with moving orbitals.  With W = V,
 *   dE/dR_I = sum_{mu on I} sum_nu (D + D^T)_mu,nu DK[.][nu][mu]
 * for E = dV sum_g V_g rho_g (gint_force).
 *   W_dev   device, N1*N2*N3 doubles, or NULL for W = 1
 *   DK_dev  device, 3*norb*norb doubles: DK[c][mu][nu] at
 *           (c*norb + mu)*norb + nu, input orbital order; overwritten.
 * One workgroup per atom pair within reach of each other walks the mesh
 * batches the two share in batch order and keeps the pair's sums on the
 * FP64 matrix cores; the plan's precision does not apply (FP64 always);
 * repeatable bits. */
gint_status gint_build_DK(gint_plan plan, const double *W_dev, double *DK_dev);

/* rho(r_g) of Sec. 3.3.1 (Gamma point, images folded):
 *   D_dev    device, norb*norb doubles, row-major, used as given (a
 *            non-symmetric D acts through its symmetric part)
 *   rho_dev  device, N1*N2*N3 doubles, overwritten. */
gint_status gint_build_rho(gint_plan plan, const double *D_dev, double *rho_dev);

/* Gradient of E = dV sum_g W_g rho_g with respect to the atom positions
 * (minus F^{loc,Pulay} of Sec. 3.3.1; W does not move with the atoms):
 *   dE/dR_I = -dV sum_g W_g sum_{mu in I} grad phit_mu(r_g) . [(D + D^T) phit(r_g)]_mu
 *   W_dev     device, N1*N2*N3 doubles
 *   D_dev     device, norb*norb doubles
 *   dEdR_dev  device, natom*3 doubles (input atom order), overwritten. */
gint_status gint_force(gint_plan plan, const double *W_dev, const double *D_dev, double *dEdR_dev);

/* As gint_force with the per-point weight w_g given directly (no dV):
 * the gradient of sum_g w_g rho_g. */
gint_status gint_force_weighted(gint_plan plan, const double *w_dev, const double *D_dev,
                                double *dEdR_dev);

/* rho and the gradient of E = dV sum_g W_g rho_g in one pass over the mesh:
 * the force's T_I = sum_J (D + D^T)_IJ phit_J also gives
 * rho_g = 1/2 sum_I phit_I(r_g) . T_I(r_g), so rho costs one dot product per
 * (point, atom) on top of the force.  Arguments as gint_build_rho and
 * gint_force; rho_dev and dEdR_dev are both overwritten. */
gint_status gint_rho_force(gint_plan plan, const double *W_dev, const double *D_dev, double *rho_dev,
                           double *dEdR_dev);

/* H (gint_build_H), rho and the force (gint_rho_force) of one potential V
 * and density matrix D in one call; results are bitwise those of the two
 * separate calls.  In the FP64 and FP32 modes one pass per mesh batch
 * evaluates the orbital tiles once for the H blocks, rho and the force (the
 * three integrals of Sec. 3.3.1 share the orbital values of a batch); in the
 * 16-bit modes, or when a batch holds too many orbitals for that pass, the H
 * path runs on the plan's stream beside the rho / force pass on a second
 * stream of the plan (default priority), forked from and joined back into the
 * plan's stream within the call (the paper runs independent integration work
 * on several streams).  Arguments as gint_build_H and gint_rho_force; H_dev,
 * rho_dev and dEdR_dev must not overlap.  Errors as the separate calls
 * (GINT_EDEVICE if the second stream cannot be created). */
gint_status gint_H_rho_force(gint_plan plan, const double *V_dev, const double *D_dev, double *H_dev,
                             double *rho_dev, double *dEdR_dev);

/* Lattice-vector blocks of H^loc (Sec. 3.3.1, H^loc(R) equation; the sum
 * over g runs over the mesh points of the whole crystal):
 *   H_mu,nu(R) = dV sum_g phi_mu(r_g - tau_I) V(r_g) phi_nu(r_g - tau_J - R),
 * R = n1 a1 + n2 a2 + n3 a3, tau the positions as given to the plan (not
 * wrapped into the cell).  sum_R e^{ik.R} H(R) is H(k) of Sec. 2.1; the sum
 * over all R is gint_build_H's Gamma-point H.
 *   V_dev   device, N1*N2*N3 doubles (Ha)
 *   nR, R   host, nR >= 1 distinct lattice multiples (n1, n2, n3) as 3*nR
 *           ints, each |n_k| <= 31
 *   HR_dev  device, nR*norb*norb doubles: block q (row-major norb x norb)
 *           is H(R_q); overwritten.  Contributions to R not in the list
 *           are dropped; gint_HR_lattice lists the R that can have any.
 * The blocks of each (I, J, R) are summed in a fixed order (repeatable
 * bits) when the block partials of the unfolded atom images fit the
 * partial-buffer budget (gint_plan_tune); otherwise they are added into
 * HR_dev with FP64 atomics (the last bits can then differ between calls).
 * The matrix-core products follow the plan's precision as in gint_build_H
 * (the atomic fallback uses FP32 tiles for every non-FP64 precision); sums
 * across batches are FP64.
 * GINT_EINVAL for bad arguments (outputs untouched); GINT_EUNSUPPORTED if
 * too many atom images reach one mesh batch. */
gint_status gint_build_HR(gint_plan plan, const double *V_dev, int nR, const int *R, double *HR_dev);

/* rho from lattice-vector blocks of the density matrix (Sec. 3.3.1, rho(r_g)
 * equation with its sums over R and R'):
 *   rho(r_g) = sum_{R, R'} sum_{mu nu} D_mu,nu(R) phi_mu(r_g - tau_I - R')
 *                                                phi_nu(r_g - tau_J - R - R'),
 * tau the positions as given (as gint_build_HR).
 *   nR, R    host, nR >= 1 distinct lattice multiples as in gint_build_HR
 *   DR_dev   device, nR*norb*norb doubles: block q is D(R_q), row-major, used
 *            as given (blocks of unlisted R are zero)
 *   rho_dev  device, N1*N2*N3 doubles, overwritten; each point written once
 *            by one workgroup (fixed order, repeatable bits).
 * FP64 plans evaluate orbitals and products in FP64, the other precisions in
 * FP32 (FP32 matrix-core products); sums are FP64.  Errors as gint_build_HR.
 * With D(R) = D for every R of gint_HR_lattice, rho is gint_build_rho's. */
gint_status gint_build_rhoR(gint_plan plan, int nR, const int *R, const double *DR_dev, double *rho_dev);

/* dE/dR for E = dV sum_g V_g rho_g with rho from lattice-vector density
 * blocks as in gint_build_rhoR (Sec. 3.3.1, F^{loc,Pulay} equation with its
 * sum over R): moving an atom moves all its images, and
 *   dE/dR_I = -dV sum_g V_g sum_{images a of I} grad phi_a . t_a,
 *   t_a = sum_{images c} [D_{I J_c}(T_c - T_a) + D_{J_c I}(T_a - T_c)^T] phi_c.
 *   V_dev     device, N1*N2*N3 doubles (Ha)
 *   nR, R     host lattice multiples as in gint_build_HR
 *   DR_dev    device, nR*norb*norb doubles, used as given
 *   dEdR_dev  device, natom*3 doubles, input atom order, overwritten
 * Per-(batch, image) partials summed per atom in a fixed order (repeatable
 * bits).  Precision and errors as gint_build_rhoR.  With D(R) = D for every
 * R of gint_HR_lattice this is gint_force's dE/dR. */
gint_status gint_forceR(gint_plan plan, const double *V_dev, int nR, const int *R, const double *DR_dev,
                        double *dEdR_dev);

/* Bloch sum of lattice-vector blocks (Sec. 2.1, H(k) equation):
 *   H(k) = sum_q e^{i k.R_q} H(R_q),  k.R_q = 2 pi (kappa . n_q),
 * kappa the fractional coordinates of k in the reciprocal basis (b_i with
 * a_i . b_j = delta_ij).  Works for any blocks of this plan's size (H(R) of
 * gint_build_HR, or S(R), ...).
 *   nR, R     host, the lattice multiples of the blocks (3*nR ints)
 *   HR_dev    device, nR*norb*norb doubles
 *   nk, kfrac host, 3*nk doubles
 *   Hk_dev    device, nk*norb*norb complex values as (re, im) double pairs,
 *             row-major per k; overwritten
 * Phases are formed in FP64 on the host; sums are FP64.  Synchronises the
 * stream once. */
gint_status gint_HR_to_Hk(gint_plan plan, int nR, const int *R, const double *HR_dev, int nk, const double *kfrac,
                          double *Hk_dev);

/* gint_HR_to_Hk for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, output and conventions, and no device allocation in
 * the call.  Its workspace (the phase table and the staged R and kfrac) is
 * a fixed device array of the library, about 1.3 MiB, that each GPU holds
 * from the first call on it until the process ends; the phases are formed
 * on the device (FP64 sincospi) instead of the host, so results agree with
 * gint_HR_to_Hk to rounding.  Limits: nR <= 8192, nk <= 8192 and
 * nR * nk <= 65536, else GINT_EINVAL (nothing enqueued).  Every call on a
 * GPU shares that GPU's workspace: calls that overlap on one GPU (several
 * streams or threads) race and must be serialised by the caller.
 * Synchronises the plan's stream once (after staging R and kfrac), then
 * enqueues the sums and returns. */
gint_status gint_HR_to_Hk_noalloc(gint_plan plan, int nR, const int *R, const double *HR_dev, int nk,
                                  const double *kfrac, double *Hk_dev);

/* The lattice vectors R = T_b - T_a over every pair of atom images (a, b)
 * that reach a common mesh batch, for the current positions: every R with
 * a non-zero H(R) block is among them (a superset; |n_k| <= 31 only).
 * Sorted by (n1, n2, n3).
 *   cap   room in R (host, 3*cap ints); cap = 0 (R may be NULL) only counts
 *   nR    host, receives the count
 * GINT_EINVAL (with *nR set) when the count exceeds cap.  Synchronises the
 * stream once. */
gint_status gint_HR_lattice(gint_plan plan, int cap, int *nR, int *R);

/* ---------------------------------------------------------------------
 * Spherical-grid projector overlaps of the velocity-gauge nonlocal
 * pseudopotential (Sec. 3.3.2, "Spherical Grid Integration for Nonlocal
 * Potentials"; the phase-modulated projector overlap of Sec. 2.2):
 *
 *   Q[p][mu] = < phit_mu | e^{-i A.r} | beta_p >
 *            = sum_{i,j} W_ij phit_mu(tau_I + x_ij) e^{-i A.(tau_I + x_ij)} beta_p(x_ij),
 *
 * evaluated on the product grid centred on the projector's atom I:
 * x_ij = r_i u_j with r_i = rb x_i and W_ij = rb q_i r_i^2 w_j, where
 * (u_j, w_j) is the caller's angular rule on the unit sphere (the paper uses
 * the 110-point Lebedev-Laikov rule), (x_i, q_i) its radial rule on [0, 1]
 * (the paper: 140-point Gauss-Legendre) and rb the largest projector cutoff
 * of I's species.  beta_p(x) = b(|x|) Y_lm(x/|x|) with b the clamped cubic
 * spline of the projector table (strict cutoff, the r = 0 limits of the
 * orbitals); phit the orbital folded over lattice images; tau_I the position
 * as given to the plan (gint_plan_set_positions), so moving an atom by a
 * lattice vector L multiplies its rows by e^{-i A.L}.
 * --------------------------------------------------------------------- */
typedef struct gint_psibeta_s *gint_psibeta;

/* Projector tables and quadrature for a plan (the plan must outlive it):
 *   nspecies  must equal the plan's species count
 *   proj      host, nspecies entries: the projector radials of each species
 *             (nradial may be 0: no projectors; l <= 2, at most 16
 *             projectors per species); projectors are ordered like the
 *             orbitals (atoms in input order; radials by l, stable; m)
 *   ang       host, nang*4 doubles: (x, y, z, w) per angular node, unit x
 *   rq        host, nrq*2 doubles: (x, q) per radial node on [0, 1]
 * The neighbour lists (atoms whose orbitals reach each projector sphere) are
 * built on the GPU now and again after the plan's atoms move.  Synchronises
 * the plan's stream. */
gint_status gint_psibeta_create(gint_plan plan, int nspecies, const gint_species *proj, int nang, const double *ang,
                                int nrq, const double *rq, gint_psibeta *out);

/* Rows of Q (projectors over all atoms), or -1. */
int gint_psibeta_nproj(gint_psibeta pb);

/* Q for the vector potential A (host, 3 doubles, bohr^-1):
 *   Q_dev  device, nproj*norb complex values as (re, im) double pairs,
 *          row-major, overwritten.
 * One workgroup per projector atom contracts its projector table against
 * the orbitals of every neighbouring atom over the quadrature points on the
 * FP64 matrix cores; each block is written once (repeatable bits).  FP64 in
 * every plan precision. */
gint_status gint_psibeta_overlap(gint_psibeta pb, const double A[3], double *Q_dev);

void gint_psibeta_destroy(gint_psibeta pb);

/* Kernel classes reported by gint_plan_timing. */
enum {
    GINT_K_BIN = 0,       /* binning kernels of plan creation / set_positions / tune */
    GINT_K_H = 1,         /* H atom-pair blocks (one workgroup per mesh batch)      */
    GINT_K_H_REDUCE = 2,  /* fixed-order block sums into dense H                    */
    GINT_K_RHO = 3,       /* rho contraction (one workgroup per mesh batch)         */
    GINT_K_PACK = 4,      /* D + D^T packed into matrix-core fragments (rho, force) */
    GINT_K_FORCE = 5,     /* force contraction (one workgroup per mesh batch)       */
    GINT_K_F_REDUCE = 6,  /* force reduction per atom                               */
    GINT_K_H_FILL = 7,    /* zero fill of dense H                                   */
    GINT_K_RHO_FORCE = 8, /* rho and force contraction in one pass                  */
    GINT_K_H_RHO_FORCE = 9, /* H blocks, rho and force in one pass (gint_H_rho_force) */
    GINT_K_HR = 10,       /* lattice-vector blocks H(R) (gint_build_HR)            */
    GINT_K_DK = 11,       /* moving-basis matrix (gint_build_DK)                    */
    GINT_K_PSIBETA = 12,  /* spherical-grid projector overlaps (gint_psibeta_overlap) */
    GINT_NKERNEL = 13
};

/* Enable (1) or disable (0) timing: each kernel launch of later calls is
 * bracketed by HIP events recorded on the plan's stream.  Enabling resets the
 * accumulated totals. */
gint_status gint_plan_set_timing(gint_plan plan, int enable);

/* Accumulated device time (ms) and launch count per kernel class since
 * timing was enabled (synchronises the stream).  ms and launches are host
 * arrays of GINT_NKERNEL entries. */
gint_status gint_plan_timing(gint_plan plan, double *ms, int *launches);

/* Wait for the plan's stream and report any asynchronous device error. */
gint_status gint_plan_sync(gint_plan plan);

/* Work counts of the current geometry (computes the exact sum_g n_g^2 on
 * the GPU; synchronises the stream). */
gint_status gint_plan_work(gint_plan plan, gint_work *out);

/* ---------------------------------------------------------------------
 * Batched cells: many independent periodic cells of uneven size, one call
 * for all of them.  The work of a call is captured once into a hipGraph of
 * concurrent chains and replayed with a single graph launch on the batch's
 * stream while the cells' geometry and the caller's device pointers stay
 * the same.  Per-cell conventions are those of the single-cell calls.
 * --------------------------------------------------------------------- */
typedef struct {
    double lattice[9];          /* rows a1, a2, a3                        */
    int grid[3];
    int natom;
    const int *species_of_atom; /* host, natom                            */
    const double *positions;    /* host, natom*3                          */
} gint_cell;

typedef struct gint_batch_s *gint_batch;

/* Create plans for ncell cells sharing one basis (nspecies, species) and
 * precision.  Synchronises the device. */
gint_status gint_batch_create(int ncell, const gint_cell *cells, int nspecies, const gint_species *species,
                              gint_precision prec, void *hip_stream, gint_batch *out);

/* H of every cell.  V_dev, H_dev: host arrays of ncell device pointers. */
gint_status gint_batch_build_H(gint_batch batch, const double *const *V_dev, double *const *H_dev);

/* rho of every cell.  D_dev, rho_dev: host arrays of ncell device pointers. */
gint_status gint_batch_build_rho(gint_batch batch, const double *const *D_dev, double *const *rho_dev);

/* dE/dR of every cell (E = dV sum W rho per cell). */
gint_status gint_batch_force(gint_batch batch, const double *const *W_dev, const double *const *D_dev,
                             double *const *dEdR_dev);

/* H, rho and dE/dR of every cell in one graph replay (gint_H_rho_force per
 * cell, on the cells' chains; the same bits as the single-cell call).  The
 * arrays hold ncell device pointers each. */
gint_status gint_batch_H_rho_force(gint_batch batch, const double *const *V_dev, const double *const *D_dev,
                                   double *const *H_dev, double *const *rho_dev, double *const *dEdR_dev);

/* Choose each cell's batch shape by timing: for every class of cells with
 * the same mesh and atom count, time `reps` rounds of H + rho + dE/dR of
 * the class's first cell on the batch stream for each candidate shape
 * (32-point boxes 4x4x2, 4x2x4, 2x4x4, 8x2x2, 2x2x8 and, except in the
 * 16-bit modes, 16-point 2x2x4 and 4x2x2) and apply the fastest to the
 * whole class.  The buffers are the caller's (device pointers as in the
 * batched calls; their contents are overwritten).  chosen (host, 3*ncell
 * ints, may be NULL) receives each cell's shape.  Synchronises the batch
 * stream; invalidates the captured graphs. */
gint_status gint_batch_autotune(gint_batch batch, const double *const *V_dev, const double *const *D_dev,
                                double *const *H_dev, double *const *rho_dev, double *const *dEdR_dev, int reps,
                                int *chosen);

gint_status gint_batch_sync(gint_batch batch);
int gint_batch_ncell(gint_batch batch);
/* The plan of cell i (owned by the batch; do not destroy).  Moving its
 * atoms or tuning it invalidates the captured graphs, which are re-captured
 * on the next call.  Batched calls run each cell on a stream of the batch
 * (gint_plan_set_stream on a cell affects only its single-cell calls, and
 * per-kernel timing must be off for batched calls: GINT_ESTATE).  Each
 * chain's cells share one H partial buffer of at most 8 GiB. */
gint_plan gint_batch_cell(gint_batch batch, int i);
void gint_batch_destroy(gint_batch batch);

/* The order the plan processes the atoms in (a Morton curve through the
 * cell, recomputed at plan creation): order[i] is the input index of the
 * i-th atom in that order.  order: host, natom ints.  Synchronises the
 * stream.  For tests and diagnostics; results never depend on it beyond
 * rounding. */
gint_status gint_plan_atom_order(gint_plan plan, int *order);

/* Failure injection for tests of the error paths: the next n list rebuilds
 * (plan creation, gint_plan_set_positions, gint_plan_tune) of any plan fail
 * with GINT_ENOMEM before enqueuing anything.  n = 0 disarms it.  Not
 * thread-safe.  When gint_plan_tune fails and restoring the previous batch
 * shape fails too, the plan is left unusable: every call but
 * gint_plan_destroy then returns GINT_ESTATE, and gint_plan_destroy still
 * releases it. */
gint_status gint_test_fail_rebuilds(int n);

/* Test switch of gint_build_rhoR and gint_forceR: with on != 0 every lane
 * gathers its D(R) and D(-R)^T elements one by one, as the calls do when an
 * image pair spans more than 31 cells (no packed blocks); on = 0 (the
 * default) restores the packed blocks.  Results agree to rounding.  Process
 * wide, not thread-safe. */
gint_status gint_test_DR_gather(int on);

int gint_norb(gint_plan plan);   /* total orbitals, or -1 for an invalid plan */
int gint_natom(gint_plan plan);  /* atoms, or -1                               */
double gint_dV(gint_plan plan);  /* mesh volume element, or -1                 */
const char *gint_status_string(gint_status s);
const char *gint_last_error(void);

/* Release the plan and everything it owns (waits for its stream).  NULL is
 * accepted. */
void gint_plan_destroy(gint_plan plan);

#ifdef __cplusplus
}
#endif

#endif /* GINT_H */
