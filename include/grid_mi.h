/*
 * grid_mi.h -- C ABI of the MI355X (gfx950) lattice hopping-operator library.
 *
 * The library applies the nearest-neighbour Wilson hopping term ("Wilson kernel", Grid paper
 * Section 2.4 and Section 3) on a periodic 4D lattice, its Ls-replicated five-dimensional
 * domain-wall extension (Section 3, Table 4 and the xc30 figure's note that the gauge field is
 * reused Ls times), a conjugate-gradient solver on the normal equations (Section 4, "Conjugate
 * gradient") and the adjoint of the hopping term with the gauge-link force that HMC needs
 * (Section 4, "HMC"). The paper names these operators without printing their formulas; the
 * definitions used are stated below and are those of the standard Wilson / Shamir formulation.
 *
 * Definitions (gamma matrices in the Euclidean chiral basis, gamma_k = [[0,-i s_k],[i s_k,0]],
 * gamma_4 = [[0,1],[1,0]], direction mu = 0..3 = x,y,z,t uses gamma_{mu+1}, gamma_5 =
 * diag(1,1,-1,-1), P_+- = (1 +- gamma_5)/2; boundaries periodic in all four directions):
 *
 *   H psi(x)  = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu)
 *   H^+       = the same with gamma_mu -> -gamma_mu
 *   D         = (4 + mass) - H/2                       (Wilson fermion operator)
 *   M psi_s   = (5 - M5) psi_s - H psi_s / 2 - P_- psi~_{s+1} - P_+ psi~_{s-1}   (Shamir DWF)
 *               with psi~_{Ls} = -mf psi_0, psi~_{-1} = -mf psi_{Ls-1};
 *   M^+ psi_s = (5 - M5) psi_s - H^+ psi_s / 2 - P_+ psi~_{s+1} - P_- psi~_{s-1}.
 *   Moebius (the Cayley form of the five-dimensional chiral fermions listed in Section 4):
 *   M_mob = D_W B + 1 - S,  D_W = (4 - M5) - H/2,  B = b5 + c5 S,
 *   (S psi)_s = P_- psi~_{s+1} + P_+ psi~_{s-1} (walls as above), S^+ with P_+ and P_- swapped;
 *   b5 = 1, c5 = 0 is the Shamir M.
 *
 * Data layout (all fields site-major, x fastest, then y, z, t; complex = interleaved re, im):
 *   spinor 4D  [Lt][Lz][Ly][Lx][4 spin][3 colour] complex
 *   spinor 5D  [Lt][Lz][Ly][Lx][Ls][4][3]           (the fifth coordinate inside the 4D site)
 *   links L18  [Lt][Lz][Ly][Lx][4 mu][3][3]          (row-major SU(3) matrix U_mu(x))
 *   links L12  [Lt][Lz][Ly][Lx][4 mu][2][3]          (rows 0, 1; row 2 = conj(row0 x row1))
 * Precisions (argument `prec`):
 *   GRID_F64   spinors and links complex double; arithmetic in double.
 *   GRID_F32   spinors and links complex float;  arithmetic in float.
 *   GRID_F16S  spinors stored as IEEE half (re, im) with one float scale per (4D or 5D) site:
 *              value = float(code) * scale; links stored as half (re, im) without scale;
 *              arithmetic in float. The codec: s = max |re|,|im| over the site's 24 reals (in
 *              float), code = half_rne(float(v) * (1.0f / s)), s = 0 codes zeros.
 *
 * Ownership and streams: the caller allocates every buffer (device memory, 16-byte aligned)
 * and keeps ownership; the library never allocates or frees caller memory. Every call except
 * grid_cg is asynchronous on the given HIP stream (`stream` is a hipStream_t; NULL is the
 * default stream). Outputs must not alias inputs.
 *
 * Errors: 0 on success, a negative GRID_E* code otherwise. Argument checks run on the host
 * before any HIP call, so a rejected call has no effect. grid_last_error() returns a message for
 * the calling thread's last failure.
 */
#ifndef GRID_MI_H
#define GRID_MI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRID_OK           0
#define GRID_EINVAL      -1   /* bad enum value, NULL pointer where one is required, aliasing  */
#define GRID_ESHAPE      -2   /* an extent below 2 (or odd for checkerboards), bad Ls, overflow */
#define GRID_EDTYPE      -3   /* precision / link-format combination not supported             */
#define GRID_EALIGN      -4   /* a pointer not 16-byte aligned                                  */
#define GRID_EHIP        -5   /* a HIP runtime call failed                                      */
#define GRID_ENOCONV     -6   /* CG reached maxiter without the requested true residual        */
#define GRID_EBREAKDOWN  -7   /* CG breakdown: <p, A p> <= 0 or a non-finite scalar            */
#define GRID_ESPACE      -8   /* workspace smaller than grid_cg_workspace_bytes() reports      */

enum grid_prec { GRID_F64 = 0, GRID_F32 = 1, GRID_F16S = 2 };
enum grid_link_fmt { GRID_L18 = 0, GRID_L12 = 1 };
enum grid_op_kind { GRID_HOP = 0, GRID_WILSON = 1, GRID_DWF = 2, GRID_MOBIUS = 3 };

/* Lattice extents (dims[0..3] = Lx, Ly, Lz, Lt, each >= 2) and fifth extent Ls (1 for 4D). */
typedef struct {
    int dims[4];
    int Ls;
} grid_geom;

/* Operator: kind GRID_HOP (H, applied on each fifth slice when Ls > 1), GRID_WILSON (D, Ls = 1),
 * GRID_DWF (Shamir M) or GRID_MOBIUS (M_mob, through grid_mobius and grid_cg only); dag != 0
 * applies the adjoint. mass is D's m; M5, mf the domain-wall parameters; b5, c5 the Moebius
 * coefficients (ignored by the other kinds). */
typedef struct {
    int kind;
    int dag;
    double mass;
    double M5;
    double mf;
    double b5;
    double c5;
} grid_op;

/* Conjugate-gradient parameters. */
typedef struct {
    double tol;        /* target true relative residual |b - A x| / |b| (FP64), e.g. 1e-10      */
    int maxiter;       /* cap on iterations (sloppy iterations in mixed mode)                     */
    int sloppy_prec;   /* GRID_F64: plain FP64 CG; GRID_F32 / GRID_F16S: mixed precision         */
    int link_fmt;      /* link format of the sloppy operator (GRID_L18 or GRID_L12)                */
    double delta;      /* reliable-update threshold (mixed modes), e.g. 0.1                       */
    int check_every;   /* iterations between host reads of the residual norm (>= 1), e.g. 10     */
    int graph;         /* nonzero: the check_every iterations between two host reads are recorded
                          once into a HIP graph (per starting parity, on a stream of the library's
                          own) and replayed on the caller's stream, one graph launch in place of
                          about six kernel launches per iteration; same kernels, same arguments,
                          bit-identical results                                                   */
} grid_cg_params;

/* CG results. */
typedef struct {
    int iterations;          /* operator iterations performed                                  */
    int reliable_updates;    /* FP64 true-residual recomputations during the iteration (mixed) */
    int converged;           /* 1 if true_residual <= tol                                      */
    double true_residual;    /* |b - A x| / |b|, recomputed in FP64 at the end                  */
    double seconds;          /* wall time of the call                                          */
} grid_cg_stats;

/*
 * grid_dhop -- apply the hopping term or a fermion operator built on it (Section 2.4's Wilson
 * kernel; Table 4's Ls-replicated dslash when kind = GRID_HOP and Ls > 1; Section 4's Wilson
 * fermion action and five-dimensional chiral fermions for GRID_WILSON / GRID_DWF).
 *
 *   U         links in precision `prec` and format `link_fmt` (see layout above)
 *   psi       input spinor (4D if geom->Ls == 1, else 5D) in precision `prec`
 *   psi_scale GRID_F16S: per-site scales of psi ([V] or [V][Ls] floats); NULL otherwise
 *   out       output spinor, same shape and precision as psi; must not overlap psi or U
 *   out_scale GRID_F16S: per-site scales written for out; NULL otherwise
 *   op        kind / dag / parameters; GRID_WILSON needs Ls == 1, GRID_DWF needs Ls >= 1
 * Returns GRID_OK, or GRID_EINVAL / GRID_ESHAPE / GRID_EDTYPE / GRID_EALIGN / GRID_EHIP.
 */
int grid_dhop(const void *U, const void *psi, const float *psi_scale, void *out, float *out_scale,
              const grid_geom *geom, const grid_op *op, int prec, int link_fmt, void *stream);

/*
 * grid_dwf_mdag_m -- out = M^+ M psi for the domain-wall operator (the normal operator the CG
 * of Section 4 iterates on). tmp (and tmp_scale for GRID_F16S) receives M psi and must have
 * psi's size. Same argument rules as grid_dhop.
 */
int grid_dwf_mdag_m(const void *U, const void *psi, const float *psi_scale, void *out, float *out_scale,
                    void *tmp, float *tmp_scale, const grid_geom *geom, double M5, double mf, int prec,
                    int link_fmt, void *stream);

/*
 * grid_dwf_mdag_m_noalloc -- grid_dwf_mdag_m for callers that cannot allocate device memory (code
 * under HIP stream capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels, with M psi held in a static scratch array of the library (64 MiB per device, held from
 * module load until the process ends) instead of a caller's tmp. Fields whose M psi needs more
 * (V Ls x 192 / 96 / 52 bytes for FP64 / FP32 / FP16 storage, rounded up) are rejected with
 * GRID_ESPACE. Calls no allocating routine. The scratch is shared by every call on a device: calls
 * that overlap in time on one device (other streams, other threads) race and must be ordered by
 * the caller. `stream` must belong to the current device. Same argument rules as grid_dwf_mdag_m.
 */
int grid_dwf_mdag_m_noalloc(const void *U, const void *psi, const float *psi_scale, void *out, float *out_scale,
                            const grid_geom *geom, double M5, double mf, int prec, int link_fmt, void *stream);

/*
 * grid_mobius -- out = M_mob psi (M_mob^+ psi when op->dag) for op->kind = GRID_MOBIUS: one
 * s-local pass (chi = B psi; for the adjoint B^+ after the hop) and one hopping pass. tmp (and
 * tmp_scale for GRID_F16S) holds the intermediate field and must have psi's size. Same argument
 * rules as grid_dhop (Ls >= 1, every precision and link format). Asynchronous.
 */
int grid_mobius(const void *U, const void *psi, const float *psi_scale, void *out, float *out_scale, void *tmp,
                float *tmp_scale, const grid_geom *geom, const grid_op *op, int prec, int link_fmt, void *stream);

/*
 * grid_cg_workspace_bytes -- device workspace grid_cg needs for this geometry and parameters.
 * Returns 0 for invalid arguments.
 */
size_t grid_cg_workspace_bytes(const grid_geom *geom, const grid_cg_params *params);

/*
 * grid_cg -- solve Op^+ Op x = b by conjugate gradients (Section 4), Op = D (op->kind =
 * GRID_WILSON), M (GRID_DWF) or M_mob (GRID_MOBIUS), in FP64 or in mixed precision with reliable updates: sloppy
 * iterations in FP32 or FP16-storage with FP32 arithmetic, the solution, the source and each
 * recomputed true residual in FP64, inner products and norms accumulated in FP64.
 *
 *   U          FP64 links, L18 layout ([V][4][3][3] complex double)
 *   b          FP64 source; x FP64 initial guess on entry, solution on exit
 *   workspace  device buffer of at least grid_cg_workspace_bytes() bytes, 256-byte aligned
 *   stats      filled on return (also on GRID_ENOCONV / GRID_EBREAKDOWN)
 * Synchronous: returns when x is final. Stops when the FP64 true relative residual is <= tol.
 * Returns GRID_OK, GRID_ENOCONV, GRID_EBREAKDOWN or an argument / HIP error.
 */
int grid_cg(const void *U, const void *b, void *x, const grid_geom *geom, const grid_op *op,
            const grid_cg_params *params, void *workspace, size_t ws_bytes, grid_cg_stats *stats,
            void *stream);

/*
 * grid_dhop_backward -- adjoint of grid_dhop for L = Re <g, Op psi> (the gradient HMC's fermion
 * force is built from, Section 4). Gradients follow the complex convention dL/dRe + i dL/dIm.
 *
 *   grad_psi  (nullable) = Op^+ g, same layout as psi
 *   grad_U    (nullable) links [V][4][3][3] complex in precision prec:
 *             force_mode 0: dL/dU_mu(x) = c sum_{s,spin} { [(1 - e gamma_mu) g(x)] psi(x+mu)^+
 *                                              + psi(x) [(1 + e gamma_mu) g(x+mu)]^+ }
 *                            with c = 1 for GRID_HOP and -1/2 otherwise, e = +1 (dag: -1);
 *             force_mode 1: its projection onto su(3), TA(G U^+), TA(A) = (A - A^+)/2 -
 *                            tr(A - A^+)/6, so that d/de L(exp(e X) U)|0 = Re tr(F^+ X).
 * prec is GRID_F64 or GRID_F32 with GRID_L18 links. Returns as grid_dhop.
 */
int grid_dhop_backward(const void *U, const void *psi, const void *grad_out, void *grad_psi, void *grad_U,
                       const grid_geom *geom, const grid_op *op, int prec, int force_mode, void *stream);

/*
 * grid_convert_spinor -- change the storage precision of n_sites spinor sites (24 reals each):
 * F64 <-> F32, and F64/F32 -> F16S (encode, dst_scale receives per-site scales) or F16S ->
 * F64/F32 (decode with src_scale). Narrowing rounds to nearest even. (The Compressor of
 * Section 2.4 changes the precision of communicated fields; here it changes storage precision.)
 */
int grid_convert_spinor(const void *src, int src_prec, const float *src_scale, void *dst, int dst_prec,
                        float *dst_scale, long n_sites, void *stream);

/*
 * grid_convert_links -- convert n_links FP64 L18 links to precision dst_prec (F64, F32, or
 * F16S = half without scale) and format dst_fmt (L18 or L12). With reunitarise != 0 each link
 * is first projected back to SU(3) in FP64: row 0 normalised, row 1 Gram-Schmidt against row 0
 * and normalised, row 2 = conj(row0 x row1). Narrowing goes FP64 -> float (RNE) -> half (RNE).
 */
int grid_convert_links(const void *src, void *dst, int dst_prec, int dst_fmt, int reunitarise, long n_links,
                       void *stream);

/*
 * Even-odd (red-black) preconditioning. Grid objects may be single-checkerboard (Section 2.2):
 * a checkerboard field holds the sites of one parity p = (x + y + z + t) mod 2, site
 * (x, y, z, t) at index (x / 2) + (Lx/2)(y + Ly(z + Lz t)) -- the full index divided by two --
 * with the Ls records of a 4D site contiguous: [Lt][Lz][Ly][Lx/2][Ls][4][3]. Every extent must
 * be even (GRID_ESHAPE otherwise). Links stay full-lattice.
 *
 * grid_dhop_cb -- out = beta * H_{p,1-p} psi + Diag(y) on checkerboard p = out_parity, psi on
 * checkerboard 1 - p (H with H^+ when op->dag). Diag by op->kind: GRID_HOP none (y must be
 * NULL); GRID_WILSON (4 + mass) y (Ls must be 1); GRID_DWF the fifth-dimension part of M,
 * (5 - M5) y_s - P_- y~_{s+1} - P_+ y~_{s-1} (M^+: P_+ and P_- swapped). All three fields in
 * precision prec (scales for GRID_F16S), n = V Ls / 2 records each. Asynchronous.
 */
int grid_dhop_cb(const void *U, const void *psi, const float *psi_scale, const void *y, const float *y_scale,
                 void *out, float *out_scale, const grid_geom *geom, const grid_op *op, int out_parity,
                 double beta, int prec, int link_fmt, void *stream);

/*
 * grid_m5inv -- out = M5^-1 psi, M5 the fifth-dimension part of the domain-wall operator (as in
 * grid_dhop_cb), or (M5^+)^-1 psi when dag != 0, on n4 4D sites of Ls records each (a full or a
 * checkerboard field). Applied per site and chirality in closed form (cyclic bidiagonal
 * system); needs 1 <= Ls <= 64 and |5 - M5| > 1 for a stable recurrence. Asynchronous.
 */
int grid_m5inv(const void *psi, const float *psi_scale, void *out, float *out_scale, long n4, int Ls, double M5,
               double mf, int dag, int prec, void *stream);

/*
 * grid_solve_eo_workspace_bytes -- device workspace grid_solve_eo needs (0 for invalid input).
 */
size_t grid_solve_eo_workspace_bytes(const grid_geom *geom, const grid_cg_params *params);

/*
 * grid_solve_eo -- solve Op x = b (Op = D or M as in grid_cg; full-lattice FP64 fields) by CG on
 * the even-odd preconditioned normal equations Mhat^+ Mhat x_e = Mhat^+ bhat with
 *   Mhat = M_ee - M_eo M_oo^-1 M_oe,  bhat = b_e - M_eo M_oo^-1 b_o,
 *   x_o  = M_oo^-1 (b_o - M_oe x_e),
 * M_eo = M_oe = -H/2 between checkerboards and M_ee = M_oo = 4 + mass (Wilson) or the
 * fifth-dimension part M5 (domain wall). Moebius (GRID_MOBIUS, M = D_W B + 1 - S with
 * B = b5 + c5 S): M_eo = -H_eo B / 2, M_oe = -H_oe B / 2 and M_ee = M_oo = alpha - beta S,
 * alpha = 1 + (4 - M5) b5, beta = 1 - (4 - M5) c5; needs Ls <= 64 and |alpha / beta| > 1 (or
 * beta = 0, alpha != 0), GRID_EINVAL otherwise. Precision options as grid_cg (params). x on entry is
 * the initial guess (its even sites are used). The CG stops when the FP64 true residual of the
 * preconditioned normal equations is <= tol relative to |Mhat^+ bhat|; stats->true_residual is
 * then |b - Op x| / |b| of the full system, recomputed in FP64, and stats->converged reports the
 * CG criterion. Synchronous. Returns as grid_cg.
 */
int grid_solve_eo(const void *U, const void *b, void *x, const grid_geom *geom, const grid_op *op,
                  const grid_cg_params *params, void *workspace, size_t ws_bytes, grid_cg_stats *stats,
                  void *stream);

/*
 * Hybrid Monte Carlo molecular dynamics (HMC, Section 4), FP64, links [V][4][3][3].
 *   S_G = beta sum_{x, mu<nu} (1 - Re tr P_munu(x) / 3),
 *   P_munu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+;
 *   S_F = phi^+ (Op^+ Op)^-1 phi (two flavours, Op = D, the Shamir M or the Moebius M of
 *   `fermion`; the Moebius force is -2 G(M X, B X), X = (M^+ M)^-1 phi, as in
 *   grid_pseudofermion_action);
 *   forces F = TA(G U^+) with G = dS/dRe U + i dS/dIm U (as grid_dhop_backward);
 *   momenta P in su(3) per link ([V][4][3][3], anti-Hermitian traceless), K = sum tr(P^+ P);
 *   dU/dt = P U, dP/dt = -F/2, leapfrog: P -= (eps/2) F/2, then n_steps times
 *   { U <- exp(eps P) U; P -= eps F/2 } with the last momentum step halved; Omelyan (second-order
 *   minimum norm, l = 0.1931833275037836) per step: P -= l eps F/2; U <- exp(eps/2 P) U;
 *   P -= (1 - 2 l) eps F/2; U <- exp(eps/2 P) U; P -= l eps F/2; force gradient (fourth order;
 *   Omelyan, Mryglod and Folk's scheme with the force-gradient term taken, as Yin and Mawhinney
 *   do, as the force at displaced links) per step: P -= eps/6 F(U)/2; U <- exp(eps/2 P) U;
 *   P -= 2 eps/3 F(U')/2 with U' = exp(-(eps^2/24) F(U)/2) U; U <- exp(eps/2 P) U;
 *   P -= eps/6 F(U)/2.
 * Random momenta and pseudofermion sources are drawn by the caller.
 */
typedef struct {
    double beta;            /* Wilson gauge coupling                                            */
    double eps;             /* leapfrog step size                                               */
    int n_steps;            /* integrator steps (0: U and P unchanged)                          */
    grid_op fermion;        /* GRID_WILSON, GRID_DWF or GRID_MOBIUS pseudofermion operator
                               (phi != NULL)                                                     */
    grid_cg_params cg;      /* the solves inside every fermion-force evaluation                 */
    int integrator;         /* GRID_LEAPFROG, GRID_OMELYAN or GRID_FORCE_GRADIENT               */
    int n_inner;            /* > 1: two time scales (Sexton and Weingarten): the fermion force
                               kicks as in the outer integrator (leapfrog: P -= eps/2 F_F/2, gauge
                               integration over eps, P -= eps/2 F_F/2; Omelyan: P -= l eps F_F/2,
                               eps/2, P -= (1 - 2 l) eps F_F/2, eps/2, P -= l eps F_F/2; force
                               gradient: P -= eps/6 F_F/2, eps/2, P -= 2 eps/3 F_F(U')/2 with
                               U' = exp(-(eps^2/24) F_F(U)/2) U, eps/2, P -= eps/6 F_F/2), each
                               gauge integration over tau being n_inner leapfrog steps of
                               tau / n_inner with the gauge force alone; 0 or 1: the integrator
                               with the total force                                              */
} grid_md_params;

enum grid_integrator { GRID_LEAPFROG = 0, GRID_OMELYAN = 1, GRID_FORCE_GRADIENT = 2 };

typedef struct {
    int solves;             /* fermion solves performed                                         */
    int cg_iterations;      /* their total CG iterations                                        */
    int failed_solves;      /* solves that stopped short of cg.tol                              */
    double seconds;         /* wall time of the call                                            */
} grid_md_stats;

/* grid_md_workspace_bytes -- device workspace of grid_md_leapfrog / grid_hmc_energy (0: invalid). */
size_t grid_md_workspace_bytes(const grid_geom *geom, const grid_md_params *params);

/* grid_gauge_force -- F = the su(3) force of S_G on every link. Asynchronous. */
int grid_gauge_force(const void *U, void *F, const grid_geom *geom, double beta, void *stream);

/* grid_link_exp -- U <- exp(eps P) U on n_links links (P in su(3)), in place. Asynchronous. */
int grid_link_exp(void *U, const void *P, double eps, long n_links, void *stream);

/*
 * grid_md_leapfrog -- integrate (U, P) in place over n_steps steps of size eps with the integrator
 * params->integrator names (leapfrog, Omelyan or force gradient); phi
 * (FP64, the 4D or 5D pseudofermion of `fermion`) adds the fermion force, NULL integrates the pure
 * gauge system. Synchronous. Returns GRID_OK or an argument / HIP error; stats->failed_solves
 * counts force solves that did not reach cg.tol.
 */
int grid_md_leapfrog(void *U, void *P, const void *phi, const grid_geom *geom, const grid_md_params *params,
                     void *workspace, size_t ws_bytes, grid_md_stats *stats, void *stream);

/*
 * grid_hmc_energy -- energies[0..3] = K, S_G, S_F (0 when phi is NULL), H = K + S_G + S_F, in FP64.
 * Synchronous.
 */
int grid_hmc_energy(const void *U, const void *P, const void *phi, const grid_geom *geom,
                    const grid_md_params *params, void *workspace, size_t ws_bytes, double energies[4],
                    grid_md_stats *stats, void *stream);

/*
 * Two-flavour pseudofermion action (the fermion part of the HMC action, Section 4) with its
 * gradients, for callers that differentiate it (an autograd function, a force evaluation):
 *   X  = (Op^+ Op)^-1 phi by grid_cg with `params` (Op = D for GRID_WILSON, the Shamir M for
 *        GRID_DWF, the Moebius M for GRID_MOBIUS); X holds the initial guess on entry and the
 *        solution on exit;
 *   *S = Re <phi, X> = phi^+ (Op^+ Op)^-1 phi, an FP64 sum in a fixed order (S nullable);
 *   dS_dU   (nullable) = grad_scale * dS/dU, dS/dU = -2 G(g = Op X, psi = X) with G the link
 *           gradient of grid_dhop_backward (c = -1/2), i.e. the sum there with coefficient 1
 *           (Moebius: psi = B X, B = b5 + c5 S, since its link dependence is -H B / 2);
 *           force_mode 1 writes its su(3) projection TA(dS/dU U^+) instead;
 *   dS_dphi (nullable) = grad_scale * 2 X.
 * U, phi, X, dS_dphi FP64 ([V][4][3][3] / spinor layout); workspace >=
 * grid_pseudofermion_workspace_bytes(), 256-byte aligned; outputs must not overlap each other or
 * the inputs. Synchronous. Returns GRID_OK, GRID_ENOCONV (S and the gradients are still written,
 * from the unconverged X), GRID_EBREAKDOWN or an argument / HIP error.
 */
size_t grid_pseudofermion_workspace_bytes(const grid_geom *geom, const grid_cg_params *params);
int grid_pseudofermion_action(const void *U, const void *phi, void *X, const grid_geom *geom, const grid_op *op,
                              const grid_cg_params *params, double grad_scale, double *S, void *dS_dU, int force_mode,
                              void *dS_dphi, void *workspace, size_t ws_bytes, grid_cg_stats *stats, void *stream);

/*
 * Generic coarse stencil and two-level multigrid for the Wilson operator D (Section 2.4's stencil
 * example is the coarse-grid operator of an adaptive multigrid inverter; Section 4 lists
 * multigrid-preconditioned GCR). FP64 throughout.
 *
 *   aggregates   blocks of block[mu] fine sites; coarse extents Lc = L / block (periodic), coarse
 *                site index xc0 + Lc0 (xc1 + Lc1 (xc2 + Lc2 xc3));
 *   basis vecs   nvec fine fields [nvec][V][4][3] complex double; after grid_mg_basis they are
 *                orthonormal on every aggregate and chirality (spins 0,1 and 2,3);
 *   coarse field [Vc][N] complex double, N = 2 nvec, component n = chi nvec + k;
 *   R, P         (R psi)(xc)[chi nvec + k] = sum over the aggregate and the spins of chi of
 *                conj(phi_k) psi; (P v)(x) = sum_k phi_k(x)|chi v(xc)[chi nvec + k];
 *   coarse op    A_c = R D P as the 9-point stencil (A_c v)(xc) = sum_d A_d(xc) v(xc + e_d),
 *                d = 0 (self), 1 + 2 mu (+mu), 2 + 2 mu (-mu); hops of D from fine x in +mu
 *                with x_mu mod block[mu] = block[mu] - 1 (in -mu with x_mu mod block[mu] = 0)
 *                make A_{1+2mu} (A_{2+2mu}), all other terms A_0. Layout [Vc][9][N][N] with
 *                element (row i, column j) of A_d(xc) at [xc][d][j][i].
 */
typedef struct {
    int block[4];       /* aggregate extents (bx, by, bz, bt), each dividing the lattice extent  */
    int nvec;           /* basis vectors (1..32; N = 2 nvec coarse components per site)          */
    int setup_rounds;   /* grid_mg_basis: rounds of near-null improvement (0: orthonormalise)  */
    int setup_iters;    /* CG iterations on D^+ D per vector and round, from zero, then unit norm */
    int coarse_iters;   /* cap on the coarse CGNR iterations per cycle                           */
    double coarse_tol;  /* the coarse CGNR stops below coarse_tol times its starting residual    */
    int smooth_iters;   /* minimal-residual steps on D z = r after the coarse correction         */
    int restart;        /* GCR restart length (1..64)                                           */
    int maxiter;        /* cap on GCR iterations                                                */
    double tol;         /* target |b - D x| / |b|                                               */
    int graph;          /* nonzero: the coarse solve of a cycle is recorded once per grid_mg_solve
                           into a HIP graph and replayed (same kernels, same results)             */
    int setup_prec;     /* grid_mg_basis: precision of the setup CG's iterations, GRID_F64 (the
                           value of a zeroed struct) or GRID_F32 / GRID_F16S (mixed, as grid_cg) */
    int cycle_prec;     /* grid_mg_solve: GRID_F64 (zeroed struct) or GRID_F32: the cycle's minimal-
                           residual smoother in FP32 (FP32 links, FP64 inner products), and R, P
                           and the coarse solve reading FP32 copies of the basis and of A (FP64
                           arithmetic and coarse vectors); the GCR stays FP64                     */
} grid_mg_params;

/*
 * grid_coarse_stencil -- out = A v (dag: A^+ v, (A^+ v)(xc) = sum_d A_d(xc - e_d)^+ v(xc - e_d)) for
 * any 9-point stencil A in the layout above; coarse_dims = Lc (each >= 1), N in 1..64.
 * out must not overlap v. Asynchronous.
 */
int grid_coarse_stencil(const void *A, const void *v, void *out, const int coarse_dims[4], int N, int dag,
                        void *stream);

/* grid_mg_workspace_bytes -- device workspace of grid_mg_basis / grid_mg_coarse_op / grid_mg_solve. */
size_t grid_mg_workspace_bytes(const grid_geom *geom, const grid_mg_params *params);

/*
 * grid_mg_basis -- in place on vecs: setup_rounds times { every vector <- setup_iters CG iterations
 * on D^+ D x = vector from x = 0, normalised to 1 }, then Gram-Schmidt in the order k = 0, 1, ...
 * on every aggregate and chirality. The starting vectors (random) are the caller's. op: GRID_WILSON
 * (op->mass). Synchronous.
 */
int grid_mg_basis(const void *U, void *vecs, const grid_geom *geom, const grid_op *op, const grid_mg_params *params,
                  void *workspace, size_t ws_bytes, void *stream);

/* grid_mg_coarse_op -- A = R D P for the basis vecs (orthonormalised). Asynchronous. */
int grid_mg_coarse_op(const void *U, const void *vecs, void *A, const grid_geom *geom, const grid_op *op,
                      const grid_mg_params *params, void *workspace, size_t ws_bytes, void *stream);

/* grid_mg_restrict / grid_mg_prolong -- vc = R psi, psi = P vc. Asynchronous. */
int grid_mg_restrict(const void *vecs, const void *psi, void *vc, const grid_geom *geom, const grid_mg_params *params,
                     void *stream);
int grid_mg_prolong(const void *vecs, const void *vc, void *psi, const grid_geom *geom, const grid_mg_params *params,
                    void *stream);

/*
 * grid_mg_solve -- D x = b by flexible GCR(restart) preconditioned with one two-level cycle:
 * r_c = R r; CGNR on A_c from zero (A_c^+ = G5 A_c G5, G5 = +1 / -1 on the two chiralities) for
 * at most coarse_iters iterations, stopping below coarse_tol times the starting normal residual;
 * z = P e_c; smooth_iters minimal-residual steps on D z = r. The GCR orthogonalises w = D z by
 * modified Gram-Schmidt and recomputes r = b - D x at every restart and at the end. x holds the
 * initial guess on entry. stats: iterations (GCR), reliable_updates (restarts), true_residual,
 * converged, seconds. Synchronous. Returns GRID_OK, GRID_ENOCONV, GRID_EBREAKDOWN or an argument /
 * HIP error.
 */
int grid_mg_solve(const void *U, const void *vecs, const void *A, const void *b, void *x, const grid_geom *geom,
                  const grid_op *op, const grid_mg_params *params, void *workspace, size_t ws_bytes,
                  grid_cg_stats *stats, void *stream);

/*
 * grid_mg_pcg -- D x = b by multigrid-preconditioned CG (Section 4 lists multigrid pCG beside
 * pGCR): flexible CG on the Hermitian positive definite normal equations N x = D^+ b, N = D^+ D,
 * preconditioned with M(rho) = K(G5 K(G5 rho)), where K is grid_mg_solve's two-level cycle and
 * G5 = gamma5 on the fine field (D^+ = G5 D G5, so M approximates N^-1 = D^-1 D^-+; with no
 * smoothing and exact coarse solves M = P (A_c^+ A_c)^-1 R). The cycle's coefficients depend on its
 * input, so each direction p_k = z_k - sum_j (<N p_j, z_k> / <p_j, N p_j>) p_j is made N-conjugate
 * to the directions kept (at most params->restart, then the true residual is recomputed and the
 * directions dropped), alpha_k = <p_k, rho_k> / <p_k, N p_k> (flexible CG in Notay's form). It is
 * run as the loop of grid_mg_solve with z_k = M(D^+ r) in place of K(r): w = D z made orthogonal
 * to the kept w_j is D p_k, and alpha = <w, r> / |w|^2. Per iteration two cycles and three
 * applications of D or D^+. Parameters, workspace (grid_mg_workspace_bytes), stats, stopping rule
 * |b - D x| <= tol |b| and return codes as grid_mg_solve. Synchronous.
 */
int grid_mg_pcg(const void *U, const void *vecs, const void *A, const void *b, void *x, const grid_geom *geom,
                const grid_op *op, const grid_mg_params *params, void *workspace, size_t ws_bytes,
                grid_cg_stats *stats, void *stream);

/* grid_last_error -- message of the calling thread's last failed call ("" if none). */
const char *grid_last_error(void);

/* grid_version -- library version as major * 10000 + minor * 100 + patch. */
int grid_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GRID_MI_H */
