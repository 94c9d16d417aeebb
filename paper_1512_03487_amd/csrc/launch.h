// Internal launcher interface between the C ABI layer (abi.hip) and the kernel files.
// Host-side only: argument structs carry already-validated pointers and sizes.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "../../include/grid_mi.h"
#include "device.h"

namespace gridmi {

// Fused epilogue of the full-lattice Wilson / domain-wall operator, for the conjugate gradient:
//   kFuseNorm: out = op psi as usual, plus per-block partial sums of |out|^2;
//   kFuseAxpy: out = r - alpha op psi with alpha = scal[num] / scal[den] (device scalars), plus the
//              partials of |out|^2. r may be out itself (each site is read before it is written).
// The partials (FP16 storage: of the coded values) go to part[0 .. nblocks), nblocks the grid size.
enum { kFuseNone = 0, kFuseNorm = 1, kFuseAxpy = 2 };
struct FuseDev {
    const void *r = nullptr;
    const float *r_scale = nullptr;
    const double *scal = nullptr;
    int num = 0, den = 0;
    double *part = nullptr;
};

// Internal operator kinds of the checkerboard column walk (the even-odd Moebius Schur operator,
// B = b5 + c5 S; see k_dhop_walk_cb): kMobHop out = beta H B psi (dag: B^dagger beta H^dagger psi),
// kMobDiag adds diag y - cs S y (dag: diag y - cs S^dagger y). Full-lattice FP32 / FP16-storage
// checkerboard fields whose Ls divides 64 (mob_cb_applies).
enum { kMobHop = 8, kMobDiag = 9 };
// kHopInv: out = (diag - S)^-1 (beta H psi) ((diag - S^dagger)^-1 with dag), the even-odd domain-wall
// M5^-1 H_oe in one checkerboard walk (S as in M5, walls -mf); same field conditions.
enum { kHopInv = 10 };
// kMobHopInv: kMobHop followed by (diag - S)^-1 across the column (diag = alpha / beta), the
// Moebius M_oo^-1 up to its factor 1 / beta.
enum { kMobHopInv = 11 };
inline bool mob_cb_applies(int prec, int Ls) {
    return (prec == GRID_F32 || prec == GRID_F16S) && Ls >= 2 && 64 % Ls == 0;
}

struct DhopArgs {
    const void *U;
    const void *psi;
    const float *psi_scale;
    void *out;
    float *out_scale;
    GeomDev g;
    int prec;
    int link_fmt;
    int kind;
    int dag;
    double diag;   // 4 + mass (Wilson) or 5 - M5 (domain wall)
    double mf;
    hipStream_t stream;
    // Custom form: out = beta * H psi + the diagonal part of `kind` applied to y, its
    // fifth-dimension hopping scaled by cs; on checkerboard fields (the even-odd form) out is on
    // checkerboard cb and psi on 1 - cb, with cb = -1 on the full lattice (the Moebius operator).
    // With custom == false: full lattice, y = psi, beta = 1 (HOP) or -1/2 (WILSON, DWF), cs = 1.
    bool custom = false;
    int cb = -1;               // output checkerboard 0 / 1, or -1 for full-lattice fields
    const void *y = nullptr;
    const float *y_scale = nullptr;
    double beta = 0.0;
    double cs = 1.0;           // DWF epilogue: coefficient of the fifth-dimension hopping of y
    // kind GRID_MOBIUS (full lattice, walk_mobius_applies): the whole operator in one kernel, with
    // diag = 1 + (4 - M5) b5 and cs = 1 - (4 - M5) c5 (M), or diag = 4 - M5 (M^dagger)
    double b5 = 1.0, c5 = 0.0;
    // Fused epilogue (kind WILSON or DWF; full lattice or the custom even-odd form): kFuseNorm
    // with dag = 0, kFuseAxpy with dag = 1.
    int fuse = kFuseNone;
    FuseDev fz;
};

hipError_t launch_dhop(const DhopArgs &a);
// The calling host thread's stream for recording HIP graphs on the current device (kept for the
// life of the process; cg.hip).
hipError_t capture_stream(hipStream_t *s);
bool walk_mobius_applies(const DhopArgs &a);
// Tiled time-walk schedule (tile.hip): full-lattice 4D FP32 / FP16-storage fields whose x, y, z
// extents the tile divides.
bool tile_applies(const DhopArgs &a);
long tile_blocks(const DhopArgs &a);
hipError_t launch_tile(const DhopArgs &a);
// Number of blocks (= partial sums written by a fused epilogue) launch_dhop uses for `a`.
long dhop_blocks(const DhopArgs &a);
// Upper bound of dhop_blocks over all schedules for a field of n5 sites and time extent Lt.
long dhop_blocks_max(long n5, int Lt);

// Moebius domain-wall operator (mobius.hip): out = M_mob psi (dag: M_mob^dagger psi) through the
// intermediate field tmp (same size and precision as psi). a.diag is unused; M5, b5, c5 given.
// a.fuse (kFuseNorm with dag = 0, kFuseAxpy with dag = 1) applies to the last kernel, whose
// partial count goes to *nparts.
hipError_t launch_mobius(const DhopArgs &a, double M5, double b5, double c5, void *tmp, float *tmp_scale,
                         long *nparts = nullptr);
// Upper bound of the partial sums any fused epilogue writes for n5 sites (hopping or s-local kernel).
long fused_parts_max(long n5, int Lt);
// The s-local pass (mobius.hip): out = a1 u + a2 S u + a3 v + a4 S v (S^dagger when dag) on n5 5D
// sites of Ls records (full or checkerboard fields); v may be NULL. fuse: kFuseNone or kFuseAxpy
// (out = r - alpha (...), partials of |out|^2 in s5_blocks(n5) blocks).
hipError_t launch_s5axpy(int prec, const void *u, const float *us, const void *v, const float *vs, void *out,
                         float *outs, long n5, int Ls, double a1, double a2, double a3, double a4, double mf, int dag,
                         hipStream_t st, int fuse = kFuseNone, const FuseDev &fz = FuseDev());
long s5_blocks(long n5);

// Fifth-dimension operator inverse of the domain-wall operator (eo.hip): out = M5^-1 psi or
// (M5^dagger)^-1 psi on n4 4D sites of Ls records each (full or checkerboard fields).
hipError_t launch_m5inv(const void *psi, const float *psi_scale, void *out, float *out_scale, long n4, int Ls,
                        double diag, double mf, int dag, int prec, hipStream_t stream);

// Even-odd solve of M x = b (eo.hip).
size_t solve_eo_workspace_bytes(const GeomDev &g, int sloppy, int link_fmt);
// op: GRID_WILSON (mass), GRID_DWF (M5, mf) or GRID_MOBIUS (M5, mf, b5, c5).
hipError_t run_solve_eo(const void *U, const void *b, void *x, const GeomDev &g, const grid_op &op,
                        const grid_cg_params &p, void *ws, hipStream_t st, grid_cg_stats *stats, int *status);

// Link gradient / force of the hopping term (backward.hip).
struct LinkGradArgs {
    const void *U;          // links (force mode only), L18 in precision prec
    const void *chi;        // upstream gradient g
    const void *psi;
    void *G;                // [V][4][3][3] complex, precision prec
    GeomDev g;
    int prec;               // GRID_F64 or GRID_F32
    int dag;
    int force_mode;
    double coef;
    hipStream_t stream;
};
hipError_t launch_link_grad(const LinkGradArgs &a);

// Codecs (codec.hip).
hipError_t launch_convert_spinor(const void *src, int src_prec, const float *src_scale, void *dst, int dst_prec,
                                 float *dst_scale, long n_sites, hipStream_t stream);
hipError_t launch_convert_links(const void *src, void *dst, int dst_prec, int dst_fmt, int reunitarise, long n_links,
                                hipStream_t stream);

// Conjugate gradient on A = op^dagger op (cg.hip). The operator is applied in the precision and
// link format asked for (GRID_F64 / GRID_L18 for true residuals, the sloppy ones in iterations).
struct CgOp {
    hipError_t (*apply)(const void *ctx, const void *U, int prec, int fmt, const void *in, const float *ins, void *out,
                        float *outs, int dag, hipStream_t st);
    const void *ctx;
    // Apply with a fused epilogue (kFuseNorm with dag 0, kFuseAxpy with dag 1), setting *nparts
    // to the number of partial sums written; the conjugate gradient needs it.
    hipError_t (*apply_fused)(const void *ctx, const void *U, int prec, int fmt, const void *in, const float *ins,
                              void *out, float *outs, int dag, int fuse, const FuseDev &fz, long *nparts,
                              hipStream_t st) = nullptr;
};
size_t cg_workspace_bytes(const GeomDev &g, int sloppy, int link_fmt);
size_t cg_workspace_bytes_n(long nsites, long nlinks, int sloppy, int link_fmt, long nparts);
hipError_t run_cg(const void *U, const void *b, void *x, const GeomDev &g, const grid_op &op, const grid_cg_params &p,
                  void *ws, hipStream_t st, grid_cg_stats *stats, int *status);
// op_tmp: the workspace was sized with the operator temporaries (cg_workspace_bytes) or not
// (cg_workspace_bytes_n); nparts: the room for fused-epilogue partials it was sized with
// (fused_parts_max).
hipError_t run_cg_op(const CgOp &op, const void *U, const void *b, void *x, long nsites, long nlinks,
                     const grid_cg_params &p, void *ws, hipStream_t st, grid_cg_stats *stats, int *status,
                     bool op_tmp, long nparts);
// ||a - b||^2 over n FP64 spinor sites (b may be NULL); part: kRedBlocks + 16 doubles of scratch.
constexpr int kNormScratch = 1024 + 16;
hipError_t norm2_diff(const void *a, const void *b, long n, double *part, hipStream_t st, double *result);
// Re <a, b> over n FP64 spinor sites, deterministic; waits for the stream.
hipError_t dot_re(const void *a, const void *b, long n, double *part, hipStream_t st, double *result);

// Hybrid Monte Carlo (hmc.hip).
hipError_t launch_gauge_force(const void *U, void *F, const GeomDev &g, double beta, double scale, int accumulate,
                              hipStream_t st);
hipError_t launch_link_exp(void *U, const void *P, double eps, long nlinks, hipStream_t st);
size_t md_workspace_bytes(const GeomDev &g, const grid_md_params &p);
hipError_t run_md_leapfrog(void *U, void *P, const void *phi, const GeomDev &g, const grid_md_params &p, void *ws,
                           hipStream_t st, grid_md_stats *stats);
hipError_t run_hmc_energy(const void *U, const void *P, const void *phi, const GeomDev &g, const grid_md_params &p,
                          void *ws, hipStream_t st, double energies[4], grid_md_stats *stats);

// Two-flavour pseudofermion action and gradients (hmc.hip); arguments validated. X: initial guess
// on entry, the solution on exit; S, dS_dU, dS_dphi nullable.
size_t pf_workspace_bytes(const GeomDev &g, const grid_cg_params &p);
hipError_t run_pseudofermion(const void *U, const void *phi, void *X, const GeomDev &g, const grid_op &op,
                             const grid_cg_params &p, double grad_scale, double *S, void *dS_dU, int force_mode,
                             void *dS_dphi, void *ws, hipStream_t st, grid_cg_stats *stats, int *status);

// Coarse stencil and two-level multigrid for the Wilson operator (mg.hip); arguments validated.
hipError_t launch_coarse_stencil(const void *A, const void *v, void *out, const int Lc[4], int N, int dag,
                                 hipStream_t st);
size_t mg_workspace_bytes(const GeomDev &g, const grid_mg_params &p);
hipError_t run_mg_basis(const void *U, void *vecs, const GeomDev &g, double mass, const grid_mg_params &p, void *ws,
                        hipStream_t st);
hipError_t run_mg_coarse_op(const void *U, const void *vecs, void *A, const GeomDev &g, double mass,
                            const grid_mg_params &p, void *ws, hipStream_t st);
hipError_t launch_mg_restrict(const void *vecs, const void *psi, void *vc, const GeomDev &g, const grid_mg_params &p,
                              hipStream_t st);
hipError_t launch_mg_prolong(const void *vecs, const void *vc, void *psi, const GeomDev &g, const grid_mg_params &p,
                             hipStream_t st);
hipError_t run_mg_solve(const void *U, const void *vecs, const void *A, const void *b, void *x, const GeomDev &g,
                        double mass, const grid_mg_params &p, void *ws, hipStream_t st, grid_cg_stats *stats,
                        int *status, bool pcg);

}  // namespace gridmi
