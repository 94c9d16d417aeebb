// Internal launcher interface between the C ABI layer (abi.hip) and the kernel files.
// Host-side only: argument structs carry already-validated pointers and sizes.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "../../include/grid_mi.h"
#include "device.h"

namespace gridmi {

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
};

hipError_t launch_dhop(const DhopArgs &a);

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

// Conjugate gradient (cg.hip).
size_t cg_workspace_bytes(const GeomDev &g, int sloppy, int link_fmt);
hipError_t run_cg(const void *U, const void *b, void *x, const GeomDev &g, int kind, double diag, double mf,
                  const grid_cg_params &p, void *ws, hipStream_t st, grid_cg_stats *stats, int *status);

}  // namespace gridmi
