// Internal: table construction (tables.hip).
#pragma once
#include "common.h"

namespace elph {

elph_status make_axis_tables(elph_ctx ctx);
elph_status build_tables(elph_ctx ctx);
// eigenvalues (ascending, may be NULL) and eigenvectors (columns, may be NULL)
// of nmat Hermitian n x n matrices stored row-major back to back
void launch_jacobi(const cd* A, int64_t nmat, int n, double* evals, cd* evecs, hipStream_t s);
// Fourier sum (Eq. 1 electrons, Eq. 3 phonons) at a device list of mesh points
elph_status fourier_points(elph_ctx ctx, bool phonon, const int32_t* pts, int64_t npts, cd* out);
// Eq. 7 without its electron overlap, F_s(q) [npts][nbr], at the mesh points
// pts (all points when pts is null) from their phonon factors Lq [npts][nbr][nbr]
void launch_frohlich(elph_ctx ctx, const int32_t* pts, int64_t npts, const cd* Lq, cd* F, hipStream_t s);
void scan_exclusive(elph_ctx ctx, const int32_t* in, int64_t n, int32_t* out, int32_t* out_total,
                    int32_t* scratch, hipStream_t s);

}  // namespace elph
