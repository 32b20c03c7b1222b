// Synthetic radiotherapy dose-influence matrix, row by row (voxels are rows,
// beamlets are columns).  Input synthesis only: shared by both sides of the
// parity tests, holds none of the solver's arithmetic.
//
// Model (the same as workloads.rt in Python): voxel centres of an X*Y*Z grid
// with unit spacing, centred at the origin; n_beams coplanar beams at equal
// angular steps around the z axis, the first at angle0; each beam a grid of nbu x nbw beamlets with
// the given spacing.  For voxel p and beamlet (b, bu, bw):
//   depth = p . e_d + half,  u = p . e_u,  w = p_z,
//   fu = u/spacing + (nbu-1)/2,  fw = w/spacing + (nbw-1)/2,
//   r = spacing * hypot(fu - bu, fw - bw),
//   a = exp(-mu * max(depth, 0)) * exp(-r / rho)   if r <= r_cut.
// Candidate beamlets are the (2*reach+1)^2 around the nearest one, in beam
// order, then du, then dw (the column order inside a row).
#include <cmath>
#include <cstdint>
#include <vector>

struct RtParams {
    int32_t X, Y, Z;
    int32_t n_beams, nbu, nbw;
    double spacing, mu, rho, r_cut;
    double angle0; // angle of the first beam (radians)
};

namespace {

inline void voxel_center(const RtParams &P, int64_t v, double &px, double &py, double &pz)
{
    const int64_t k = v % P.Z, j = (v / P.Z) % P.Y, i = v / ((int64_t)P.Y * P.Z);
    px = (i + 0.5) - P.X / 2.0;
    py = (j + 0.5) - P.Y / 2.0;
    pz = (k + 0.5) - P.Z / 2.0;
}

template <class Emit>
inline void row_entries(const RtParams &P, int64_t v, Emit emit)
{
    double px, py, pz;
    voxel_center(P, v, px, py, pz);
    const double half = 0.5 * (P.X > P.Y ? P.X : P.Y);
    const int reach = (int)std::ceil(P.r_cut / P.spacing) + 1;
    for (int b = 0; b < P.n_beams; ++b) {
        const double th = P.angle0 + 2.0 * M_PI * b / P.n_beams;
        const double ed0 = std::cos(th), ed1 = std::sin(th);
        const double eu0 = -std::sin(th), eu1 = std::cos(th);
        const double depth = px * ed0 + py * ed1 + half;
        const double u = px * eu0 + py * eu1, w = pz;
        const double fu = u / P.spacing + (P.nbu - 1) / 2.0;
        const double fw = w / P.spacing + (P.nbw - 1) / 2.0;
        const int64_t bu0 = (int64_t)std::nearbyint(fu), bw0 = (int64_t)std::nearbyint(fw);
        const double att = std::exp(-P.mu * (depth > 0.0 ? depth : 0.0));
        for (int du = -reach; du <= reach; ++du)
            for (int dw = -reach; dw <= reach; ++dw) {
                const int64_t bu = bu0 + du, bw = bw0 + dw;
                if (bu < 0 || bu >= P.nbu || bw < 0 || bw >= P.nbw) continue;
                const double r = P.spacing * std::hypot(fu - (double)bu, fw - (double)bw);
                if (!(r <= P.r_cut)) continue;
                emit((int32_t)(b * P.nbu * P.nbw + bu * P.nbw + bw), att * std::exp(-r / P.rho));
            }
    }
}

} // namespace

extern "C" {

// Entries of every voxel row.
void rt_count(const RtParams *P, int64_t *counts)
{
    const int64_t nv = (int64_t)P->X * P->Y * P->Z;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < nv; ++v) {
        int64_t c = 0;
        row_entries(*P, v, [&](int32_t, double) { ++c; });
        counts[v] = c;
    }
}

// Columns and unscaled values of every voxel row at row_ptr[v].
void rt_fill(const RtParams *P, const int64_t *row_ptr, int32_t *cols, double *vals)
{
    const int64_t nv = (int64_t)P->X * P->Y * P->Z;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < nv; ++v) {
        int64_t q = row_ptr[v];
        row_entries(*P, v, [&](int32_t c, double a) {
            cols[q] = c;
            vals[q] = a;
            ++q;
        });
    }
}

} // extern "C"
