// Host-side validation of lbib parameters and cell sets.  Pure C++ (no HIP calls), so the
// rules can be exercised on a machine without a GPU.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "lbib.h"

namespace lbib {

static lbib_status fail(std::string& msg, const char* fmt, double a = 0, double b = 0, double c = 0)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, fmt, a, b, c);
    msg = buf;
    return LBIB_EINVAL;
}

lbib_status check_params(const lbib_params* p, std::string& msg)
{
    if (!p) return fail(msg, "params is NULL");
    if (p->nx < 4 || p->nx > 32767 || p->ny < 4 || p->ny > 32767)
        return fail(msg, "lattice %g x %g outside 4..32767", p->nx, p->ny);
    if (p->bc_y != LBIB_PERIODIC && p->bc_y != LBIB_WALLS) return fail(msg, "bc_y %g unknown", p->bc_y);
    if (p->delta_kernel != LBIB_DELTA_COS4 && p->delta_kernel != LBIB_DELTA_PESKIN4)
        return fail(msg, "delta_kernel %g unknown", p->delta_kernel);
    if (!std::isfinite(p->tau) || !(p->tau > 0.5)) return fail(msg, "tau = %g must exceed 1/2", p->tau);
    if (!std::isfinite(p->rho0) || !(p->rho0 > 0.0)) return fail(msg, "rho0 = %g must be positive", p->rho0);
    if (!std::isfinite(p->body_accel[0]) || !std::isfinite(p->body_accel[1]))
        return fail(msg, "body_accel not finite");
    if (!std::isfinite(p->k_spring) || !std::isfinite(p->phi_m) || !std::isfinite(p->kappa_area))
        return fail(msg, "force-law constants not finite");
    if (!std::isfinite(p->mass_source) || !std::isfinite(p->area_alpha) || !std::isfinite(p->mass_phi_gamma))
        return fail(msg, "mass-source constants not finite");
    if (p->area_alpha < 0.0) return fail(msg, "area_alpha = %g must not be negative", p->area_alpha);
    if (p->pressure_ring != 0 && p->pressure_ring != 1)
        return fail(msg, "pressure_ring = %g must be 0 or 1", p->pressure_ring);
    if (p->interp_half_force != 0 && p->interp_half_force != 1)
        return fail(msg, "interp_half_force = %g must be 0 or 1", p->interp_half_force);
    if (p->no_flux_zeroth != 0 && p->no_flux_zeroth != 1)
        return fail(msg, "no_flux_zeroth = %g must be 0 or 1", p->no_flux_zeroth);
    if (p->no_flux_bounce != 0 && p->no_flux_bounce != 1)
        return fail(msg, "no_flux_bounce = %g must be 0 or 1", p->no_flux_bounce);
    if (p->no_flux_bounce && p->no_flux_zeroth)
        return fail(msg, "no_flux_bounce works on the first-order form's cut links (no_flux_zeroth = 0)");
    if (p->monitor_every < 0 || p->monitor_every % LBIB_GRAPH_STEPS != 0 || p->monitor_every > (1 << 30))
        return fail(msg, "monitor_every = %g must be 0 or a positive multiple of 16", p->monitor_every);
    if (p->reserved != 0) return fail(msg, "reserved = %g must be 0", p->reserved);
    if (p->n_species < 0 || p->n_species > 2) return fail(msg, "n_species = %g outside 0..2", p->n_species);
    if (p->storage < LBIB_STORAGE_FP32 || p->storage > LBIB_STORAGE_BF16)
        return fail(msg, "storage %g unknown", p->storage);
    if (p->mass_phi_gamma != 0.0 && p->n_species < 1)
        return fail(msg, "mass_phi_gamma needs a species (its source reads species 0)");
    int n_sch = 0;
    for (int s = 0; s < p->n_species; ++s) {
        const lbib_species& sp = p->species[s];
        if (!std::isfinite(sp.D) || !(sp.D > 0.0)) return fail(msg, "species %g: D = %g must be positive", s, sp.D);
        if (!std::isfinite(sp.phi_ref)) return fail(msg, "species %g: phi_ref not finite", s);
        if (sp.flags & ~LBIB_SPECIES_NO_FLUX) return fail(msg, "species %g: unknown flags", s);
        for (int k = 0; k < 4; ++k)
            if (!std::isfinite(sp.c[k])) return fail(msg, "species %g: reaction constant %g not finite", s, k);
        if (sp.reaction < LBIB_REACT_NONE || sp.reaction > LBIB_REACT_SCHNAKENBERG)
            return fail(msg, "species %g: reaction %g unknown", s, sp.reaction);
        if (sp.reaction == LBIB_REACT_SCHNAKENBERG) ++n_sch;
    }
    if (n_sch) {
        if (p->n_species != 2 || n_sch != 2)
            return fail(msg, "Schnakenberg kinetics need two species that both name it");
        for (int k = 0; k < 3; ++k)
            if (p->species[0].c[k] != p->species[1].c[k])
                return fail(msg, "Schnakenberg constants c[%g] differ between the species", k);
    }
    return LBIB_OK;
}

lbib_status check_cells(const lbib_params* p, int32_t n_cells, const int32_t* off, const double* xy,
                        const double* rest_len, const double* rest_area, std::string& msg)
{
    if (n_cells < 0 || n_cells > 65535) return fail(msg, "n_cells = %g outside 0..65535", n_cells);
    if (n_cells == 0) return LBIB_OK;
    if (!off || !xy) return fail(msg, "offsets or xy is NULL");
    if (off[0] != 0) return fail(msg, "offsets[0] = %g, expected 0", off[0]);
    for (int32_t c = 0; c < n_cells; ++c) {
        const long long n = (long long)off[c + 1] - off[c];
        if (n < 3) return fail(msg, "cell %g has %g nodes (need >= 3)", c, (double)n);
        if (n > 4096) return fail(msg, "cell %g has %g nodes (limit 4096)", c, (double)n);
    }
    const long long N = off[n_cells];
    if (N > 200000000LL) return fail(msg, "%g nodes in total (limit 2e8)", (double)N);
    for (long long i = 0; i < 2 * N; ++i)
        if (!std::isfinite(xy[i]) || std::fabs(xy[i]) >= 1048576.0)
            return fail(msg, "node coordinate %g not finite or beyond 2^20", (double)(i / 2));
    if (rest_len)
        for (long long i = 0; i < N; ++i)
            if (!std::isfinite(rest_len[i]) || rest_len[i] < 0.0)
                return fail(msg, "rest length of edge %g invalid", (double)i);
    if (rest_area)
        for (int32_t c = 0; c < n_cells; ++c)
            if (!std::isfinite(rest_area[c])) return fail(msg, "rest area of cell %g not finite", c);
    for (int32_t c = 0; c < n_cells; ++c) {
        const long long a = off[c], n = off[c + 1] - off[c];
        double A = 0.0, xmin = xy[2 * a], xmax = xmin, ymin = xy[2 * a + 1], ymax = ymin;
        for (long long k = 0; k < n; ++k) {
            const long long i = a + k, j = a + (k + 1) % n;
            A += (xy[2 * i] - xy[2 * a]) * (xy[2 * j + 1] - xy[2 * a + 1]) -
                 (xy[2 * j] - xy[2 * a]) * (xy[2 * i + 1] - xy[2 * a + 1]);
            xmin = std::fmin(xmin, xy[2 * i]);
            xmax = std::fmax(xmax, xy[2 * i]);
            ymin = std::fmin(ymin, xy[2 * i + 1]);
            ymax = std::fmax(ymax, xy[2 * i + 1]);
        }
        if (!(A > 0.0)) return fail(msg, "cell %g is not counter-clockwise (signed area %g)", c, 0.5 * A);
        if (xmax - xmin >= p->nx - 4) return fail(msg, "cell %g spans %g >= nx - 4 in x", c, xmax - xmin);
        if (ymax - ymin >= p->ny - 4) return fail(msg, "cell %g spans %g >= ny - 4 in y", c, ymax - ymin);
        if (p->bc_y == LBIB_WALLS && (ymin < 1.5 || ymax > p->ny - 2.5))
            return fail(msg, "cell %g has a node within 2 lattice units of a wall (y in [%g, %g])", c, ymin, ymax);
    }
    return LBIB_OK;
}

}  // namespace lbib

static void copy_msg(const std::string& m, char* msg, size_t len)
{
    if (!msg || len == 0) return;
    std::snprintf(msg, len, "%s", m.c_str());
}

extern "C" lbib_status lbib_validate_params(const lbib_params* p, char* msg, size_t msg_len)
{
    std::string m;
    lbib_status s = lbib::check_params(p, m);
    copy_msg(m, msg, msg_len);
    return s;
}

extern "C" lbib_status lbib_validate_cells(const lbib_params* p, int32_t n_cells, const int32_t* offsets,
                                           const double* xy, const double* rest_len, const double* rest_area,
                                           char* msg, size_t msg_len)
{
    std::string m;
    lbib_status s = lbib::check_params(p, m);
    if (s == LBIB_OK) s = lbib::check_cells(p, n_cells, offsets, xy, rest_len, rest_area, m);
    copy_msg(m, msg, msg_len);
    return s;
}
