"""Planted mistakes: each plausible error in the oracle (a flipped sign, a
dropped term, a swapped operand) must make at least one pin fail.  The
mistakes are planted in a temporary copy of oracle.c compiled on the CPU.

Not pinned: the HLLC wave-speed estimate (the paper does not state it; the
Davis bounds are a reading), so a change there is only caught by parity.

Not a mistake: reversing the wall ghost's tangential velocity.  The wall's
Riemann problem is symmetric, so its contact speed is exactly zero and both
solvers take the tangential velocity from the cell's side only; the flux is
the same either way."""
import os

import pytest

import oracle
import oracle_pins as pins

SRC = open(oracle.SRC_PATH).read()

# (name, original text, planted text, pins expected to catch it)
MUTATIONS = [
    ("gradient r_ij reversed",
     "double rx = m->px[i] - v.rx, ry = m->py[i] - v.ry;",
     "double rx = v.rx - m->px[i], ry = v.ry - m->py[i];",
     [pins.gradient_linear]),
    ("gradient c_ij term dropped",
     "g[2 * q] += v.L * (dphi * cx / r - mean * rx / r);",
     "g[2 * q] += v.L * (0.0 * cx / r - mean * rx / r);",
     [pins.gradient_linear]),
    ("gradient x/y swapped in c_ij",
     "g[2 * q + 1] += v.L * (dphi * cy / r - mean * ry / r);",
     "g[2 * q + 1] += v.L * (dphi * cx / r - mean * ry / r);",
     [pins.gradient_linear]),
    ("periodic shift sign on the far side",
     "v->rx = m->px[j] - shx;",
     "v->rx = m->px[j] + shx;",
     [pins.gradient_periodic, pins.uniform_flow]),
    ("global limiter uses the minimum for increases",
     "psi = (pmax[q] - phi_i[q]) / dphi;",
     "psi = (pmin[q] - phi_i[q]) / dphi;",
     [pins.tvd_example, pins.limiter_bounds]),
    ("local limiter without theta",
     "psi = (dphi != 0.0) ? fmax(p->theta * (phi_j[q] - phi_i[q]) / dphi, 0.0) : 1.0;",
     "psi = (dphi != 0.0) ? fmax((phi_j[q] - phi_i[q]) / dphi, 0.0) : 1.0;",
     [pins.tvd_example, pins.limiter_bounds]),
    ("per-cell acceleration: components swapped",
     "      gx += ax[i];\n      gy += ay[i];",
     "      gx += ay[i];\n      gy += ax[i];",
     [pins.accel_field]),
    ("per-cell acceleration: ignored",
     "    if (ax) {\n      gx += ax[i];",
     "    if (ax && 0) {\n      gx += ax[i];",
     [pins.accel_field]),
    ("edge waves: star pressure reported for u*",
     "      ss = star[1];",
     "      ss = star[0];",
     [pins.edge_waves_uniform]),
    ("HLLC contact speed: pressure difference reversed",
     "*ss = (pr - pl + rl * ul * (*sl - ul) - rr * ur * (*sr - ur)) /",
     "*ss = (pl - pr + rl * ul * (*sl - ul) - rr * ur * (*sr - ur)) /",
     [pins.hllc_weak_waves]),
    ("HLLC star pressure sign",
     "double ps = pk + rho * (sk - u) * (ss - u);",
     "double ps = pk - rho * (sk - u) * (ss - u);",
     [pins.hllc_cases, pins.hllc_weak_waves]),
    ("exact solver shock branch: wrong B_K",
     "double A = 2.0 / ((g + 1.0) * rk), B = (g - 1.0) / (g + 1.0) * pk;",
     "double A = 2.0 / ((g + 1.0) * rk), B = (g + 1.0) / (g - 1.0) * pk;",
     [pins.exact_shock_tube, pins.exact_two_shocks]),
    ("exact solver fan: wrong density exponent",
     "W[0] = rl * pow(c / cl, g4);",
     "W[0] = rl * pow(c / cl, g3);",
     [pins.exact_shock_tube]),
    ("edge velocity: (w_j - w_i) instead of (w_i - w_j)",
     "double a = ((wix - wjx) * cx + (wiy - wjy) * cy) / d;",
     "double a = ((wjx - wix) * cx + (wjy - wiy) * cy) / d;",
     [pins.uniform_state_moving]),
    ("momentum flux not boosted back",
     "flux[ne + e] = fpx + F[0] * wex;",
     "flux[ne + e] = fpx;",
     [pins.uniform_state_moving, pins.galilean]),
    ("energy flux misses the kinetic term of the edge motion",
     "flux[3 * ne + e] = F[3] + fpx * wex + fpy * wey + 0.5 * (wex * wex + wey * wey) * F[0];",
     "flux[3 * ne + e] = F[3] + fpx * wex + fpy * wey;",
     [pins.uniform_state_moving, pins.galilean]),
    ("update sign per side reversed",
     "double sgn = (m->idx[k] & 1) ? -1.0 : 1.0;",
     "double sgn = (m->idx[k] & 1) ? 1.0 : -1.0;",
     [pins.uniform_state_moving, pins.sod_accuracy]),
    ("wall ghost does not reverse the normal velocity",
     "WR[0] = phiL[0]; WR[1] = -WL[1];",
     "WR[0] = phiL[0]; WR[1] = WL[1];",
     [pins.conservation]),
    ("wall ghost does not reverse the normal velocity (images)",
     "WR[0] = phiL[0]; WR[1] = -WL[1];",
     "WR[0] = phiL[0]; WR[1] = WL[1];",
     [pins.wall_images]),
    ("wall ghost state taken at the cell centre (not extrapolated)",
     "    WR[0] = phiL[0]; WR[1] = -WL[1]; WR[2] = WL[2]; WR[3] = phiL[3];",
     "    WR[0] = prim[i]; WR[1] = -WL[1]; WR[2] = WL[2]; WR[3] = prim[3 * n + i];",
     [pins.wall_images]),
    ("wall ghost gradient not mirrored (ghost extrapolated from the mirrored centroid)",
     "    WR[0] = phiL[0]; WR[1] = -WL[1]; WR[2] = WL[2]; WR[3] = phiL[3];",
     "    { double smx, smy, g[4];\n"
     "      mirror_point(m, code, m->sx[i], m->sy[i], &smx, &smy);\n"
     "      face_state(prim, lgrad, n, i, fx - smx, fy - smy, g);\n"
     "      WR[0] = g[0]; WR[1] = -WL[1]; WR[2] = WL[2]; WR[3] = g[3]; }",
     [pins.wall_images]),
    ("wall edge moves with the cell's normal velocity",
     "    wex = w[i] - wn * nx;\n    wey = w[n + i] - wn * ny;",
     "    wex = w[i];\n    wey = w[n + i];",
     [pins.wall_images]),
    ("wall ghost in the gradient keeps the cell's velocity (not mirrored)",
     "    mirror_vec(v->wall, prim[1 * n + i], prim[2 * n + i], &phi[1], &phi[2]);",
     "    phi[1] = prim[1 * n + i]; phi[2] = prim[2 * n + i];",
     [pins.wall_images]),
    ("rounding correction points away from the centroid",
     "double dx = m->sx[i] - m->px[i], dy = m->sy[i] - m->py[i];\n    double d = sqrt(dx * dx + dy * dy);\n    double R = sqrt(m->area[i] / OR_PI);\n    if (d > p->eta * R) {",
     "double dx = m->px[i] - m->sx[i], dy = m->py[i] - m->sy[i];\n    double d = sqrt(dx * dx + dy * dy);\n    double R = sqrt(m->area[i] / OR_PI);\n    if (d > p->eta * R) {",
     [pins.point_velocity]),
    ("shock detector ignores compression",
     "int shock = (-(G[2] + G[5]) > p->delta_v * ci / R);",
     "int shock = 0;",
     [pins.shock_detector]),
    ("shock detector: pressure ratio test inverted",
     "if (p->delta_p > ratio) shock = 1;",
     "if (p->delta_p < ratio) shock = 1;",
     [pins.shock_detector]),
    ("acceleration source taken from the base state",
     "double sm = Qsrc[i], spx = Qsrc[n + i], spy = Qsrc[2 * n + i];",
     "double sm = Qbase[i], spx = Qbase[n + i], spy = Qbase[2 * n + i];",
     [pins.free_fall, pins.accel_field]),
    ("work of the external acceleration dropped",
     "Qout[3 * n + i] += h * (spx * gx + spy * gy);",
     "Qout[3 * n + i] += 0.0 * h * (spx * gx + spy * gy);",
     [pins.free_fall, pins.accel_field]),
    ("extrapolated fluxes: advection of the density reversed",
     "double rho_t = -(ux * drx + uy * dry) - rho * div;",
     "double rho_t = +(ux * drx + uy * dry) - rho * div;",
     [pins.extrapolated_second_order]),
    ("extrapolated fluxes: compression term of the density dropped",
     "double rho_t = -(ux * drx + uy * dry) - rho * div;",
     "double rho_t = -(ux * drx + uy * dry);",
     [pins.extrapolated_second_order]),
    ("extrapolated fluxes: pressure gradient missing from the velocity",
     "double vx_t = -(ux * dvxx + uy * dvxy) - dpx / rho;",
     "double vx_t = -(ux * dvxx + uy * dvxy);",
     [pins.extrapolated_second_order]),
    ("extrapolated fluxes: transposed velocity gradient",
     "double vx_t = -(ux * dvxx + uy * dvxy) - dpx / rho;",
     "double vx_t = -(ux * dvxx + uy * dvyx) - dpx / rho;",
     [pins.extrapolated_second_order]),
    ("extrapolated fluxes: gamma missing from the pressure equation",
     "double p_t = -(ux * dpx + uy * dpy) - gamma * pr * div;",
     "double p_t = -(ux * dpx + uy * dpy) - pr * div;",
     [pins.extrapolated_second_order]),
    ("extrapolated fluxes: advanced a full step instead of half",
     "half_step_primitives(m, prim, grad, w, p->gamma, 0.5 * h, prim_h);",
     "half_step_primitives(m, prim, grad, w, p->gamma, h, prim_h);",
     [pins.extrapolated_second_order]),
    ("primitive pressure misses the kinetic energy",
     "double pr = (p->gamma - 1.0) * (E / A - 0.5 * rho * (vx * vx + vy * vy));",
     "double pr = (p->gamma - 1.0) * (E / A);",
     [pins.uniform_flow, pins.cfl_uniform]),
    ("Courant minimum skips a cell without a sound speed",
     "    if (!(t > 0.0) || !isfinite(t)) t = 0.0;\n",
     "\n",
     [pins.cfl_uniform]),
    ("Voronoi centroid without the factor 1/3",
     "sx[i] = xi + cx / (3.0 * A2);",
     "sx[i] = xi + cx / A2;",
     [pins.voronoi_identities]),
    ("Voronoi edge midpoint taken at one end",
     "fx[i * max_fan + d] = 0.5 * (ax + bx);",
     "fx[i * max_fan + d] = ax;",
     [pins.voronoi_lattices, pins.voronoi_identities]),
    ("Voronoi clip labels the new edge with the old neighbour",
     "Q.lab[Q.nv] = s0 <= 0.0 ? lab : P->lab[k];",
     "Q.lab[Q.nv] = s0 <= 0.0 ? P->lab[k] : lab;",
     [pins.voronoi_host_agreement]),
    ("Voronoi periodic image code of the lower side",
     "(4u << 28));    /* shift (0, -1) */",
     "(3u << 28));    /* shift (0, -1) */",
     [pins.voronoi_lattices]),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new,catchers", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(tmp_path, name, old, new, catchers):
    assert SRC.count(old) == 1, name
    path = oracle.build_variant(SRC.replace(old, new), os.path.join(str(tmp_path), "liboracle_mut.so"))
    caught = []
    with oracle.use_library(path):
        for pin in catchers:
            try:
                pin(oracle)
            except AssertionError:
                caught.append(pin.__name__)
            except Exception as e:  # a crash on bad numbers also counts
                caught.append(f"{pin.__name__}:{type(e).__name__}")
    assert caught, f"no pin caught: {name}"
