"""Planted mistakes in the oracle, for tests/test_oracle_mutants.py.

Each mutant is one plausible error in one oracle file (a dropped term, a
wrong sign, index or constant, a transposed operand), given as the exact
source text it replaces.  The pins must fail for every one of them: a mutant
that survives means some part of the oracle is not pinned to anything but
itself."""

# (name, oracle file, original text (must occur exactly once), replacement)
MUTANTS = [
    # mip pyramid and its adjoint (2x2x2 mean, Section 4.3.3)
    ("mips_mean_over_4", "vct_oracle.py", "mips.append(total / 8.0)", "mips.append(total / 4.0)"),
    ("mips_child_index_repeated", "vct_oracle.py", "m[dz::2, dy::2, dx::2] for dz",
     "m[dz::2, dy::2, dy::2] for dz"),
    ("mip_adjoint_scale", "vct_oracle.py", "+ up / 8.0", "+ up / 4.0"),
    # quadrilinear sampler (Section 4.3.3)
    ("sampler_no_half_texel", "vct_oracle.py", "* nl[:, None] - 0.5", "* nl[:, None]"),
    ("sampler_level_weights_swapped", "vct_oracle.py", "((l0, 1.0 - f), (l1, f))", "((l0, f), (l1, 1.0 - f))"),
    ("sampler_y_weights_swapped", "vct_oracle.py", "(phi[:, 1] if dy else 1.0 - phi[:, 1])",
     "(1.0 - phi[:, 1] if dy else phi[:, 1])"),
    ("sampler_clamp_one_short", "vct_oracle.py", "hi = (n0 >> lev) - 1", "hi = max((n0 >> lev) - 2, 0)"),
    # cone set (Section 4.2)
    ("origin_offset_not_in_voxels", "vct_oracle.py", "o = x + nn * (params.normal_offset * v0)",
     "o = x + nn * params.normal_offset * 0.5"),
    ("bitangent_sign", "vct_oracle.py", "bb = np.cross(nn, tt)", "bb = np.cross(tt, nn)"),
    ("reflection_sign", "vct_oracle.py", "r = vdir - 2.0 * np.sum", "r = vdir + 2.0 * np.sum"),
    ("specular_aperture_ignores_roughness", "vct_oracle.py", "rough * float(params.spec_aperture_scale)",
     "0.5 + 0.0 * rough * float(params.spec_aperture_scale)"),
    ("occlusion_ignores_light_distance", "vct_oracle.py", "np.minimum(float(params.max_dist), dist)",
     "np.full_like(dist, float(params.max_dist))"),
    # march (Section 4.3.2)
    ("diameter_full_angle", "vct_oracle.py", "2.0 * ti * np.tan(gamma[idx] / 2.0)", "2.0 * ti * np.tan(gamma[idx])"),
    ("lod_of_radius", "vct_oracle.py", "np.log2(d / v0), 0.0", "np.log2(d / (2.0 * v0)), 0.0"),
    ("colour_without_transmittance", "vct_oracle.py", "c[idx] += (1.0 - a_prev)[:, None] * s[:, 0:3]",
     "c[idx] += s[:, 0:3]"),
    ("alpha_without_transmittance", "vct_oracle.py", "alpha[idx] = a_prev + (1.0 - a_prev) * s[:, 3]",
     "alpha[idx] = a_prev + s[:, 3]"),
    ("step_without_beta", "vct_oracle.py", "t[idx] = ti + beta * d", "t[idx] = ti + d"),
    ("threshold_inclusive", "vct_oracle.py", "(t[idx] <= tmax[idx]) & (alpha[idx] < thresh)",
     "(t[idx] <= tmax[idx]) & (alpha[idx] <= thresh - 0.02)"),
    ("tmax_exclusive", "vct_oracle.py", "active[idx] = (t[idx] <= tmax[idx])", "active[idx] = (t[idx] < tmax[idx] - 1e-3)"),
    # epilogue (Section 4.2)
    ("diffuse_weights_dropped", "vct_oracle.py", 'out[pix[sel], 0:3] += wq[q] * res["c"][sel]',
     'out[pix[sel], 0:3] += res["c"][sel]'),
    ("specular_and_occlusion_slots_swapped", "vct_oracle.py",
     '    sel = slot == nd\n    out[pix[sel], 4:7] = res["c"][sel]\n    sel = slot == nd + 1\n',
     '    sel = slot == nd + 1\n    out[pix[sel], 4:7] = res["c"][sel]\n    sel = slot == nd\n'),
    # adjoint (derivatives of the Section 4.3.2 recurrences)
    ("adjoint_colour_without_transmittance", "vct_oracle.py", "g_c = T[:, None] * gc[idx]", "g_c = gc[idx]"),
    ("adjoint_alpha_sign", "vct_oracle.py", "(-np.sum(gc[idx] * R[idx], axis=1) + ga[idx] * U[idx])",
     "(np.sum(gc[idx] * R[idx], axis=1) + ga[idx] * U[idx])"),
    ("adjoint_suffix_colour", "vct_oracle.py", "R[idx] = s[:, 0:3] + (1.0 - s[:, 3])[:, None] * R[idx]",
     "R[idx] = s[:, 0:3] + R[idx]"),
    ("adjoint_suffix_alpha", "vct_oracle.py", "U[idx] = (1.0 - s[:, 3]) * U[idx]", "U[idx] = U[idx]"),
    ("adjoint_diffuse_weight_dropped", "vct_oracle.py", "ga[sel] = wq[q] * g[pix[sel], 3]",
     "ga[sel] = g[pix[sel], 3]"),
    # shading variants (Section 5.4.4)
    ("falloff_linear_in_t", "vct_shade.py", "np.sqrt(ti) * shade.shadow_strength", "ti * shade.shadow_strength"),
    ("first_hit_keeps_marching", "vct_shade.py", "active[idx] = (~hit) & (t[idx] <= tmax[idx])",
     "active[idx] = t[idx] <= tmax[idx]"),
    ("falloff_without_transmittance", "vct_shade.py", "occ[idx] = occ[idx] + (1.0 - occ[idx]) * a_s",
     "occ[idx] = occ[idx] + a_s"),
    ("o_min_as_product", "vct_shade.py", "o_min = np.minimum(o_min, vis)", "o_min = o_min * vis"),
    ("phong_reflection_sign", "vct_shade.py", "refl = 2.0 * ndl[:, None] * nn - ld",
     "refl = 2.0 * ndl[:, None] * nn + ld"),
    ("diffuse_not_occluded", "vct_shade.py", "o_min[pix, None] * diffuse[pix]", "diffuse[pix]"),
    ("grace_sign", "vct_shade.py", "np.maximum(0.0, gamma - p)", "np.maximum(0.0, gamma + p)"),
    ("direct_not_shadowed", "vct_shade.py", "direct += vis[:, None] * term", "direct += term"),
    # voxelization (Section 4.4)
    ("dominant_axis_signed", "vct_voxelize.py", "dom = int(np.argmax(np.abs(nrm)))", "dom = int(np.argmax(nrm))"),
    ("no_top_left_rule", "vct_voxelize.py", "inside &= (e > 0) | ((e == 0) & _top_left(dx, dy))",
     "inside &= e >= 0"),
    ("pixel_corner_not_centre", "vct_voxelize.py", "PX = I.ravel() * SUB + h", "PX = I.ravel() * SUB"),
    ("attenuation_linear_twice", "vct_voxelize.py", "att[0] + att[1] * dist + att[2] * dist * dist",
     "att[0] + att[1] * dist + att[2] * dist"),
    ("lambert_two_sided", "vct_voxelize.py", "lam = np.maximum(0.0, ldir @ nn)", "lam = np.abs(ldir @ nn)"),
    ("colour_sum_not_mean", "vct_voxelize.py", "out[hit, 0:3] = acc[hit] / cnt[hit][:, None]",
     "out[hit, 0:3] = acc[hit]"),
    ("snap_floor", "vct_voxelize.py", "u = np.rint((t - o) * scale)", "u = np.floor((t - o) * scale)"),
    ("no_ambient", "vct_voxelize.py", "(ambient + diffuse * lam)", "(diffuse * lam)"),
    # further bounce (Sections 6.2.2 and 5.1.3)
    ("voxel_centre_y_from_z", "vct_bounce.py", "pr[0, 0, :, 1] = o[1] + (y + 0.5) * v0",
     "pr[0, 0, :, 1] = o[1] + (z + 0.5) * v0"),
    ("voxel_corner_not_centre", "vct_bounce.py", "pr[0, 0, :, 0] = o[0] + (x + 0.5) * v0",
     "pr[0, 0, :, 0] = o[0] + x * v0"),
    ("bounce_ignores_alpha", "vct_bounce.py", "vals[:, 0:3] += base[z, y, x, 3:4] * alb * gathered",
     "vals[:, 0:3] += alb * gathered"),
    ("bounces_restart_from_direct", "vct_bounce.py", "extent, gather_from=cur)", "extent, gather_from=None)"),
    # anisotropic pyramids (Section 5.1.3)
    ("aniso_composite_without_transmittance", "vct_aniso.py",
     "out[..., 0:3] = f[..., 0:3] + (1.0 - f[..., 3:4]) * b[..., 0:3]", "out[..., 0:3] = f[..., 0:3] + b[..., 0:3]"),
    ("aniso_front_child_swapped", "vct_aniso.py", "        front_even = d % 2 == 0\n        pyr = [m0]",
     "        front_even = d % 2 == 1\n        pyr = [m0]"),
    ("aniso_axis_reversed", "vct_aniso.py", "        axis = 2 - d // 2                  # x is array axis 2",
     "        axis = d // 2                  # x is array axis 2"),
    ("aniso_weight_not_squared", "vct_aniso.py", "(wa[sel] ** 2)[:, None]", "np.abs(wa[sel])[:, None]"),
    ("aniso_direction_sign", "vct_aniso.py", "for d, sel in ((2 * a, wa >= 0), (2 * a + 1, wa < 0)):",
     "for d, sel in ((2 * a, wa < 0), (2 * a + 1, wa >= 0)):"),
    ("aniso_adjoint_front_sign", "vct_aniso.py", "gf[..., 3] -= 0.25 * np.sum(Gu * b, axis=-1)",
     "gf[..., 3] += 0.25 * np.sum(Gu * b, axis=-1)"),
    ("aniso_adjoint_back_transmittance", "vct_aniso.py", "gb = 0.25 * Gu * (1.0 - f[..., 3:4])", "gb = 0.25 * Gu"),
    ("aniso_scatter_level0_unweighted", "vct_aniso.py",
     "np.add.at(grads[0][0], (iz[sel], iy[sel], ix[sel]), (wt[sel] * w2[sel, a])[:, None] * gs[sel])",
     "np.add.at(grads[0][0], (iz[sel], iy[sel], ix[sel]), wt[sel][:, None] * gs[sel])"),
]

# The pin files, and which of them to run first for each oracle file (pytest
# stops at the first failure, so the pins closest to the mutated code go first).
PIN_FILES = ["test_oracle_pins.py", "test_shade_pins.py", "test_voxelize_pins.py", "test_bounce_pins.py",
             "test_aniso_pins.py"]
FIRST = {"vct_oracle.py": "test_oracle_pins.py", "vct_shade.py": "test_shade_pins.py",
         "vct_voxelize.py": "test_voxelize_pins.py", "vct_bounce.py": "test_bounce_pins.py",
         "vct_aniso.py": "test_aniso_pins.py"}
