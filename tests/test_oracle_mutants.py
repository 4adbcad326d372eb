"""Plant one mistake at a time in a copy of the oracle; some pin must fail.

Each mutant is a plausible slip (a wrong sign, a dropped term, a transposed
operand or index, an off-by-one).  The copy is compiled into a temporary
library on the CPU; the oracle's own source is never changed.
"""
import os

import pytest

import filter_pins
import map_pins
import nbd_pins
import oracle
import oracle_pins as pins

MUTANTS = {
    "diff_sign": ("float diff = p - mn;", "float diff = mn - p;"),
    "floor_to_round": ("return (uint32_t)std::floor(t);", "return (uint32_t)std::round(t);"),
    "dims_off_by_one": ("g->d[a] = (uint32_t)std::floor(t) + 1u;", "g->d[a] = (uint32_t)std::floor(t);"),
    "linear_wrong_dim": ("(uint64_t)d[0] * ((uint64_t)k[1]", "(uint64_t)d[1] * ((uint64_t)k[1]"),
    "linear_axis_swap": ("return (uint64_t)k[0] + (uint64_t)d[0] * ((uint64_t)k[1] + (uint64_t)d[1] * (uint64_t)k[2]);",
                         "return (uint64_t)k[2] + (uint64_t)d[2] * ((uint64_t)k[1] + (uint64_t)d[1] * (uint64_t)k[0]);"),
    "morton_axis_order": ("key |= bit << (3 * b + a);", "key |= bit << (3 * b + (2 - a));"),
    "morton_bits_short": ("for (int b = 0; b < 21; ++b) {", "for (int b = 0; b < 20; ++b) {"),
    "sum_transposed": ("c.sum[a] += p[a];", "c.sum[a] += p[(a + 1) % 3];"),
    "local_sign": ("c.local[a] += p[a] - c.ref_p[a];", "c.local[a] += p[a] + c.ref_p[a];"),
    "colour_no_half": ("(c.rgb[a] + c.n / 2) / c.n", "(c.rgb[a]) / c.n"),
    "ref_last_seen": ("if (c.n == 0) {\n        c.ref = i;", "{\n        c.ref = i;"),
    "validity_drops_z": ("std::isfinite(y) && std::isfinite(z)", "std::isfinite(y)"),
    "overflow_inclusive": ("if (!(t < kMaxCellsPerAxis))", "if (!(t <= kMaxCellsPerAxis))"),
    "backward_no_div": ("dx[i] = gx[c] / nn;", "dx[i] = gx[c];"),
    "min_uses_max": ("if (v < g->mn[a]) g->mn[a] = v;", "if (v > g->mn[a]) g->mn[a] = v;"),
    "leaf_not_checked": ("if (!std::isfinite(r)) return VGO_ERR_LEAF;", ""),
    "point_cell_off": ("point_cell[i] = (int32_t)cells.find(keys[i])->second.rank;",
                       "point_cell[i] = (int32_t)cells.find(keys[i])->second.rank + 1;"),
    "mean_divides_n_plus_1": ("if (cx) cx[r] = c.sum[0] / nn;", "if (cx) cx[r] = c.sum[0] / (nn + 1);"),
    "fixed_sum_transposed": ("s[3 * c + 1] += y[i];", "s[3 * c + 1] += z[i];"),
    "fixed_constant_offset": ("cx[k] = cnt[k] ? s[3 * k + 0] / nn : 0.0;",
                              "cx[k] = cnt[k] ? s[3 * k + 0] / nn + 1e-3 : 0.0;"),
    "fixed_drops_row_0": ("if (c < 0 || c >= m) continue;", "if (c <= 0 || c >= m) continue;"),
    # neighbour-bucket decimation
    "nbd_threshold_inclusive": ("if (cnt > umbral) m.push_back(i);", "if (cnt >= umbral) m.push_back(i);"),
    "nbd_loop_test_inclusive": ("if ((int64_t)m.size() > round_size) {", "if ((int64_t)m.size() >= round_size) {"),
    "nbd_radius_exclusive": ("if (dist2(x[i], y[i], z[i], x[q], y[q], z[q]) <= r2)",
                             "if (dist2(x[i], y[i], z[i], x[q], y[q], z[q]) < r2)"),
    "nbd_drops_lower_z_cells": ("for (int dz = -1; dz <= 1; ++dz)", "for (int dz = 0; dz <= 1; ++dz)"),
    "nbd_deletes_largest": ("std::sort(pri.begin(), pri.end());", "std::sort(pri.rbegin(), pri.rend());"),
    "nbd_keeps_last_marked": ("for (int64_t i : m) present[i] = 0;\n      break;", "break;"),
    "nbd_philox_no_key_bump": ("k0 += kPhiloxW0;", ""),
    "nbd_round_in_wrong_word": ("{(uint64_t)i, (uint64_t)round, 0, 0}", "{(uint64_t)i, 0, (uint64_t)round, 0}"),
    "nbd_deletes_one_fewer": ("for (int64_t k = 0; k < round_size; ++k)", "for (int64_t k = 1; k < round_size; ++k)"),
    "nbd_counts_itself": ("if (q == i) continue;\n            if (dist2", "if (dist2"),
    "nbd_dist_axis_slip": ("float dz = bz - az;", "float dz = by - ay;"),
    "nbd_counts_deleted": ("for (int64_t q : nbr[i]) cnt += present[q];", "for (int64_t q : nbr[i]) cnt += 1;"),
    # transform, height limit, minimum points per cell
    "filter_trans_sign": ("q[a] = s012 + trans[a];", "q[a] = s012 - trans[a];"),
    "filter_rot_column_slip": ("float s1 = rot[3 * a + 1] * p[1];", "float s1 = rot[3 * a + 1] * p[2];"),
    "filter_rot_transposed_row": ("float s0 = rot[3 * a + 0] * p[0];", "float s0 = rot[a] * p[0];"),
    "filter_limit_exclusive": ("q[2] >= z_min && q[2] <= z_max", "q[2] > z_min && q[2] <= z_max"),
    "filter_limit_on_y": ("q[2] >= z_min && q[2] <= z_max", "q[1] >= z_min && q[1] <= z_max"),
    "filter_limit_before_transform": ("q[2] >= z_min && q[2] <= z_max", "p[2] >= z_min && p[2] <= z_max"),
    "filter_min_points_strict": ("if (acount[k] < min_points) continue;", "if (acount[k] <= min_points) continue;"),
    "filter_rows_not_renumbered": ("point_cell[i] = apc[i] < 0 ? -1 : (int32_t)row[apc[i]];",
                                   "point_cell[i] = apc[i];"),
    # global voxel map
    "map_floor_to_trunc": ("float f = std::floor(t);", "float f = std::trunc(t);"),
    "map_key_axis_slip": ("k |= (uint64_t)c << (21 * a);", "k |= (uint64_t)c << (21 * (2 - a));"),
    "map_range_inclusive": ("if (!(f >= -(float)kVoxelHalfRange && f < (float)kVoxelHalfRange)) return false;",
                            "if (!(f >= -(float)kVoxelHalfRange && f <= (float)kVoxelHalfRange)) return false;"),
    "map_rotation_not_transposed": ("float s1 = R[1 * 3 + j] * d[1];", "float s1 = R[j * 3 + 1] * d[1];"),
    "map_centre_at_corner": ("float kc = (float)k + 0.5f;", "float kc = (float)k;"),
    "map_u_bound_off": ("u <= (float)width - 0.5f", "u <= (float)width + 0.5f"),
    "map_far_exclusive": ("q[2] >= z_near && q[2] <= z_far", "q[2] >= z_near && q[2] < z_far"),
    "map_keeps_first_stamp": ("if (voxel_key(m, x[i], y[i], z[i], &k)) m.vox[k] = stamp;",
                              "if (voxel_key(m, x[i], y[i], z[i], &k)) m.vox.insert({k, stamp});"),
    "map_expire_inclusive": ("if (it->second < min_stamp) {", "if (it->second <= min_stamp) {"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "vgo.cpp")).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation anchor not unique/found: {name}"
    mpath = tmp_path / "vgo_mutant.cpp"
    mpath.write_text(src.replace(old, new))
    lib = oracle.load(oracle.build(str(mpath), str(tmp_path / "libmutant.so")))
    caught = []
    for pin in (pins.ALL_PINS + nbd_pins.ALL_NBD_PINS + filter_pins.ALL_FILTER_PINS +
                map_pins.ALL_MAP_PINS):
        try:
            pin(lib)
        except Exception as err:  # any failure of a pin counts as catching the mutant
            caught.append((pin.__name__, type(err).__name__))
    assert caught, f"mutant {name} passed every pin"


# Slips in the batched form (oracle/__init__.py), planted in a copy of the
# function's source and passed to the batched pin in place of the original.
BATCHED_MUTANTS = {
    "next_frame_leaf": ("leaves[b],", "leaves[min(b + 1, len(leaves) - 1)],"),
    "slice_off_by_one": ("s, e = int(frame_offsets[b]), int(frame_offsets[b + 1])",
                         "s, e = int(frame_offsets[b]), int(frame_offsets[b + 1]) - (b % 2)"),
    "swallows_errors": ("if err.status != ERR_GRID_OVERFLOW:\n                raise", "if False:\n                raise"),
    "axes_swapped": ("downsample(x[s:e], y[s:e], z[s:e]", "downsample(x[s:e], z[s:e], y[s:e]"),
    "status_ok_on_overflow": ("status.append(err.status)", "status.append(OK)"),
}


@pytest.mark.parametrize("name", sorted(BATCHED_MUTANTS))
def test_batched_mutant_is_caught(name):
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(oracle.downsample_batched))
    old, new = BATCHED_MUTANTS[name]
    assert src.count(old) == 1, f"mutation anchor not unique/found: {name}"
    ns = dict(vars(oracle))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    with pytest.raises(Exception):
        pins.pin_batched(oracle.load(), batched=ns["downsample_batched"])
