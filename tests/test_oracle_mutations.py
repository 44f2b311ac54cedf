"""Plant plausible mistakes in copies of the oracle and check the pins catch each.

Every mutation edits the oracle's C source text (never the file on disk),
builds the copy with gcc into a temporary directory and runs the pin suite
against it; at least one pin must fail. This is what makes the pins a check
on the oracle rather than a restatement of it.
"""
import pytest

from oracle import ranc_oracle as O
from tests import oracle_pins as P

_SRC = O.source_text()
XBLOCK = _SRC[_SRC.index("    while (dx != 0) {"):_SRC.index("    while (dy != 0) {")]
YBLOCK = _SRC[_SRC.index("    while (dy != 0) {"):_SRC.index("    return y * n->grid_w + x;\n}")]

MUTATIONS = [
    ("strict_threshold", "if (u >= n->threshold[cj])", "if (u > n->threshold[cj])"),
    ("no_leak", "+ acc + n->leak[cj];", "+ acc;"),
    ("leak_twice", "+ acc + n->leak[cj];", "+ acc + 2 * n->leak[cj];"),
    ("no_low_clamp", "if (u < vmin) u = vmin;", ""),
    ("no_high_clamp", "if (u > vmax) u = vmax;", ""),
    ("reset_to_zero", "s->potential[cj] = n->reset[cj];", "s->potential[cj] = 0;"),
    ("type_by_axon_index", "acc += hit * n->weight[cj * G + type];",
     "acc += hit * n->weight[cj * G + (a % G)];"),
    ("ignore_connection", "int hit = row[a] & connected(n, c, a, j);", "int hit = row[a];"),
    ("transposed_crossbar", "uint32_t w = n->crossbar[((size_t)c * n->num_axons + a) * words + j / 32];\n    return (int)((w >> (j % 32)) & 1u);",
     "uint32_t w = n->crossbar[((size_t)c * n->num_axons + (j % n->num_axons)) * words + (a % n->num_neurons) / 32];\n    return (int)((w >> ((a % n->num_neurons) % 32)) & 1u);"),
    ("delay_minus_one", "int row = (s->curr[dest] + n->dest_delay[cj]) % s->rows;",
     "int row = (s->curr[dest] + n->dest_delay[cj] + s->rows - 1) % s->rows;"),
    ("delay_plus_one", "int row = (s->curr[dest] + n->dest_delay[cj]) % s->rows;",
     "int row = (s->curr[dest] + n->dest_delay[cj] + 1) % s->rows;"),
    ("toggle_merge", "sram_row(s, dest, row)[n->dest_axon[cj]] = 1;",
     "sram_row(s, dest, row)[n->dest_axon[cj]] ^= 1;"),
    ("no_row_clear", "memset(sram_row(s, c, s->curr[c]), 0, (size_t)A);", ""),
    ("swap_dx_dy", "route_hops(n, c, n->dest_dx[cj], n->dest_dy[cj], &s->counters[ORC_HOPS], s->links);",
     "route_hops(n, c, n->dest_dy[cj], n->dest_dx[cj], &s->counters[ORC_HOPS], s->links);"),
    ("wrong_dy_sign", "int step = dy > 0 ? 1 : -1;   /* along y */",
     "int step = dy > 0 ? -1 : 1;   /* along y */"),
    ("input_next_tick", "if (input_bit(ext, n, k, i, a))", "if (k > 0 && input_bit(ext, n, k - 1, i, a))"),
    ("input_wrong_core", "int c = n->input_cores[i];", "int c = i;"),
    ("dest_axon_off_by_one", "sram_row(s, dest, row)[n->dest_axon[cj]] = 1;",
     "sram_row(s, dest, row)[(n->dest_axon[cj] + 1) % A] = 1;"),
    ("route_before_integrate_sees_same_tick",  # spikes delivered into the current row
     "int row = (s->curr[dest] + n->dest_delay[cj]) % s->rows;", "int row = s->curr[dest];"),
    ("saturate_at_p_minus_1", "const int64_t vmax = ((int64_t)1 << (n->potential_bits - 1)) - 1;",
     "const int64_t vmax = ((int64_t)1 << (n->potential_bits - 2)) - 1;"),
    ("linear_reset_absolute", "int64_t r = u - n->threshold[cj];", "int64_t r = n->reset[cj];"),
    ("linear_reset_unclamped", "if (r > vmax) r = vmax;", ""),
    ("linear_reset_to_zero", "int64_t r = u - n->threshold[cj];", "int64_t r = 0;"),
    ("no_floor", "if (n->floor && u < n->floor[cj])", "if (0)"),
    ("floor_as_ceiling", "if (n->floor && u < n->floor[cj])", "if (n->floor && u > n->floor[cj])"),
    ("floor_on_reset_value", "                        s->potential[cj] = n->reset[cj];\n",
     "                        s->potential[cj] = (n->floor && n->reset[cj] < n->floor[cj]) ? n->floor[cj] : n->reset[cj];\n"),
    ("leak_width_off_by_one", "const int64_t lmax = ((int64_t)1 << (n->leak_bits - 1)) - 1,",
     "const int64_t lmax = ((int64_t)1 << (n->leak_bits - 1)),"),
    ("reset_width_unchecked", "if (n->reset[i] < rmin || n->reset[i] > rmax)", "if (0)"),
    ("route_y_before_x", XBLOCK + YBLOCK, YBLOCK + XBLOCK),
    ("link_counted_at_next_core",
     "            ++links[((size_t)y * n->grid_w + x) * ORC_NLINKS + (step > 0 ? ORC_LINK_XPLUS : ORC_LINK_XMINUS)];\n        x += step;",
     "            ++links[((size_t)y * n->grid_w + x + step) * ORC_NLINKS + (step > 0 ? ORC_LINK_XPLUS : ORC_LINK_XMINUS)];\n        x += step;"),
    ("x_link_directions_swapped", "(step > 0 ? ORC_LINK_XPLUS : ORC_LINK_XMINUS)", "(step > 0 ? ORC_LINK_XMINUS : ORC_LINK_XPLUS)"),
    ("y_link_as_x_link", "(step > 0 ? ORC_LINK_YPLUS : ORC_LINK_YMINUS)", "(step > 0 ? ORC_LINK_XPLUS : ORC_LINK_XMINUS)"),
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_mutation(name, old, new, tmp_path):
    src = O.source_text()
    assert old in src, f"mutation anchor for {name} not found"
    lib = O.build_variant(src.replace(old, new, 1), str(tmp_path / f"orc_{name}.so"))
    caught = []
    for pin in P.ALL_PINS:
        try:
            pin(lib)
        except (AssertionError, RuntimeError, ValueError) as e:  # noqa: PERF203
            caught.append(f"{pin.__name__}: {str(e)[:80]}")
            break
    assert caught, f"no pin caught mutation {name}"
