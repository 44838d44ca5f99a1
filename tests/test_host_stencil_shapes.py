"""Host logic of the z-march stencil shapes (compiled with g++, no GPU): the
shell shapes hold exactly the bonds of their shells, and the shared
partial-sum tables that isotropic shapes use cover every bond once.

A bond (target a, source b, cell offset dx, dy, dz, shell) is covered by a
table when exactly one (sum, use) pair gives it: the sum has the member
(b, dx, dy) and the use is (a, dz, shell).  The operation counts per
component and input plane (adds = members - sums, FMAs = uses) are fixed by
the shell structure: bcc 5 shells 32 + 28 against 116 bonds.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2605_26016_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include "spx_stencil.hpp"
using namespace spx;
int main() {
    for (int kind = 0; kind < SHAPE_COUNT; ++kind) {
        const ShapeTable t = make_shape(kind);
        const SumTable st = make_sums(kind);
        int members = 0, bad = 0;
        for (int m = 0; m < st.nsum; ++m) members += st.sums[m].n;
        // every bond: count the (sum member, use) pairs that produce it
        for (int k = 0; k < t.nb; ++k) {
            const ZBond &bd = t.bonds[k];
            int hits = 0;
            for (int m = 0; m < st.nsum; ++m) {
                const ZSum &z = st.sums[m];
                for (int e = 0; e < z.n; ++e) {
                    if (z.b[e] != bd.b || z.dx[e] != bd.dx || z.dy[e] != bd.dy) continue;
                    for (int u = z.u0; u < z.u0 + z.nu; ++u)
                        if (st.uses[u].a == bd.a && st.uses[u].dz == bd.dz && st.uses[u].shell == bd.shell) ++hits;
                }
            }
            if (hits != 1) ++bad;
        }
        // and nothing else: sum of members x uses equals the bond count
        int pairs = 0;
        for (int m = 0; m < st.nsum; ++m) pairs += st.sums[m].n * st.sums[m].nu;
        std::printf("%d %d %d %d %d %d %d %d\n", kind, t.nb, st.nsum, members - st.nsum, st.nuse, pairs, bad,
                    (int)st.ok);
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def table(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("shapes")
    src, exe = d / "shapes.cpp", d / "shapes"
    src.write_text(PROGRAM)
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    rows = {}
    for line in out.split("\n"):
        if line.strip():
            v = [int(x) for x in line.split()]
            rows[v[0]] = dict(nb=v[1], nsum=v[2], adds=v[3], fmas=v[4], pairs=v[5], bad=v[6], ok=v[7])
    return rows


# shapes: 0 sc NN, 1 sc shells 1-3, 2 sc shells 1-4, 3 bcc shells 1-5
# bonds per site: sc 6 / 6+12+8 / +6; bcc 8+6+12+24+8 = 58 per sublattice
@pytest.mark.parametrize("kind,nb", [(0, 6), (1, 26), (2, 32), (3, 116)])
def test_shapes_hold_their_shells(table, kind, nb):
    assert table[kind]["nb"] == nb


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_partial_sums_cover_every_bond_once(table, kind):
    r = table[kind]
    assert r["ok"] == 1 and r["bad"] == 0 and r["pairs"] == r["nb"]


@pytest.mark.parametrize("kind,adds,fmas", [(0, 3, 3), (1, 6, 8), (2, 9, 11), (3, 32, 28)])
def test_partial_sum_operation_counts(table, kind, adds, fmas):
    # sc NN: the four in-plane neighbours form one sum and the two z
    # neighbours share the centre (3 adds, 3 FMAs for 6 bonds); bcc: per
    # target sublattice the 2x2 box, the 4-point cross, the centre, the
    # diagonals and the 8-point ring feed 14 (shell, dz) uses
    assert (table[kind]["adds"], table[kind]["fmas"]) == (adds, fmas)
