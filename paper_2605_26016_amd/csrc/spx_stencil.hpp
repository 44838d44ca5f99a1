// spx_stencil.hpp -- compile-time stencil shapes for the z-marching LDS
// stencil engine (spx_stencil.hip), shared with the host code that matches a
// runtime bond table against them.
//
// A shape is the set of directed bonds (target a, source b, cell offset
// dx, dy, dz) of one structured neighbour pattern (the "structured sparse
// shell" kernels of the sparse backend, Methods: backend representations).
// The couplings stay runtime values; only the offsets are compile-time, which
// lets the kernel address LDS with immediate offsets and share neighbour
// loads between bonds.
#pragma once

namespace spx {

struct ZBond {
    int a, b, dx, dy, dz;
    int shell;  // index of the bond's shell within the shape (0 = nearest)
};

enum ShapeKind { SHAPE_SC_NN = 0, SHAPE_SC_3SH = 1, SHAPE_SC_4SH = 2, SHAPE_BCC_5SH = 3, SHAPE_COUNT = 4 };

constexpr int kMaxShapeBonds = 128;

struct ShapeTable {
    int nsub;
    int nb;
    ZBond bonds[kMaxShapeBonds];
    int rx, ry, dzlo, dzhi;
    int nshell;
};

// Squared bond length in units where the cubic cell edge is 2 (so bcc body
// centres are integer): r2 = |2 (delta + f_b - f_a)|^2.
constexpr int shape_r2(int kind, int a, int b, int dx, int dy, int dz) {
    int ox = 2 * dx, oy = 2 * dy, oz = 2 * dz;
    if (kind == SHAPE_BCC_5SH) {
        const int s = (b - a);  // body centre at (1,1,1) in these units
        ox += s;
        oy += s;
        oz += s;
    }
    return ox * ox + oy * oy + oz * oz;
}

// Shell radii of each shape, as squared lengths in the units of shape_r2.
constexpr int shape_shell_r2(int kind, int k) {
    switch (kind) {
    case SHAPE_SC_NN: return k == 0 ? 4 : -1;                                 // shell 1
    case SHAPE_SC_3SH: return k < 3 ? (k + 1) * 4 : -1;                        // shells 1-3
    case SHAPE_SC_4SH: return k < 4 ? (k + 1) * 4 : -1;                        // shells 1-4
    case SHAPE_BCC_5SH: {                                                      // shells 1-5
        constexpr int r[5] = {3, 4, 8, 11, 12};
        return k < 5 ? r[k] : -1;
    }
    default: return -1;
    }
}

// Shell index of a bond of squared length r2, -1 if it is not in the shape.
constexpr int shape_shell(int kind, int r2) {
    for (int k = 0; k < 8; ++k) {
        const int v = shape_shell_r2(kind, k);
        if (v < 0) break;
        if (v == r2) return k;
    }
    return -1;
}

constexpr bool shape_has(int kind, int r2) { return shape_shell(kind, r2) >= 0; }

constexpr int shape_nsub(int kind) { return kind == SHAPE_BCC_5SH ? 2 : 1; }

// Bonds are ordered by source position (b, dy, dx), then (a, dz), so that the
// bonds reading one staged neighbour value are adjacent.
constexpr void shape_add(ShapeTable &t, int kind, int a, int b, int dx, int dy, int dz) {
    if (a >= t.nsub || b >= t.nsub) return;
    const int r2 = shape_r2(kind, a, b, dx, dy, dz);
    if (r2 == 0 || !shape_has(kind, r2)) return;
    const int sh = shape_shell(kind, r2);
    t.bonds[t.nb] = ZBond{a, b, dx, dy, dz, sh};
    t.nb++;
    if (sh + 1 > t.nshell) t.nshell = sh + 1;
    const int ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy;
    if (ax > t.rx) t.rx = ax;
    if (ay > t.ry) t.ry = ay;
    if (dz < t.dzlo) t.dzlo = dz;
    if (dz > t.dzhi) t.dzhi = dz;
}

constexpr ShapeTable make_shape(int kind) {
    ShapeTable t{};
    t.nsub = shape_nsub(kind);
    t.nb = 0;
    t.rx = t.ry = 0;
    t.dzlo = 0;
    t.dzhi = 0;
    t.nshell = 0;
    for (int b = 0; b < 2; ++b)
        for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx)
                for (int a = 0; a < 2; ++a)
                    for (int dz = -2; dz <= 2; ++dz) shape_add(t, kind, a, b, dx, dy, dz);
    return t;
}

// Shared partial sums of an isotropic shape.  With one coupling per shell,
// the bonds of one (target a, dz, shell) group all take the same J, so the
// group's staged sources are summed first and multiplied once; groups with
// the same source set (a shell's sources at dz and -dz, or two shells on
// one set: on bcc the 2x2 box feeds the 1st and 4th shells) share one sum.
// On the bcc 5-shell shape this turns 116 FMAs per component and input
// plane into 32 adds and 28 FMAs.
constexpr int kMaxSums = 48, kMaxMembers = 32, kMaxUses = 128;
struct ZSum {
    int n;                  // members (staged source positions)
    int b[kMaxMembers], dx[kMaxMembers], dy[kMaxMembers];
    int u0, nu;             // its uses: uses[u0 .. u0 + nu)
};
struct ZUse {
    int a, dz, shell;
};
struct SumTable {
    int nsum, nuse;
    ZSum sums[kMaxSums];
    ZUse uses[kMaxUses];
    bool ok;                // false if the shape overflows the table
};

constexpr SumTable make_sums(int kind) {
    const ShapeTable t = make_shape(kind);
    SumTable st{};
    st.ok = true;
    // groups keyed by (a, dz, shell), members in bond order
    int ng = 0;
    int ga[kMaxUses] = {}, gdz[kMaxUses] = {}, gsh[kMaxUses] = {}, gn[kMaxUses] = {};
    int gb[kMaxUses][kMaxMembers] = {}, gx[kMaxUses][kMaxMembers] = {}, gy[kMaxUses][kMaxMembers] = {};
    for (int k = 0; k < t.nb; ++k) {
        const ZBond &bd = t.bonds[k];
        int g = 0;
        while (g < ng && !(ga[g] == bd.a && gdz[g] == bd.dz && gsh[g] == bd.shell)) ++g;
        if (g == ng) {
            if (ng == kMaxUses) { st.ok = false; return st; }
            ga[g] = bd.a;
            gdz[g] = bd.dz;
            gsh[g] = bd.shell;
            gn[g] = 0;
            ++ng;
        }
        if (gn[g] == kMaxMembers) { st.ok = false; return st; }
        gb[g][gn[g]] = bd.b;
        gx[g][gn[g]] = bd.dx;
        gy[g][gn[g]] = bd.dy;
        ++gn[g];
    }
    // one sum per distinct member list (bond order makes equal sets equal lists)
    int gsum[kMaxUses] = {};
    for (int g = 0; g < ng; ++g) {
        int m = 0;
        for (; m < st.nsum; ++m) {
            const ZSum &z = st.sums[m];
            bool same = z.n == gn[g];
            for (int e = 0; same && e < z.n; ++e)
                same = z.b[e] == gb[g][e] && z.dx[e] == gx[g][e] && z.dy[e] == gy[g][e];
            if (same) break;
        }
        if (m == st.nsum) {
            if (st.nsum == kMaxSums) { st.ok = false; return st; }
            ZSum &z = st.sums[st.nsum++];
            z.n = gn[g];
            for (int e = 0; e < z.n; ++e) {
                z.b[e] = gb[g][e];
                z.dx[e] = gx[g][e];
                z.dy[e] = gy[g][e];
            }
        }
        gsum[g] = m;
    }
    // uses grouped by sum
    for (int m = 0; m < st.nsum; ++m) {
        st.sums[m].u0 = st.nuse;
        for (int g = 0; g < ng; ++g)
            if (gsum[g] == m) st.uses[st.nuse++] = ZUse{ga[g], gdz[g], gsh[g]};
        st.sums[m].nu = st.nuse - st.sums[m].u0;
    }
    return st;
}

}  // namespace spx
