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

}  // namespace spx
