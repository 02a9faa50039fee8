// Marching-cubes triangle table for the library, generated at start-up from
// a face-consistent rule (the surface extraction closing Sec. III-B; the mesh
// is to be watertight and manifold, Sec. I).  No published table is used.
//
// Corner k of a cell sits at offset (k&1, (k>>1)&1, (k>>2)&1); a corner is
// inside when A > L.  Cube edge id = 4 axis + b_lo + 2 b_hi, with b_lo, b_hi
// the offset bits of the two other axes in x < y < z order.
//
// Rule, per case:
//  1. Walk each face's four corners counter-clockwise as seen from outside the
//     cube.  An edge where the walk goes outside -> inside "enters", one
//     where it goes inside -> outside "leaves".  Each entering edge is joined
//     to the next leaving edge of the walk by a segment directed enter ->
//     leave; the inside corners then lie to the segment's right seen from
//     outside, and a face with inside corners on a diagonal gets two segments
//     that keep those corners apart.  Both cells sharing a face see the same
//     corner values and build the same segments, reversed.
//  2. Segments chain into closed loops (every crossing edge lies on two faces).
//  3. Loops are taken in order of their smallest edge id, each walked along
//     its direction from that id (right-hand normal: inside -> outside).
//  4. A loop is fanned from its first vertex, in walk order, whose fan draws
//     no diagonal between two edges of one face, so no triangle edge can be
//     shared by more than the two cells of that face.
#include <cstdint>
#include <cstring>
#include <stdexcept>

#include "fvr_common.h"

namespace fvr {

namespace {

int other_axes(int axis, int which) {
    const int o[3][2] = {{1, 2}, {0, 2}, {0, 1}};
    return o[axis][which];
}

int edge_between(int c0, int c1) {
    const int diff = c0 ^ c1;
    const int axis = diff == 1 ? 0 : diff == 2 ? 1 : 2;
    const int lo = c0 & c1;  // the corner with the axis bit clear
    const int bl = (lo >> other_axes(axis, 0)) & 1;
    const int bh = (lo >> other_axes(axis, 1)) & 1;
    return 4 * axis + bl + 2 * bh;
}

// faces[f][0..3]: corner cycle counter-clockwise seen from outside.
void face_cycles(int faces[6][4]) {
    int f = 0;
    for (int a = 0; a < 3; ++a) {
        const int u = (a + 1) % 3, v = (a + 2) % 3;  // u x v = +e_a
        for (int side = 0; side < 2; ++side, ++f) {
            const int base = side << a;
            const int uv[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
            for (int i = 0; i < 4; ++i) {
                // seen from -e_a (side 0) the (u, v) cycle runs clockwise: reverse it
                const int j = side ? i : (4 - i) % 4;
                faces[f][i] = base | (uv[j][0] << u) | (uv[j][1] << v);
            }
        }
    }
}

}  // namespace

void mc_generate_table(uint8_t counts[256], int8_t edges[256 * kMcRow]) {
    int faces[6][4];
    face_cycles(faces);
    // face membership of each edge
    int face_mask[12] = {0};
    for (int f = 0; f < 6; ++f)
        for (int i = 0; i < 4; ++i) face_mask[edge_between(faces[f][i], faces[f][(i + 1) % 4])] |= 1 << f;

    std::memset(counts, 0, 256);
    std::memset(edges, -1, 256 * kMcRow);
    for (int cs = 0; cs < 256; ++cs) {
        int next[12];
        for (int e = 0; e < 12; ++e) next[e] = -1;
        for (int f = 0; f < 6; ++f) {
            int ein[4], kind[4];  // kind: +1 enter, -1 leave, 0 none
            for (int i = 0; i < 4; ++i) {
                const int c0 = faces[f][i], c1 = faces[f][(i + 1) % 4];
                const int i0 = (cs >> c0) & 1, i1 = (cs >> c1) & 1;
                ein[i] = edge_between(c0, c1);
                kind[i] = (!i0 && i1) ? 1 : (i0 && !i1) ? -1 : 0;
            }
            for (int i = 0; i < 4; ++i) {
                if (kind[i] != 1) continue;
                for (int d = 1; d < 4; ++d) {
                    const int j = (i + d) % 4;
                    if (kind[j] == -1) {
                        if (next[ein[i]] != -1) throw std::logic_error("mc table: edge left twice");
                        next[ein[i]] = ein[j];
                        break;
                    }
                }
            }
        }
        int nt = 0;
        bool seen[12] = {false};
        for (int start = 0; start < 12; ++start) {
            if (next[start] < 0 || seen[start]) continue;
            int loop[12], k = 0;
            int e = start;
            do {
                seen[e] = true;
                loop[k++] = e;
                e = next[e];
                if (e < 0 || k > 12) throw std::logic_error("mc table: open loop");
            } while (e != start);
            int anchor = -1;
            for (int s = 0; s < k && anchor < 0; ++s) {
                bool clean = true;
                for (int i = 2; i < k - 1; ++i)
                    if (face_mask[loop[s]] & face_mask[loop[(s + i) % k]]) clean = false;
                if (clean) anchor = s;
            }
            if (anchor < 0) throw std::logic_error("mc table: no clean fan anchor");
            for (int i = 1; i < k - 1; ++i) {
                if (nt >= kMcMaxTris) throw std::logic_error("mc table: too many triangles");
                edges[cs * kMcRow + 3 * nt + 0] = (int8_t)loop[anchor];
                edges[cs * kMcRow + 3 * nt + 1] = (int8_t)loop[(anchor + i) % k];
                edges[cs * kMcRow + 3 * nt + 2] = (int8_t)loop[(anchor + i + 1) % k];
                ++nt;
            }
        }
        counts[cs] = (uint8_t)nt;
    }
}

}  // namespace fvr
