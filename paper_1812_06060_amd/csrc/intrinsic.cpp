// Intrinsic Delaunay triangulation of a mesh (Sec. 5.3), built on the host
// when a mesh is created with hg_mesh_create_intrinsic.
//
// The surface is kept as connectivity plus one length per edge.  An interior
// edge is Delaunay when the two angles facing it sum to at most pi
// (cot a + cot b >= 0); edges that are not are flipped:
//   * lengths start as the 3D edge lengths;
//   * a first-in-first-out queue holds interior edges, initially all of them
//     in canonical order ((smaller id, larger id) ascending); an edge is
//     queued at most once at a time;
//   * a popped edge {u, v} (u < v), f1 the face running u -> v and f2 the
//     face running v -> u, c and d their third vertices, is flipped to
//     {c, d} when cot(c) + cot(d) < -1e-12, unless c == d or c and d are
//     already joined (the mesh stays simplicial; such an edge is left
//     non-Delaunay and counted at the end);
//   * the new length is the distance of c and d once the two triangles are
//     unfolded into the plane on either side of u v; f1 becomes (c, u, d),
//     f2 becomes (d, v, c), and u c, c v, v d, d u are queued.
// Each flip of a non-Delaunay edge lowers the triangulation's Dirichlet
// energy, so the loop ends (a cap of 64 flips per edge guards it anyway).
//
// A flip is a floating-point decision taken on integers (the connectivity),
// so the arithmetic is fixed to these FP64 expressions, evaluated as written
// without contraction into fused multiply-adds:
//   area(a >= b >= c) = sqrt((a + (b + c)) (c - (a - b)) (c + (a - b)) (a + (b - c))) / 4
//                       (0 if the product is not positive),
//   cot of the corner facing side a = (b b + c c - a a) / (4 area),
//   x_c = (L L + l_uc l_uc - l_vc l_vc) / (2 L),  y_c =  2 area(f1) / L,
//   x_d = (L L + l_ud l_ud - l_vd l_vd) / (2 L),  y_d = -2 area(f2) / L,
//   l_cd = sqrt((x_c - x_d)^2 + (y_c - y_d)^2).
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>
#include <deque>
#include <string>
#include <unordered_map>

#include "hgeo_internal.h"

namespace hg {

namespace {

constexpr double kFlipTol = 1e-12;

inline uint64_t ekey(int32_t a, int32_t b) {
    const uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
    return ((uint64_t)lo << 32) | hi;
}

double tri_area(double a, double b, double c) {
    double t;
    if (a < b) { t = a; a = b; b = t; }
    if (b < c) { t = b; b = c; c = t; }
    if (a < b) { t = a; a = b; b = t; }
    const double p = (a + (b + c)) * (c - (a - b)) * (c + (a - b)) * (a + (b - c));
    return p > 0.0 ? 0.25 * std::sqrt(p) : 0.0;
}

struct ERec {
    int32_t a, b;     // a < b
    int32_t f[2];     // face running a -> b, face running b -> a (-1 if none)
    double len;
    bool queued;
};

}  // namespace

void build_intrinsic(const double* xyz, int64_t nv, const int32_t* tri_in, int64_t nf, IntrinsicTri& out) {
    if (nv <= 0 || nf <= 0) throw Error{HG_E_INVALID_ARG, "empty mesh"};
    if (nv >= (1ll << 31) || 3 * nf >= (1ll << 31))
        throw Error{HG_E_INVALID_ARG, "mesh too large for 32-bit element indices"};
    for (int64_t i = 0; i < 3 * nv; ++i)
        if (!std::isfinite(xyz[i])) throw Error{HG_E_INVALID_ARG, "non-finite vertex position"};
    auto& T = out.tri;
    T.assign(tri_in, tri_in + 3 * nf);
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t a = T[3 * f], b = T[3 * f + 1], c = T[3 * f + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv)
            throw Error{HG_E_BAD_MESH, "triangle " + std::to_string(f) + " has a vertex index out of range"};
        if (a == b || b == c || a == c)
            throw Error{HG_E_BAD_MESH, "triangle " + std::to_string(f) + " repeats a vertex"};
    }

    // edges in canonical order
    std::vector<uint64_t> keys;
    keys.reserve(3 * nf);
    for (int64_t h = 0; h < 3 * nf; ++h) keys.push_back(ekey(T[h], T[(h / 3) * 3 + (h % 3 + 1) % 3]));
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    const int64_t ne = (int64_t)keys.size();
    std::vector<ERec> E(ne);
    out.input_a.clear();
    out.input_len.clear();
    out.input_a.reserve(ne);
    out.input_len.reserve(ne);
    std::unordered_map<uint64_t, int32_t> index;
    index.reserve((size_t)(1.3 * (double)ne) + 16);
    double lsum = 0.0;
    for (int64_t i = 0; i < ne; ++i) {
        ERec& r = E[i];
        r.a = (int32_t)(keys[i] >> 32);
        r.b = (int32_t)(keys[i] & 0xffffffffu);
        r.f[0] = r.f[1] = -1;
        r.queued = false;
        const double* p = xyz + 3 * (int64_t)r.a;
        const double* q = xyz + 3 * (int64_t)r.b;
        const double dx = q[0] - p[0], dy = q[1] - p[1], dz = q[2] - p[2];
        r.len = std::sqrt(dx * dx + dy * dy + dz * dz);
        lsum += r.len;
        out.input_a.push_back(r.a);
        out.input_len.push_back(r.len);
        index.emplace(keys[i], (int32_t)i);
    }
    keys.clear();
    keys.shrink_to_fit();
    out.hbar_input = lsum / (double)ne;
    auto set_sides = [&](int64_t f) {
        for (int k = 0; k < 3; ++k) {
            const int32_t a = T[3 * f + k], b = T[3 * f + (k + 1) % 3];
            ERec& r = E[index.at(ekey(a, b))];
            r.f[a < b ? 0 : 1] = (int32_t)f;
        }
    };
    for (int64_t f = 0; f < nf; ++f)
        for (int k = 0; k < 3; ++k) {
            const int32_t a = T[3 * f + k], b = T[3 * f + (k + 1) % 3];
            ERec& r = E[index.at(ekey(a, b))];
            if (r.f[a < b ? 0 : 1] >= 0) throw Error{HG_E_BAD_MESH, "non-manifold or inconsistently oriented edge"};
            r.f[a < b ? 0 : 1] = (int32_t)f;
        }
    auto third = [&](int32_t f, int32_t a, int32_t b) {
        for (int k = 0; k < 3; ++k) {
            const int32_t x = T[3 * (int64_t)f + k];
            if (x != a && x != b) return x;
        }
        return -1;
    };
    auto len_of = [&](int32_t a, int32_t b) { return E[index.at(ekey(a, b))].len; };
    struct Quad {
        int32_t c, d;
        double L, luc, lvc, lud, lvd, A1, A2, s;
    };
    auto quad = [&](const ERec& r) {
        Quad q;
        q.c = third(r.f[0], r.a, r.b);
        q.d = third(r.f[1], r.a, r.b);
        q.L = r.len;
        q.luc = len_of(r.a, q.c);
        q.lvc = len_of(r.b, q.c);
        q.lud = len_of(r.a, q.d);
        q.lvd = len_of(r.b, q.d);
        q.A1 = tri_area(q.L, q.lvc, q.luc);
        q.A2 = tri_area(q.L, q.lvd, q.lud);
        const double cot_c = (q.lvc * q.lvc + q.luc * q.luc - q.L * q.L) / (4.0 * q.A1);
        const double cot_d = (q.lvd * q.lvd + q.lud * q.lud - q.L * q.L) / (4.0 * q.A2);
        q.s = cot_c + cot_d;
        return q;
    };
    auto interior = [&](const ERec& r) { return r.f[0] >= 0 && r.f[1] >= 0; };

    std::deque<int32_t> queue;
    for (int64_t i = 0; i < ne; ++i)
        if (interior(E[i])) {
            queue.push_back((int32_t)i);
            E[i].queued = true;
        }
    int64_t flips = 0;
    const int64_t cap = 64 * ne + 1024;
    while (!queue.empty()) {
        const int32_t i = queue.front();
        queue.pop_front();
        ERec& r = E[i];
        r.queued = false;
        if (!interior(r)) continue;
        const Quad q = quad(r);
        if (q.s >= -kFlipTol) continue;
        if (q.c == q.d || index.count(ekey(q.c, q.d))) continue;
        if (++flips > cap) throw Error{HG_E_BAD_MESH, "intrinsic Delaunay flips did not terminate"};
        const int32_t u = r.a, v = r.b, f1 = r.f[0], f2 = r.f[1];
        const double xc = (q.L * q.L + q.luc * q.luc - q.lvc * q.lvc) / (2.0 * q.L);
        const double yc = 2.0 * q.A1 / q.L;
        const double xd = (q.L * q.L + q.lud * q.lud - q.lvd * q.lvd) / (2.0 * q.L);
        const double yd = -2.0 * q.A2 / q.L;
        const double dx = xc - xd, dy = yc - yd;
        index.erase(ekey(u, v));
        r.a = q.c < q.d ? q.c : q.d;
        r.b = q.c < q.d ? q.d : q.c;
        r.len = std::sqrt(dx * dx + dy * dy);
        r.f[0] = r.f[1] = -1;
        index.emplace(ekey(r.a, r.b), i);
        T[3 * (int64_t)f1] = q.c;
        T[3 * (int64_t)f1 + 1] = u;
        T[3 * (int64_t)f1 + 2] = q.d;
        T[3 * (int64_t)f2] = q.d;
        T[3 * (int64_t)f2 + 1] = v;
        T[3 * (int64_t)f2 + 2] = q.c;
        set_sides(f1);
        set_sides(f2);
        const int32_t outer[4][2] = {{u, q.c}, {q.c, v}, {v, q.d}, {q.d, u}};
        for (const auto& o : outer) {
            const int32_t j = index.at(ekey(o[0], o[1]));
            if (interior(E[j]) && !E[j].queued) {
                queue.push_back(j);
                E[j].queued = true;
            }
        }
    }
    int64_t bad = 0;
    for (int64_t i = 0; i < ne; ++i)
        if (interior(E[i]) && quad(E[i]).s < -kFlipTol) ++bad;
    out.n_flips = flips;
    out.n_nondelaunay = bad;
    out.length.clear();
    out.length.reserve(index.size());
    for (const auto& r : E) out.length.emplace(ekey(r.a, r.b), r.len);
}

double IntrinsicTri::edge_length(int32_t a, int32_t b) const { return length.at(ekey(a, b)); }

}  // namespace hg
