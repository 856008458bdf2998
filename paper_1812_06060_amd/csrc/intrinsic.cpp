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

// Open-addressing map from an edge key to its record (linear probing;
// erased slots become tombstones, the table is rebuilt when they pile up).
void EdgeTable::init(size_t n_keys) {
    size_t cap = 16;
    while (cap < 2 * n_keys + 16) cap <<= 1;
    key.assign(cap, kEmpty);
    val.assign(cap, -1);
    used = tomb = 0;
}
size_t EdgeTable::slot_of(uint64_t k) const {
    return (size_t)((k * 0x9E3779B97F4A7C15ull) >> 17) & (key.size() - 1);
}
int32_t EdgeTable::find(uint64_t k) const {
    for (size_t i = slot_of(k);; i = (i + 1) & (key.size() - 1)) {
        if (key[i] == k) return val[i];
        if (key[i] == kEmpty) return -1;
    }
}
void EdgeTable::insert(uint64_t k, int32_t v) {
    if (2 * (used + tomb + 1) > key.size()) rehash();
    for (size_t i = slot_of(k);; i = (i + 1) & (key.size() - 1)) {
        if (key[i] == kEmpty || key[i] == kTomb) {
            if (key[i] == kTomb) --tomb;
            key[i] = k;
            val[i] = v;
            ++used;
            return;
        }
    }
}
void EdgeTable::erase(uint64_t k) {
    for (size_t i = slot_of(k);; i = (i + 1) & (key.size() - 1)) {
        if (key[i] == k) {
            key[i] = kTomb;
            ++tomb;
            --used;
            return;
        }
        if (key[i] == kEmpty) return;
    }
}
void EdgeTable::rehash() {
    std::vector<uint64_t> k0;
    std::vector<int32_t> v0;
    k0.swap(key);
    v0.swap(val);
    init(used + 1);
    for (size_t i = 0; i < k0.size(); ++i)
        if (k0[i] != kEmpty && k0[i] != kTomb) insert(k0[i], v0[i]);
}

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
    const int64_t nh = 3 * nf;
    auto head_of = [&](int64_t h) { return T[(h / 3) * 3 + (h % 3 + 1) % 3]; };

    // unique edges in canonical order; FE[h] = record of halfedge h's edge
    std::vector<std::pair<uint64_t, int32_t>> hk(nh);
    for (int64_t h = 0; h < nh; ++h) hk[h] = {ekey(T[h], head_of(h)), (int32_t)h};
    std::sort(hk.begin(), hk.end());
    std::vector<int32_t> FE(nh);
    std::vector<ERec> E;
    E.reserve(nh / 2 + 16);
    for (int64_t i = 0; i < nh; ++i) {
        if (i == 0 || hk[i].first != hk[i - 1].first) {
            ERec r;
            r.a = (int32_t)(hk[i].first >> 32);
            r.b = (int32_t)(hk[i].first & 0xffffffffu);
            r.f[0] = r.f[1] = -1;
            r.queued = false;
            const double* p = xyz + 3 * (int64_t)r.a;
            const double* q = xyz + 3 * (int64_t)r.b;
            const double dx = q[0] - p[0], dy = q[1] - p[1], dz = q[2] - p[2];
            r.len = std::sqrt(dx * dx + dy * dy + dz * dz);
            E.push_back(r);
        }
        FE[hk[i].second] = (int32_t)E.size() - 1;
    }
    hk.clear();
    hk.shrink_to_fit();
    const int64_t ne = (int64_t)E.size();
    double lsum = 0.0;
    out.input_a.resize(ne);
    out.input_len.resize(ne);
    for (int64_t i = 0; i < ne; ++i) {
        lsum += E[i].len;
        out.input_a[i] = E[i].a;
        out.input_len[i] = E[i].len;
    }
    out.hbar_input = lsum / (double)ne;
    for (int64_t h = 0; h < nh; ++h) {
        ERec& r = E[FE[h]];
        const int side = T[h] < head_of(h) ? 0 : 1;
        if (r.f[side] >= 0) throw Error{HG_E_BAD_MESH, "non-manifold or inconsistently oriented edge"};
        r.f[side] = (int32_t)(h / 3);
    }
    EdgeTable& index = out.index;
    index.init((size_t)ne);
    for (int64_t i = 0; i < ne; ++i) index.insert(ekey(E[i].a, E[i].b), (int32_t)i);

    // slot of face f whose halfedge starts at vertex a
    auto slot_from = [&](int32_t f, int32_t a) {
        const int64_t b = 3 * (int64_t)f;
        return T[b] == a ? 0 : (T[b + 1] == a ? 1 : 2);
    };
    struct Quad {
        int32_t c, d;
        int32_t e_vc, e_cu, e_ud, e_dv;   // records of the four outer edges
        double L, luc, lvc, lud, lvd, A1, A2, s;
    };
    auto quad = [&](const ERec& r) {
        Quad q;
        const int32_t f1 = r.f[0], f2 = r.f[1];
        const int k1 = slot_from(f1, r.a);   // f1 runs a -> b
        const int k2 = slot_from(f2, r.b);   // f2 runs b -> a
        q.c = T[3 * (int64_t)f1 + (k1 + 2) % 3];
        q.d = T[3 * (int64_t)f2 + (k2 + 2) % 3];
        q.e_vc = FE[3 * (int64_t)f1 + (k1 + 1) % 3];
        q.e_cu = FE[3 * (int64_t)f1 + (k1 + 2) % 3];
        q.e_ud = FE[3 * (int64_t)f2 + (k2 + 1) % 3];
        q.e_dv = FE[3 * (int64_t)f2 + (k2 + 2) % 3];
        q.L = r.len;
        q.luc = E[q.e_cu].len;
        q.lvc = E[q.e_vc].len;
        q.lud = E[q.e_ud].len;
        q.lvd = E[q.e_dv].len;
        q.A1 = tri_area(q.L, q.lvc, q.luc);
        q.A2 = tri_area(q.L, q.lvd, q.lud);
        const double cot_c = (q.lvc * q.lvc + q.luc * q.luc - q.L * q.L) / (4.0 * q.A1);
        const double cot_d = (q.lvd * q.lvd + q.lud * q.lud - q.L * q.L) / (4.0 * q.A2);
        q.s = cot_c + cot_d;
        return q;
    };
    auto interior = [&](const ERec& r) { return r.f[0] >= 0 && r.f[1] >= 0; };
    auto set_face = [&](int32_t f, int32_t x, int32_t y, int32_t z, int32_t exy, int32_t eyz, int32_t ezx) {
        const int64_t b = 3 * (int64_t)f;
        T[b] = x;
        T[b + 1] = y;
        T[b + 2] = z;
        FE[b] = exy;
        FE[b + 1] = eyz;
        FE[b + 2] = ezx;
        E[exy].f[x < y ? 0 : 1] = f;
        E[eyz].f[y < z ? 0 : 1] = f;
        E[ezx].f[z < x ? 0 : 1] = f;
    };

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
        if (q.c == q.d || index.find(ekey(q.c, q.d)) >= 0) continue;
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
        index.insert(ekey(r.a, r.b), i);
        set_face(f1, q.c, u, q.d, q.e_cu, q.e_ud, i);   // (c, u, d)
        set_face(f2, q.d, v, q.c, q.e_dv, q.e_vc, i);   // (d, v, c)
        const int32_t outer[4] = {q.e_cu, q.e_vc, q.e_dv, q.e_ud};   // u c, c v, v d, d u
        for (int32_t j : outer)
            if (interior(E[j]) && !E[j].queued) {
                queue.push_back(j);
                E[j].queued = true;
            }
    }
    int64_t bad = 0;
    for (int64_t i = 0; i < ne; ++i)
        if (interior(E[i]) && quad(E[i]).s < -kFlipTol) ++bad;
    out.n_flips = flips;
    out.n_nondelaunay = bad;
    out.rec_len.resize(ne);
    for (int64_t i = 0; i < ne; ++i) out.rec_len[i] = E[i].len;
}

double IntrinsicTri::edge_length(int32_t a, int32_t b) const {
    const int32_t r = index.find(ekey(a, b));
    if (r < 0) throw Error{HG_E_DEVICE, "intrinsic triangulation: unknown edge"};
    return rec_len[r];
}

}  // namespace hg
