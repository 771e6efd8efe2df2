// Problem setup on the host: node graph, CSR pattern, element-pair slot map and
// the external load vector.  Runs once per mesh (fem_build_pattern); the hot path
// (assembly, SpMV, Krylov, Newton, adjoint) runs entirely in device kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "internal.h"

namespace fem {

void *dev_alloc(fem_handle *h, size_t bytes) {
    void *p = nullptr;
    if (bytes == 0) bytes = 256;
    FEM_HIP(hipMalloc(&p, bytes));
    h->allocations.push_back(p);
    return p;
}

template <typename T>
static T *upload(fem_handle *h, const std::vector<T> &v) {
    T *p = static_cast<T *>(dev_alloc(h, v.size() * sizeof(T)));
    if (!v.empty()) FEM_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
}

// Runs fn(begin, end) over [0, n) split into contiguous chunks on host threads.
template <typename F>
static void parallel_for(int64_t n, F fn) {
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 4096 || nt == 1) {
        fn(int64_t(0), n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        int64_t b = t * chunk, e = std::min(n, b + chunk);
        if (b >= e) break;
        th.emplace_back([=] { fn(b, e); });
    }
    for (auto &t : th) t.join();
}

HostGraph host_graph(const fem_mesh_desc *d, const std::vector<uint8_t> &mask) {
    HostGraph g;
    const int64_t Nn = d->n_nodes, Ne = d->n_elems;
    const int nd = d->ndpn;
    const int32_t *conn = d->conn;
    g.Nn = Nn;
    g.Ne = Ne;
    g.nd = nd;
    g.N = Nn * nd;
    if (Ne >= (int64_t(1) << 25)) throw Error(FEM_ERANGE, "more than 2^25 elements: slot encodings overflow int32");
    for (int64_t i = 0; i < Ne * 8; ++i)
        if (conn[i] < 0 || conn[i] >= Nn) throw Error(FEM_EINVAL, "element connectivity references a missing node");

    // node -> (element, local node) incidence, element ascending within a node
    std::vector<int64_t> &ne_ptr = g.ne_ptr;
    ne_ptr.assign(Nn + 1, 0);
    for (int64_t i = 0; i < Ne * 8; ++i) ne_ptr[conn[i] + 1]++;
    for (int64_t n = 0; n < Nn; ++n) ne_ptr[n + 1] += ne_ptr[n];
    std::vector<int32_t> ne_list(Ne * 8);
    {
        std::vector<int64_t> fill(ne_ptr.begin(), ne_ptr.end() - 1);
        for (int64_t e = 0; e < Ne; ++e)
            for (int a = 0; a < 8; ++a) ne_list[fill[conn[8 * e + a]]++] = int32_t(e * 8 + a);
    }
    // Element outputs are written in this node-major incidence order: (e, a) goes to
    // slot kpos[e*8 + a], so the contributions of node n are the contiguous slots
    // ne_ptr[n] .. ne_ptr[n+1] and the gathers read them as one run.
    std::vector<int32_t> &kpos = g.kpos;
    kpos.resize(Ne * 8);
    for (int64_t s = 0; s < Ne * 8; ++s) kpos[ne_list[s]] = int32_t(s);

    // neighbour sets: nodes sharing an element, ascending, unique
    std::vector<int64_t> &node_ptr = g.node_ptr;
    node_ptr.assign(Nn + 1, 0);
    auto neighbours = [&](int64_t n, std::vector<int32_t> &buf) {
        buf.clear();
        for (int64_t s = ne_ptr[n]; s < ne_ptr[n + 1]; ++s) {
            int64_t e = ne_list[s] >> 3;
            for (int b = 0; b < 8; ++b) buf.push_back(conn[8 * e + b]);
        }
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
    };
    parallel_for(Nn, [&](int64_t b, int64_t e) {
        std::vector<int32_t> buf;
        for (int64_t n = b; n < e; ++n) {
            neighbours(n, buf);
            node_ptr[n + 1] = int64_t(buf.size());
        }
    });
    for (int64_t n = 0; n < Nn; ++n) node_ptr[n + 1] += node_ptr[n];
    const int64_t nnzb = node_ptr[Nn];
    g.nnzb = nnzb;
    g.nnz = nnzb * nd * nd;
    if (g.nnz >= (int64_t(1) << 31)) throw Error(FEM_ERANGE, "nnz >= 2^31 does not fit 32-bit CSR positions");
    std::vector<int32_t> &node_nb = g.node_nb, &blk_row = g.blk_row;
    node_nb.resize(nnzb);
    blk_row.resize(nnzb);
    parallel_for(Nn, [&](int64_t b, int64_t e) {
        std::vector<int32_t> buf;
        for (int64_t n = b; n < e; ++n) {
            neighbours(n, buf);
            std::copy(buf.begin(), buf.end(), node_nb.begin() + node_ptr[n]);
            std::fill(blk_row.begin() + node_ptr[n], blk_row.begin() + node_ptr[n + 1], int32_t(n));
        }
    });
    auto find_block = [&](int64_t n, int32_t m) -> int64_t {
        auto first = node_nb.begin() + node_ptr[n], last = node_nb.begin() + node_ptr[n + 1];
        auto it = std::lower_bound(first, last, m);
        return (it != last && *it == m) ? int64_t(it - node_nb.begin()) : -1;
    };
    std::vector<int32_t> &mirror = g.mirror, &bdiag = g.bdiag;
    mirror.resize(nnzb);
    bdiag.resize(Nn);
    parallel_for(Nn, [&](int64_t b, int64_t e) {
        for (int64_t n = b; n < e; ++n) {
            for (int64_t k = node_ptr[n]; k < node_ptr[n + 1]; ++k) mirror[k] = int32_t(find_block(node_nb[k], int32_t(n)));
            bdiag[n] = int32_t(find_block(n, int32_t(n)));
        }
    });

    // element-pair -> block slot, and its inverse (contributions per block)
    std::vector<int32_t> &bslot = g.bslot;
    bslot.resize(Ne * 64);
    parallel_for(Ne, [&](int64_t b, int64_t e_end) {
        for (int64_t e = b; e < e_end; ++e)
            for (int a = 0; a < 8; ++a)
                for (int c = 0; c < 8; ++c) bslot[e * 64 + a * 8 + c] = int32_t(find_block(conn[8 * e + a], conn[8 * e + c]));
    });
    // node-centric gather: for slot k (element row block) and column block b, the
    // position of the target block in the row node's neighbour list
    int64_t max_deg = 0;
    for (int64_t n = 0; n < Nn; ++n) max_deg = std::max(max_deg, node_ptr[n + 1] - node_ptr[n]);
    g.max_deg = int(max_deg);
    std::vector<uint8_t> &tgt = g.tgt;
    if (max_deg <= 255) {
        tgt.resize(Ne * 64);
        parallel_for(Ne, [&](int64_t b, int64_t e_end) {
            for (int64_t e = b; e < e_end; ++e)
                for (int a = 0; a < 8; ++a) {
                    const int64_t k = kpos[e * 8 + a], n = conn[8 * e + a];
                    for (int c = 0; c < 8; ++c) tgt[k * 8 + c] = uint8_t(bslot[e * 64 + a * 8 + c] - node_ptr[n]);
                }
        });
    }
    std::vector<int64_t> &blk_ptr = g.blk_ptr;
    blk_ptr.assign(nnzb + 1, 0);
    for (int64_t i = 0; i < Ne * 64; ++i) blk_ptr[bslot[i] + 1]++;
    for (int64_t k = 0; k < nnzb; ++k) blk_ptr[k + 1] += blk_ptr[k];
    std::vector<int32_t> &blk_src = g.blk_src;
    blk_src.resize(Ne * 64);
    {
        std::vector<int64_t> fill(blk_ptr.begin(), blk_ptr.end() - 1);
        // contribution (e, a, b) lives in element row block kpos[e*8+a], column block b
        for (int64_t i = 0; i < Ne * 64; ++i) blk_src[fill[bslot[i]]++] = kpos[i >> 3] * 8 + int32_t(i & 7);
    }

    // scalar CSR row starts: the nd rows of node n share the node's block list
    std::vector<int64_t> &row_ptr = g.row_ptr;
    row_ptr.resize(g.N + 1);
    for (int64_t n = 0; n < Nn; ++n) {
        int64_t deg = node_ptr[n + 1] - node_ptr[n];
        for (int c = 0; c < nd; ++c) row_ptr[nd * n + c] = int64_t(nd) * nd * node_ptr[n] + int64_t(c) * nd * deg;
    }
    row_ptr[g.N] = g.nnz;

    // symmetric block layout: the upper blocks of node n are the tail of its sorted
    // neighbour list, starting at the diagonal block
    std::vector<int64_t> &up_base = g.up_base;
    up_base.assign(Nn + 1, 0);
    for (int64_t n = 0; n < Nn; ++n) up_base[n + 1] = up_base[n] + (node_ptr[n + 1] - bdiag[n]);
    std::vector<int32_t> &lo_val = g.lo_val;
    lo_val.assign(nnzb, -1);
    parallel_for(Nn, [&](int64_t b, int64_t e) {
        for (int64_t n = b; n < e; ++n)
            for (int64_t k = node_ptr[n]; k < bdiag[n]; ++k) {  // lower blocks (n, m), m < n
                const int64_t m = node_nb[k];
                lo_val[k] = int32_t(up_base[m] + (mirror[k] - bdiag[m]));
            }
    });
    g.nnzb_up = up_base[Nn];
    {  // 16-bit neighbour offsets for the SpMV when the numbering keeps neighbours close
        bool fits = true;
        std::vector<int16_t> dnb(nnzb);
        for (int64_t n = 0; n < Nn && fits; ++n)
            for (int64_t k = node_ptr[n]; k < node_ptr[n + 1]; ++k) {
                const int64_t dd = int64_t(node_nb[k]) - n;
                if (dd < -32768 || dd > 32767) {
                    fits = false;
                    break;
                }
                dnb[k] = int16_t(dd);
            }
        if (fits) g.dnb = std::move(dnb);
    }
    // Dirichlet bits of every block's column node (one load per neighbour in the gather)
    g.nb_bits.assign(nnzb, 0);
    if (!mask.empty())
        for (int64_t k = 0; k < nnzb; ++k)
            for (int c = 0; c < nd; ++c) g.nb_bits[k] |= uint8_t((mask[int64_t(nd) * node_nb[k] + c] != 0) << c);
    return g;
}

void build_graph(fem_handle *h, const fem_mesh_desc *d) {
    HostGraph hg = host_graph(d, h->m.host_mask);
    Graph &g = h->g;
    g.Nn = hg.Nn;
    g.Ne = hg.Ne;
    g.nd = hg.nd;
    g.N = hg.N;
    g.nnz = hg.nnz;
    g.nnzb = hg.nnzb;
    g.nnzb_up = hg.nnzb_up;
    g.max_deg = hg.max_deg;
    g.up_base = upload(h, hg.up_base);
    g.lo_val = upload(h, hg.lo_val);
    g.node_ptr = upload(h, hg.node_ptr);
    g.node_nb = upload(h, hg.node_nb);
    if (!hg.dnb.empty()) g.node_dnb = upload(h, hg.dnb);
    g.nb_bits = upload(h, hg.nb_bits);
    g.blk_row = upload(h, hg.blk_row);
    g.mirror = upload(h, hg.mirror);
    g.bdiag = upload(h, hg.bdiag);
    g.blk_ptr = upload(h, hg.blk_ptr);
    g.blk_src = upload(h, hg.blk_src);
    g.ne_ptr = upload(h, hg.ne_ptr);
    g.kpos = upload(h, hg.kpos);
    if (!hg.tgt.empty()) g.tgt = upload(h, hg.tgt);
    g.bslot = upload(h, hg.bslot);
    g.row_ptr = upload(h, hg.row_ptr);
}

// ------------------------------------------------------------------ external loads
// Trilinear shape functions of the HEX8 reference cube at (s0, s1, s2).
static void hex8_shape(const double s[3], double N[8], double dN[8][3]) {
    static const int sg[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                 {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
    for (int a = 0; a < 8; ++a) {
        double l0 = 0.5 * (1 + sg[a][0] * s[0]), l1 = 0.5 * (1 + sg[a][1] * s[1]), l2 = 0.5 * (1 + sg[a][2] * s[2]);
        N[a] = l0 * l1 * l2;
        dN[a][0] = 0.5 * sg[a][0] * l1 * l2;
        dN[a][1] = 0.5 * sg[a][1] * l0 * l2;
        dN[a][2] = 0.5 * sg[a][2] * l0 * l1;
    }
}

std::vector<double> host_load_vector(const fem_mesh_desc *d) {
    const int64_t Nn = d->n_nodes, Ne = d->n_elems, N = Nn * d->ndpn;
    const int nd = d->ndpn;
    std::vector<double> F(N, 0.0);
    if (d->f_nodal)
        for (int64_t i = 0; i < N; ++i) F[i] = d->f_nodal[i];
    const double gp = 1.0 / std::sqrt(3.0);
    // Neumann term of the weak form: integral of t . phi over each loaded face (2x2 Gauss).
    for (int64_t f = 0; f < d->n_traction_faces; ++f) {
        int64_t e = d->traction_faces[2 * f];
        int face = d->traction_faces[2 * f + 1];
        if (e < 0 || e >= Ne || face < 0 || face > 5) throw Error(FEM_EINVAL, "bad traction face");
        int ax = face / 2, u1 = (ax + 1) % 3, u2 = (ax + 2) % 3;
        const double *t = d->traction + nd * f;
        for (int q = 0; q < 4; ++q) {
            double s[3], N8[8], dN[8][3], a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
            s[ax] = (face & 1) ? 1.0 : -1.0;
            s[u1] = (q & 1) ? gp : -gp;
            s[u2] = (q & 2) ? gp : -gp;
            hex8_shape(s, N8, dN);
            for (int k = 0; k < 8; ++k) {
                const double *X = d->coords + 3 * int64_t(d->conn[8 * e + k]);
                for (int i = 0; i < 3; ++i) {
                    a[i] += X[i] * dN[k][u1];
                    b[i] += X[i] * dN[k][u2];
                }
            }
            double nx = a[1] * b[2] - a[2] * b[1], ny = a[2] * b[0] - a[0] * b[2], nz = a[0] * b[1] - a[1] * b[0];
            double area = std::sqrt(nx * nx + ny * ny + nz * nz);
            for (int k = 0; k < 8; ++k)
                for (int i = 0; i < nd; ++i) F[nd * int64_t(d->conn[8 * e + k]) + i] += t[i] * N8[k] * area;
        }
    }
    // body source interpolated from nodal values: integral of b_h . phi (2x2x2 Gauss)
    if (d->source_nodal) {
        for (int64_t e = 0; e < Ne; ++e) {
            for (int q = 0; q < 8; ++q) {
                double s[3] = {(q & 1) ? gp : -gp, (q & 2) ? gp : -gp, (q & 4) ? gp : -gp};
                double N8[8], dN[8][3], J[3][3] = {{0}};
                hex8_shape(s, N8, dN);
                for (int k = 0; k < 8; ++k) {
                    const double *X = d->coords + 3 * int64_t(d->conn[8 * e + k]);
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) J[i][j] += X[i] * dN[k][j];
                }
                double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                             J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                             J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                if (!(det > 0.0)) throw Error(FEM_EMESH, "non-positive Jacobian determinant in the source integral");
                for (int i = 0; i < nd; ++i) {
                    double bq = 0.0;
                    for (int k = 0; k < 8; ++k) bq += N8[k] * d->source_nodal[nd * int64_t(d->conn[8 * e + k]) + i];
                    for (int k = 0; k < 8; ++k) F[nd * int64_t(d->conn[8 * e + k]) + i] += det * N8[k] * bq;
                }
            }
        }
    }
    return F;
}

void build_load_vector(fem_handle *h, const fem_mesh_desc *d) {
    const int64_t N = d->n_nodes * d->ndpn;
    std::vector<double> F = host_load_vector(d);
    double nrm = 0.0;
    for (int64_t i = 0; i < N; ++i)
        if (!(d->dirichlet_mask && d->dirichlet_mask[i])) nrm += F[i] * F[i];
    h->m.fext_norm = std::sqrt(nrm);
    h->m.fext = upload(h, F);
    if (d->model == FEM_J2_PLASTIC) {  // history of the path, zero (unstressed) at the start
        const size_t bytes = size_t(d->n_elems) * 96 * sizeof(double);
        h->hist = static_cast<double *>(dev_alloc(h, bytes));
        FEM_HIP(hipMemset(h->hist, 0, bytes == 0 ? 256 : bytes));
        h->hist_partials = static_cast<double *>(dev_alloc(h, j2_partials_count(d->n_elems) * sizeof(double)));
    }
    h->red_partials = static_cast<double *>(dev_alloc(h, kRedGrid * sizeof(double)));
}

}  // namespace fem
