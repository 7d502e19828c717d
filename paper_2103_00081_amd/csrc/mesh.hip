// Meshes: creation, materials, boundary data, sources and the derived
// device data every solve uses.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

using namespace hts;

namespace hts {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

template <typename F>
static hts_status guard(F &&f)
{
    try {
        f();
        return HTS_OK;
    } catch (const Error &e) {
        set_error(e.what());
        return (hts_status)e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return HTS_ERR_NOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return HTS_ERR_ARG;
    }
}

#define ARG_CHECK(cond, msg) \
    do { if (!(cond)) throw Error(HTS_ERR_ARG, msg); } while (0)

// 1D Lagrange basis of degree p on the equispaced nodes of [0,1].
static void basis1(int p, double xi, double *N)
{
    if (p == 1) {
        N[0] = 1.0 - xi;
        N[1] = xi;
    } else {
        N[0] = 2.0 * (xi - 0.5) * (xi - 1.0);
        N[1] = -4.0 * xi * (xi - 1.0);
        N[2] = 2.0 * xi * (xi - 0.5);
    }
}

static void gauss(int nq, double *x, double *w)
{
    if (nq == 2) {
        const double a = 0.5 / std::sqrt(3.0);
        x[0] = 0.5 - a; x[1] = 0.5 + a; w[0] = w[1] = 0.5;
    } else {
        const double a = 0.5 * std::sqrt(0.6);
        x[0] = 0.5 - a; x[1] = 0.5; x[2] = 0.5 + a;
        w[0] = w[2] = 5.0 / 18.0; w[1] = 8.0 / 18.0;
    }
}

static int locate(const hts_mesh *m, int d, double x, double *xi)
{
    if (m->graded) {
        // last cell whose lower edge is <= x, within 0 .. n-1
        int lo = 0, hi = m->n[d] - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (m->edge[d][mid] <= x) lo = mid;
            else hi = mid - 1;
        }
        *xi = (x - m->edge[d][lo]) / (m->edge[d][lo + 1] - m->edge[d][lo]);
        return lo;
    }
    double s = (x - m->x0[d]) / m->h[d];
    int c = (int)std::floor(s);
    c = std::max(0, std::min(c, m->n[d] - 1));
    *xi = s - c;
    return c;
}

// Node nearest to x along axis d: round half up on uniform axes; on graded
// axes the node at the smallest distance, the higher one on a tie.
static int nearest_node(const hts_mesh *m, int d, double x)
{
    if (!m->graded) {
        const double hn = m->L[d] / (m->p * m->n[d]);
        const int c = (int)std::floor((x - m->x0[d]) / hn + 0.5);
        return std::max(0, std::min(c, m->N[d] - 1));
    }
    int best = 0;
    double bd = std::fabs(m->node[d][0] - x);
    for (int i = 1; i < m->N[d]; i++) {
        const double dd = std::fabs(m->node[d][i] - x);
        if (dd <= bd) { bd = dd; best = i; }
    }
    return best;
}

static inline int64_t node_index(const hts_mesh *m, int i, int j, int k)
{
    return (int64_t)i + (int64_t)m->N[0] * ((int64_t)j + (int64_t)m->N[1] * k);
}

bool is_constrained(const hts_mesh *m, int field, int i, int j, int k)
{
    const int dm = m->dmask[field];
    if (((dm & 1) && i == 0) || ((dm & 2) && i == m->N[0] - 1) || ((dm & 4) && j == 0) ||
        ((dm & 8) && j == m->N[1] - 1) || ((dm & 16) && k == 0) || ((dm & 32) && k == m->N[2] - 1))
        return true;
    const int packed = m->h_dcol[field].empty() ? DCOL_NONE : m->h_dcol[field][i + (int64_t)m->N[0] * j];
    const int lo = packed & 0xFFFF, hi = (packed >> 16) & 0xFFFF;
    return k >= lo && k <= hi;
}

// Segments of a vertical line [z0, z1] per cell layer.
struct Seg {
    int cz;
    double a, b;   // absolute z range
};
static std::vector<Seg> segments(const hts_mesh *m, double z0, double z1)
{
    std::vector<Seg> out;
    for (int cz = 0; cz < m->n[2]; cz++) {
        double lo = m->cell_lo(2, cz), hi = lo + m->cell_h(2, cz);
        double a = std::max(z0, lo), b = std::min(z1, hi);
        if (b > a) out.push_back({cz, a, b});
    }
    return out;
}

static void build_sources(hts_mesh *m)
{
    const int p = m->p, n1 = p + 1;
    for (int f = 0; f < 2; f++) {
        std::map<int64_t, std::map<int, double>> acc;   // node -> (src -> w)
        std::vector<SrcDev> srcs;
        auto add_src = [&](const hts_timefn &tf, double scale, int posonly) {
            SrcDev s{};
            s.tf = to_dev(tf);
            s.scale = scale;
            s.posonly = posonly;
            s.inst = 0;
            srcs.push_back(s);
            return (int)srcs.size() - 1;
        };
        // line sources
        for (const LineSpec &ln : m->lines) {
            int sid = -1;
            double L = ln.z1 - ln.z0;
            if (f == 0 && ln.kind == HTS_LINE_WELL) sid = add_src(ln.rate, 1.0 / L, 0);
            if (f == 1 && ln.kind == HTS_LINE_HEAT) sid = add_src(ln.rate, 1.0, 0);
            if (f == 1 && ln.kind == HTS_LINE_WELL) sid = add_src(ln.rate, m->c_w * ln.T_inj / L, 1);
            if (sid < 0) continue;
            double xi, eta;
            int cx = locate(m, 0, ln.x, &xi), cy = locate(m, 1, ln.y, &eta);
            double Bx[3], By[3];
            basis1(p, xi, Bx);
            basis1(p, eta, By);
            double gx[3], gw[3];
            gauss(n1, gx, gw);
            for (const Seg &sg : segments(m, ln.z0, ln.z1)) {
                double zlo = m->cell_lo(2, sg.cz), hz = m->cell_h(2, sg.cz);
                double Iz[3] = {0, 0, 0};
                for (int q = 0; q < n1; q++) {
                    double z = sg.a + (sg.b - sg.a) * gx[q];
                    double Bz[3];
                    basis1(p, (z - zlo) / hz, Bz);
                    for (int s = 0; s < n1; s++) Iz[s] += gw[q] * (sg.b - sg.a) * Bz[s];
                }
                for (int az = 0; az < n1; az++)
                    for (int ay = 0; ay < n1; ay++)
                        for (int ax = 0; ax < n1; ax++) {
                            double w = Bx[ax] * By[ay] * Iz[az];
                            if (w == 0.0) continue;
                            acc[node_index(m, p * cx + ax, p * cy + ay, p * sg.cz + az)][sid] += w;
                        }
            }
        }
        // Neumann faces: value = -flux
        for (const FaceSpec &fs : m->bcs[f]) {
            if (fs.kind != HTS_BC_NEUMANN) continue;
            int sid = add_src(fs.tf, -1.0, 0);
            const int dn = fs.face / 2, side = fs.face % 2;
            const int d1 = (dn + 1) % 3, d2 = (dn + 2) % 3;
            // int_0^h N_a: Q1 h/2, h/2; Q2 h/6, 2h/3, h/6
            double U[3];
            for (int a = 0; a < n1; a++) U[a] = (p == 1) ? 0.5 : (a == 1 ? 2.0 / 3.0 : 1.0 / 6.0);
            const int cn = side ? m->n[dn] - 1 : 0, an = side ? p : 0;
            for (int c2 = 0; c2 < m->n[d2]; c2++)
                for (int c1 = 0; c1 < m->n[d1]; c1++)
                    for (int a2 = 0; a2 < n1; a2++)
                        for (int a1 = 0; a1 < n1; a1++) {
                            const double I1a = U[a1] * m->cell_h(d1, c1), I2a = U[a2] * m->cell_h(d2, c2);
                            int idx[3];
                            idx[dn] = p * cn + an;
                            idx[d1] = p * c1 + a1;
                            idx[d2] = p * c2 + a2;
                            acc[node_index(m, idx[0], idx[1], idx[2])][sid] += I1a * I2a;
                        }
        }
        SrcRows &R = m->src[f];
        R.rows.clear(); R.rowptr.assign(1, 0); R.ents.clear();
        R.srcs = srcs;
        for (auto &kv : acc) {
            R.rows.push_back(kv.first);
            for (auto &e : kv.second) {
                SrcEnt se{};
                se.src = e.first;
                se.w = e.second;
                R.ents.push_back(se);
            }
            R.rowptr.push_back((int32_t)R.ents.size());
        }
    }
}

static void build_line_operator(hts_mesh *m)
{
    const int p = m->p, n1 = p + 1;
    m->line_srcs.clear();
    // (column, k) -> (col node, src) -> w
    std::map<std::pair<int64_t, int>, std::map<std::pair<int64_t, int>, double>> rows;
    for (const LineSpec &ln : m->lines) {
        if (ln.kind != HTS_LINE_WELL) continue;
        SrcDev s{};
        s.tf = to_dev(ln.rate);
        s.scale = m->c_w / (ln.z1 - ln.z0);
        s.posonly = 1;
        int sid = (int)m->line_srcs.size();
        m->line_srcs.push_back(s);
        double xi, eta;
        int cx = locate(m, 0, ln.x, &xi), cy = locate(m, 1, ln.y, &eta);
        double Bx[3], By[3];
        basis1(p, xi, Bx);
        basis1(p, eta, By);
        double gx[3], gw[3];
        gauss(n1, gx, gw);
        for (const Seg &sg : segments(m, ln.z0, ln.z1)) {
            double zlo = m->cell_lo(2, sg.cz), hz = m->cell_h(2, sg.cz);
            double Mz[3][3] = {{0}};
            for (int q = 0; q < n1; q++) {
                double z = sg.a + (sg.b - sg.a) * gx[q];
                double Bz[3];
                basis1(p, (z - zlo) / hz, Bz);
                for (int s1 = 0; s1 < n1; s1++)
                    for (int t1 = 0; t1 < n1; t1++) Mz[s1][t1] += gw[q] * (sg.b - sg.a) * Bz[s1] * Bz[t1];
            }
            for (int az = 0; az < n1; az++)
                for (int ay = 0; ay < n1; ay++)
                    for (int ax = 0; ax < n1; ax++) {
                        int I = p * cx + ax, J = p * cy + ay, K = p * sg.cz + az;
                        int64_t colid = I + (int64_t)m->N[0] * J;
                        for (int bz = 0; bz < n1; bz++)
                            for (int by = 0; by < n1; by++)
                                for (int bx = 0; bx < n1; bx++) {
                                    double w = Bx[ax] * By[ay] * Bx[bx] * By[by] * Mz[az][bz];
                                    if (w == 0.0) continue;
                                    int64_t cn = node_index(m, p * cx + bx, p * cy + by, p * sg.cz + bz);
                                    rows[{colid, K}][{cn, sid}] += w;
                                }
                    }
        }
    }
    m->has_lineop = !rows.empty();
    if (!m->has_lineop) {
        m->lcol.release(); m->lrows.release(); m->lents.release();
        m->lfcol.release(); m->lflat.release();
        return;
    }
    std::vector<int32_t> lcol((size_t)m->N[0] * m->N[1], -1);
    std::vector<LineRow> lr;
    std::vector<LineEnt> le;
    for (auto &kv : rows) {
        LineRow r{};
        r.col = (int32_t)kv.first.first;
        r.k = kv.first.second;
        int i = (int)(kv.first.first % m->N[0]), j = (int)(kv.first.first / m->N[0]);
        r.row_constrained = is_constrained(m, 1, i, j, r.k);
        r.beg = (int32_t)le.size();
        for (auto &e : kv.second) {
            LineEnt en{};
            en.col = (int32_t)e.first.first;
            en.src = e.first.second;
            int64_t c = e.first.first;
            int ci = (int)(c % m->N[0]), cj = (int)((c / m->N[0]) % m->N[1]), ck = (int)(c / ((int64_t)m->N[0] * m->N[1]));
            en.col_constrained = is_constrained(m, 1, ci, cj, ck);
            en.w = e.second;
            le.push_back(en);
        }
        r.end = (int32_t)le.size();
        if (lcol[r.col] < 0) lcol[r.col] = (int32_t)lr.size();
        lr.push_back(r);
    }
    // Q1: the same rows by column and plane with entries as node offsets
    // (all within one node along each axis for Q1 lines); kept only when
    // every row fits LINE_MAXE entries
    m->lfcol.release();
    m->lflat.release();
    if (p == 1) {
        std::vector<LineCol> hdr((size_t)m->N[0] * m->N[1], LineCol{-1, 0, -1, 0});
        std::vector<LineFlat> flat;
        bool ok = true;
        for (size_t a = 0; a < lr.size() && ok;) {
            size_t b = a;
            while (b < lr.size() && lr[b].col == lr[a].col) b++;
            LineCol &h = hdr[lr[a].col];
            h.first = (int32_t)flat.size();
            h.kmin = lr[a].k;
            h.kmax = lr[b - 1].k;
            flat.resize(flat.size() + (size_t)(h.kmax - h.kmin + 1));
            const int i = lr[a].col % m->N[0], j = lr[a].col / m->N[0];
            for (size_t r = a; r < b && ok; r++) {
                LineFlat &f = flat[(size_t)h.first + (lr[r].k - h.kmin)];
                f.row_constrained = lr[r].row_constrained;
                for (int e = lr[r].beg; e < lr[r].end; e++) {
                    const int64_t c = le[e].col;
                    const int ci = (int)(c % m->N[0]), cj = (int)((c / m->N[0]) % m->N[1]),
                              ck = (int)(c / ((int64_t)m->N[0] * m->N[1]));
                    const int dx = ci - i, dy = cj - j, dk = ck - lr[r].k;
                    if (f.n >= LINE_MAXE || dx < -1 || dx > 1 || dy < -1 || dy > 1 || dk < -1 || dk > 1) {
                        ok = false;
                        break;
                    }
                    f.off[f.n] = (uint8_t)((dx + 1) | (dy + 1) << 2 | (dk + 1) << 4);
                    f.src[f.n] = le[e].src;
                    f.w[f.n] = le[e].w;
                    f.n++;
                }
            }
            a = b;
        }
        if (ok) {
            m->lfcol.upload(&m->alloc, hdr, m->stream);
            m->lflat.upload(&m->alloc, flat, m->stream);
        }
    }
    LineRow sent{};
    sent.col = -1;
    sent.k = 1 << 30;
    lr.push_back(sent);
    m->lcol.upload(&m->alloc, lcol, m->stream);
    m->lrows.upload(&m->alloc, lr, m->stream);
    m->lents.upload(&m->alloc, le, m->stream);
}

void prepare_mesh(hts_mesh *m)
{
    if (!m->dirty) return;
    if (!m->has_mat) throw Error(HTS_ERR_STATE, "materials not set");
    const int64_t ncol = (int64_t)m->N[0] * m->N[1];
    for (int f = 0; f < 2; f++) {
        int dm = 0;
        for (const FaceSpec &fs : m->bcs[f])
            if (fs.kind == HTS_BC_DIRICHLET) dm |= 1 << fs.face;
        m->dmask[f] = dm;
        m->h_dcol[f].clear();
        m->h_colspec[f].clear();
        std::vector<TimeFnDev> tfs;
        if (!m->cols[f].empty()) {
            m->h_dcol[f].assign(ncol, DCOL_NONE);
            m->h_colspec[f].assign(ncol, -1);
            const double tol = 1e-9 * m->L[2];
            for (size_t s = 0; s < m->cols[f].size(); s++) {
                const ColSpec &c = m->cols[f][s];
                const int ci = nearest_node(m, 0, c.x), cj = nearest_node(m, 1, c.y);
                int lo = -1, hi = -1;
                for (int k = 0; k < m->N[2]; k++) {
                    const double z = m->node[2][k];
                    if (z >= c.z0 - tol && z <= c.z1 + tol) {
                        if (lo < 0) lo = k;
                        hi = k;
                    }
                }
                if (lo < 0) continue;
                int64_t cc = ci + (int64_t)m->N[0] * cj;
                int old = m->h_dcol[f][cc];
                int olo = old & 0xFFFF, ohi = (old >> 16) & 0xFFFF;
                if (olo <= ohi) {
                    if (hi < olo - 1 || lo > ohi + 1)
                        throw Error(HTS_ERR_UNSUPPORTED, "disjoint Dirichlet columns on one node column");
                    lo = std::min(lo, olo);
                    hi = std::max(hi, ohi);
                }
                m->h_dcol[f][cc] = lo | (hi << 16);
                m->h_colspec[f][cc] = (int32_t)tfs.size();
                tfs.push_back(to_dev(c.tf));
            }
            m->dcol[f].upload(&m->alloc, m->h_dcol[f], m->stream);
            m->colspec[f].upload(&m->alloc, m->h_colspec[f], m->stream);
            m->coltf[f].upload(&m->alloc, tfs, m->stream);
        } else {
            m->dcol[f].release();
            m->colspec[f].release();
            m->coltf[f].release();
        }
    }
    build_line_operator(m);
    build_sources(m);
    // static loads
    for (int f = 0; f < 2; f++) m->load[f].alloc(&m->alloc, m->nnode);
    OpDev op = make_op(m, 0, false, 1.0, true, false);
    {
        std::vector<double> beta(m->ncell);
        for (int64_t c = 0; c < m->ncell; c++) beta[c] = -m->rho_w * m->g * m->hk[c];
        DBuf<double> db;
        db.upload(&m->alloc, beta, m->stream);
        launch_cell_loads(op, nullptr, db.p, m->load[0].p, m->stream);
        if (!m->vsrc.empty()) {
            DBuf<double> da;
            da.upload(&m->alloc, m->vsrc, m->stream);
            launch_cell_loads(op, da.p, nullptr, m->load[1].p, m->stream);
            HTS_HIP(hipStreamSynchronize(m->stream));
        } else {
            m->load[1].zero(m->stream);
        }
        HTS_HIP(hipStreamSynchronize(m->stream));
    }
    forget_batches(m);
    m->dirty = false;
    m->nn_ready = false;
}

OpDev make_op(const hts_mesh *m, int field, bool fp32, double dt, bool steady, bool mass_only)
{
    OpDev o{};
    o.nx = m->n[0]; o.ny = m->n[1]; o.nz = m->n[2];
    o.NX = m->N[0]; o.NY = m->N[1]; o.NZ = m->N[2];
    o.p = m->p;
    o.dmask = m->dmask[field];
    o.hx = m->h[0]; o.hy = m->h[1]; o.hz = m->h[2];
    o.hxs = m->graded ? m->dh[0].p : nullptr;
    o.hys = m->graded ? m->dh[1].p : nullptr;
    o.hzs = m->graded ? m->dh[2].p : nullptr;
    o.ihzs = m->graded ? m->dihz.p : nullptr;
    o.zn = m->graded ? m->dnode[2].p : nullptr;
    o.rho_g = m->rho_w * m->g;
    o.field = field;
    o.nnode = m->nnode;
    o.off = 0;
    if (field == 0) {
        o.cm = steady ? 0.0 : 1.0;
        o.cs = steady ? 1.0 : dt * m->B;
        if (mass_only) { o.cm = 1.0; o.cs = 0.0; }
        o.cadv = 0.0;
    } else {
        o.cm = 1.0;
        o.cs = mass_only ? 0.0 : dt;
        o.cadv = mass_only ? 0.0 : dt * m->c_w;
    }
    o.k = fp32 ? (const void *)m->k32.p : (const void *)m->k64.p;
    o.lam = fp32 ? (const void *)m->lam32.p : (const void *)m->lam64.p;
    o.cT = fp32 ? (const void *)m->cT32.p : (const void *)m->cT64.p;
    o.P = nullptr;
    o.dcol = m->dcol[field].p;
    o.lcol = (field == 1 && m->has_lineop && !mass_only) ? m->lcol.p : nullptr;
    o.lrows = m->lrows.p;
    o.lents = m->lents.p;
    o.lfcol = (o.lcol && m->lfcol.p) ? m->lfcol.p : nullptr;
    o.lflat = m->lflat.p;
    o.lcoef = nullptr;
    o.xyz = m->general ? m->xyz.p : nullptr;
    {
        const double V = o.hx * o.hy * o.hz, cw8 = o.cadv * V * 0.125;
        o.q1m = V / 216.0;
        o.q1x = o.cs * (o.hy * o.hz / o.hx) / 36.0;
        o.q1y = o.cs * (o.hx * o.hz / o.hy) / 36.0;
        o.q1z = o.cs * (o.hx * o.hy / o.hz) / 36.0;
        o.q1vx = -cw8 / (o.hx * o.hx);
        o.q1vy = -cw8 / (o.hy * o.hy);
        o.q1vz = -cw8 / (o.hz * o.hz);
    }
    return o;
}

}  // namespace hts

// =================================================================== C ABI
extern "C" {

const char *hts_last_error(void) { return g_err.c_str(); }

void hts_default_opts(hts_solver_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->mode = HTS_MODE_FP64;
    o->rtol = 1e-8;
    o->max_iter = 500;
    o->gmres_restart = 30;
    o->cheb_degree = 2;
    o->mg_coarse_max = 600;
    o->heat_cheb_degree = 0;
    o->inner_rtol = 1e-5;
    o->check_every = 1;
    o->use_graph = 0;
    o->nn = nullptr;
    o->verbose = 0;
    o->heat_precond = 1;
    o->extrapolate = 2;
}

// General hexahedra: det J > 0 at the 2 x 2 x 2 Gauss points of every cell
// (the points the operators integrate at), and all coordinates finite.
static void check_hex_cells(const double *xyz, const int n[3])
{
    const int NX = n[0] + 1, NY = n[1] + 1;
    const int64_t nnode = (int64_t)NX * NY * (n[2] + 1);
    const double g[2] = {0.21132486540518711775, 0.78867513459481288225};
    for (int64_t i = 0; i < 3 * nnode; i++) ARG_CHECK(std::isfinite(xyz[i]), "node coordinates must be finite");
    for (int cz = 0; cz < n[2]; cz++)
        for (int cy = 0; cy < n[1]; cy++)
            for (int cx = 0; cx < n[0]; cx++) {
                double X[8][3];
                for (int a = 0; a < 8; a++) {
                    const int64_t nd = (int64_t)(cx + (a & 1)) + (int64_t)NX * ((cy + ((a >> 1) & 1)) +
                                                                                (int64_t)NY * (cz + (a >> 2)));
                    for (int d = 0; d < 3; d++) X[a][d] = xyz[3 * nd + d];
                }
                for (int q = 0; q < 8; q++) {
                    const double p3[3] = {g[q & 1], g[(q >> 1) & 1], g[q >> 2]};
                    double J[3][3] = {{0.0}};
                    for (int a = 0; a < 8; a++)
                        for (int j = 0; j < 3; j++) {
                            double r = 1.0;
                            for (int d = 0; d < 3; d++) {
                                const int ad = (a >> d) & 1;
                                r *= d == j ? (ad ? 1.0 : -1.0) : (ad ? p3[d] : 1.0 - p3[d]);
                            }
                            for (int i = 0; i < 3; i++) J[i][j] += X[a][i] * r;
                        }
                    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                    ARG_CHECK(det > 0.0, "a hexahedron is inverted or degenerate (det J <= 0 at a Gauss point)");
                }
            }
}

hts_status hts_create_mesh(const hts_mesh_desc *desc, hts_mesh **out)
{
    return guard([&] {
        ARG_CHECK(desc && out, "null argument");
        ARG_CHECK(desc->degree == 1 || desc->degree == 2, "degree must be 1 or 2");
        bool graded = false;
        for (int d = 0; d < 3; d++) {
            ARG_CHECK(desc->ncells[d] >= 1, "ncells must be >= 1");
            ARG_CHECK(desc->extent[d] > 0.0, "extent must be > 0");
            ARG_CHECK((int64_t)desc->degree * desc->ncells[d] + 1 < 65535, "too many nodes along an axis");
            if (const double *e = desc->edges[d]) {
                graded = true;
                const double tol = 1e-9 * desc->extent[d];
                ARG_CHECK(std::fabs(e[0] - desc->origin[d]) <= tol &&
                              std::fabs(e[desc->ncells[d]] - (desc->origin[d] + desc->extent[d])) <= tol,
                          "graded axis must span [origin, origin + extent]");
                for (int i = 0; i < desc->ncells[d]; i++)
                    ARG_CHECK(e[i + 1] > e[i], "cell edges must increase strictly");
            }
        }
        {
            // the operator kernels address an instance's vectors with 32-bit
            // byte offsets: one FP64 vector of the mesh stays below 4 GiB
            int64_t nn = 1;
            for (int d = 0; d < 3; d++) nn *= (int64_t)desc->degree * desc->ncells[d] + 1;
            ARG_CHECK(nn < (int64_t)1 << 29, "mesh too large: 2^29 nodes or more");
        }
        if (desc->coords) {
            ARG_CHECK(desc->degree == 1, "node coordinates (general hexahedra) need degree 1");
            ARG_CHECK(!graded, "give either node coordinates or graded edges");
            check_hex_cells(desc->coords, desc->ncells);
        }
        HTS_HIP(hipSetDevice(desc->device));
        std::unique_ptr<hts_mesh> m(new hts_mesh());
        m->desc = *desc;
        m->alloc.a = desc->alloc;
        m->stream = (hipStream_t)desc->stream;
        m->alloc.s = m->stream;
        m->p = desc->degree;
        m->nnode = 1;
        m->ncell = 1;
        for (int d = 0; d < 3; d++) {
            m->n[d] = desc->ncells[d];
            m->N[d] = m->p * m->n[d] + 1;
            m->x0[d] = desc->origin[d];
            m->L[d] = desc->extent[d];
            m->h[d] = m->L[d] / m->n[d];
            m->nnode *= m->N[d];
            m->ncell *= m->n[d];
        }
        // node coordinates of every axis; graded meshes keep their edges and
        // upload the cell sizes and node coordinates
        m->graded = graded;
        for (int d = 0; d < 3; d++) {
            m->edge[d].resize(m->n[d] + 1);
            for (int i = 0; i <= m->n[d]; i++)
                m->edge[d][i] = desc->edges[d] ? desc->edges[d][i] : m->x0[d] + i * m->h[d];
            if (desc->edges[d]) {
                m->edge[d][0] = m->x0[d];
                m->edge[d][m->n[d]] = m->x0[d] + m->L[d];
            }
            // nodes: the cell edges, and for degree 2 also the cell midpoints
            m->node[d].resize(m->N[d]);
            const double hn = m->L[d] / (m->p * m->n[d]);
            for (int i = 0; i < m->N[d]; i++) {
                if (!graded) m->node[d][i] = m->x0[d] + i * hn;
                else if (m->p == 1) m->node[d][i] = m->edge[d][i];
                else m->node[d][i] = (i & 1) ? 0.5 * (m->edge[d][i / 2] + m->edge[d][i / 2 + 1]) : m->edge[d][i / 2];
            }
            m->desc.edges[d] = nullptr;   // the caller's array is not kept
        }
        if (graded) {
            for (int d = 0; d < 3; d++) {
                std::vector<double> hs(m->n[d]);
                for (int i = 0; i < m->n[d]; i++) hs[i] = m->edge[d][i + 1] - m->edge[d][i];
                m->dh[d].upload(&m->alloc, hs, m->stream);
                m->dnode[d].upload(&m->alloc, m->node[d], m->stream);
                if (d == 2) {
                    for (double &v : hs) v = 1.0 / v;
                    m->dihz.upload(&m->alloc, hs, m->stream);
                }
            }
            HTS_HIP(hipStreamSynchronize(m->stream));
        }
        if (desc->coords) {
            m->general = true;
            m->hxyz.assign(desc->coords, desc->coords + 3 * m->nnode);
            m->xyz.upload(&m->alloc, m->hxyz, m->stream);
            m->desc.coords = nullptr;   // the caller's array is not kept
        }
        m->P.alloc(&m->alloc, m->nnode);
        m->T.alloc(&m->alloc, m->nnode);
        m->Pprev.alloc(&m->alloc, m->nnode);
        m->Tprev.alloc(&m->alloc, m->nnode);
        m->Pprev2.alloc(&m->alloc, m->nnode);
        m->Tprev2.alloc(&m->alloc, m->nnode);
        m->P.zero(m->stream);
        m->T.zero(m->stream);
        m->Pprev.zero(m->stream);
        m->Tprev.zero(m->stream);
        m->Pprev2.zero(m->stream);
        m->Tprev2.zero(m->stream);
        *out = m.release();
    });
}

void hts_destroy_mesh(hts_mesh *m)
{
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    try {
        forget_batches(m);
    } catch (...) {
    }
    delete m;
}

hts_status hts_mesh_sizes(const hts_mesh *m, int64_t *nnode, int64_t *ncell)
{
    return guard([&] {
        ARG_CHECK(m, "null mesh");
        if (nnode) *nnode = m->nnode;
        if (ncell) *ncell = m->ncell;
    });
}

hts_status hts_set_materials(hts_mesh *m, const hts_materials *mat)
{
    return guard([&] {
        ARG_CHECK(m && mat, "null argument");
        ARG_CHECK(mat->porosity || (mat->lambda_bulk && mat->rhoc_bulk), "porosity required");
        ARG_CHECK(mat->permeability || mat->hydraulic_conductivity, "permeability or conductivity required");
        ARG_CHECK(mat->rho_w > 0 && mat->mu_w > 0 && mat->c_w > 0 && mat->g > 0, "water constants must be > 0");
        ARG_CHECK(mat->lambda_bulk || (mat->lambda_solid && mat->lambda_w >= 0), "conductivities required");
        ARG_CHECK(mat->rhoc_bulk || mat->rhoc_solid, "heat capacities required");
        HTS_HIP(hipSetDevice(m->desc.device));
        const int64_t C = m->ncell;
        m->rho_w = mat->rho_w; m->mu_w = mat->mu_w; m->c_w = mat->c_w;
        m->lambda_w = mat->lambda_w; m->g = mat->g; m->B = mat->B_poro;
        m->hk.resize(C); m->hlam.resize(C); m->hcT.resize(C);
        for (int64_t c = 0; c < C; c++) {
            // mobility k = K_i / mu_w = K / (rho_w g)
            m->hk[c] = mat->permeability ? mat->permeability[c] / mat->mu_w
                                         : mat->hydraulic_conductivity[c] / (mat->rho_w * mat->g);
            const double phi = mat->porosity ? mat->porosity[c] : 0.0;
            // mixture rules
            m->hlam[c] = mat->lambda_bulk ? mat->lambda_bulk[c]
                                          : (1.0 - phi) * mat->lambda_solid[c] + phi * mat->lambda_w;
            m->hcT[c] = mat->rhoc_bulk ? mat->rhoc_bulk[c] : (1.0 - phi) * mat->rhoc_solid[c] + phi * mat->c_w;
            if (!std::isfinite(m->hk[c]) || !std::isfinite(m->hlam[c]) || !std::isfinite(m->hcT[c]) ||
                m->hk[c] < 0 || m->hcT[c] <= 0 || m->hlam[c] < 0)
                throw Error(HTS_ERR_ARG, "invalid material value in cell " + std::to_string(c));
        }
        m->k64.upload(&m->alloc, m->hk, m->stream);
        m->lam64.upload(&m->alloc, m->hlam, m->stream);
        m->cT64.upload(&m->alloc, m->hcT, m->stream);
        std::vector<float> f(C);
        for (int64_t c = 0; c < C; c++) f[c] = (float)m->hk[c];
        m->k32.upload(&m->alloc, f, m->stream);
        for (int64_t c = 0; c < C; c++) f[c] = (float)m->hlam[c];
        m->lam32.upload(&m->alloc, f, m->stream);
        for (int64_t c = 0; c < C; c++) f[c] = (float)m->hcT[c];
        m->cT32.upload(&m->alloc, f, m->stream);
        m->has_mat = true;
        m->dirty = true;
        m->heat_spec[0] = 0.0;   // operator data changed: the heat spectrum is estimated again
    });
}

hts_status hts_set_face_bc(hts_mesh *m, hts_field field, int32_t face, int32_t kind, const hts_timefn *value)
{
    return guard([&] {
        ARG_CHECK(m, "null mesh");
        ARG_CHECK(field == 0 || field == 1, "bad field");
        ARG_CHECK(face >= 0 && face < 6, "face must be 0..5");
        ARG_CHECK(kind == HTS_BC_DIRICHLET || kind == HTS_BC_NEUMANN || kind == HTS_BC_NONE, "bad kind");
        ARG_CHECK(kind == HTS_BC_NONE || value, "null value");
        if (kind == HTS_BC_NEUMANN) {
            ARG_CHECK(value->cx == 0 && value->cy == 0 && value->cz == 0, "Neumann flux must be spatially constant");
            if (m->general) throw Error(HTS_ERR_UNSUPPORTED, "Neumann faces need a box mesh");
        }
        if (value) ARG_CHECK(value->kind >= 0 && value->kind <= 2, "bad time function kind");
        if (value && value->kind != 0) ARG_CHECK(value->period > 0, "period must be > 0");
        auto &v = m->bcs[field];
        v.erase(std::remove_if(v.begin(), v.end(), [&](const FaceSpec &f) { return f.face == face; }), v.end());
        if (kind != HTS_BC_NONE) v.push_back({face, kind, *value});
        m->dirty = true;
        m->heat_spec[0] = 0.0;   // operator data changed: the heat spectrum is estimated again
    });
}

hts_status hts_set_volume_source(hts_mesh *m, const double *w)
{
    return guard([&] {
        ARG_CHECK(m, "null mesh");
        if (w) m->vsrc.assign(w, w + m->ncell);
        else m->vsrc.clear();
        m->dirty = true;
        m->heat_spec[0] = 0.0;   // operator data changed: the heat spectrum is estimated again
    });
}

hts_status hts_add_line_source(hts_mesh *m, double x, double y, double z0, double z1, int32_t kind,
                               const hts_timefn *rate, double T_inj)
{
    return guard([&] {
        ARG_CHECK(m && rate, "null argument");
        ARG_CHECK(kind == HTS_LINE_HEAT || kind == HTS_LINE_WELL, "bad line kind");
        ARG_CHECK(z1 > z0, "z1 must exceed z0");
        ARG_CHECK(rate->cx == 0 && rate->cy == 0 && rate->cz == 0, "line rate must be spatially constant");
        ARG_CHECK(rate->kind == 0 || rate->period > 0, "period must be > 0");
        if (m->general) throw Error(HTS_ERR_UNSUPPORTED, "line sources need a box mesh (vertical node columns)");
        m->lines.push_back({x, y, z0, z1, kind, *rate, T_inj});
        m->dirty = true;
        m->heat_spec[0] = 0.0;   // operator data changed: the heat spectrum is estimated again
    });
}

hts_status hts_add_dirichlet_column(hts_mesh *m, hts_field field, double x, double y, double z0, double z1,
                                    const hts_timefn *value)
{
    return guard([&] {
        ARG_CHECK(m && value, "null argument");
        ARG_CHECK(field == 0 || field == 1, "bad field");
        ARG_CHECK(z1 >= z0, "z1 must not be below z0");
        if (m->general) throw Error(HTS_ERR_UNSUPPORTED, "Dirichlet columns need a box mesh (vertical node columns)");
        m->cols[field].push_back({x, y, z0, z1, *value});
        m->dirty = true;
        m->heat_spec[0] = 0.0;   // operator data changed: the heat spectrum is estimated again
    });
}

hts_status hts_set_state(hts_mesh *m, hts_field field, const double *host, double t)
{
    return guard([&] {
        ARG_CHECK(m && host, "null argument");
        ARG_CHECK(field == 0 || field == 1, "bad field");
        for (int64_t i = 0; i < m->nnode; i++)
            if (!std::isfinite(host[i])) throw Error(HTS_ERR_ARG, "non-finite state value");
        HTS_HIP(hipSetDevice(m->desc.device));
        DBuf<double> &s = field == 0 ? m->P : m->T;
        HTS_HIP(hipMemcpyAsync(s.p, host, m->nnode * sizeof(double), hipMemcpyHostToDevice, m->stream));
        HTS_HIP(hipStreamSynchronize(m->stream));
        m->t = t;
        m->has_state[field] = true;
        m->hist_dt[field] = m->hist_dt2[field] = 0.0;   // the previous levels no longer belong to this state
    });
}

hts_status hts_set_previous_state(hts_mesh *m, hts_field field, int32_t level, const double *host, double dt_prev)
{
    return guard([&] {
        ARG_CHECK(m, "null mesh");
        ARG_CHECK(field == 0 || field == 1, "bad field");
        ARG_CHECK(level == 1 || level == 2, "level must be 1 or 2");
        ARG_CHECK(std::isfinite(dt_prev) && dt_prev >= 0.0, "dt_prev must be finite and >= 0");
        ARG_CHECK(host || dt_prev == 0.0, "null values with dt_prev > 0");
        ARG_CHECK(level == 1 || dt_prev == 0.0 || m->hist_dt[field] > 0.0, "level 2 needs level 1 first");
        HTS_HIP(hipSetDevice(m->desc.device));
        if (dt_prev > 0.0) {
            for (int64_t i = 0; i < m->nnode; i++)
                if (!std::isfinite(host[i])) throw Error(HTS_ERR_ARG, "non-finite state value");
            DBuf<double> &s = field == 0 ? (level == 1 ? m->Pprev : m->Pprev2) : (level == 1 ? m->Tprev : m->Tprev2);
            HTS_HIP(hipMemcpyAsync(s.p, host, m->nnode * sizeof(double), hipMemcpyHostToDevice, m->stream));
            HTS_HIP(hipStreamSynchronize(m->stream));
        }
        if (level == 1) {
            m->hist_dt[field] = dt_prev;
            m->hist_dt2[field] = 0.0;   // level 2 belongs to the old level 1
        } else {
            m->hist_dt2[field] = dt_prev;
        }
    });
}

hts_status hts_get_heat_spectrum(hts_mesh *m, double *out)
{
    return guard([&] {
        ARG_CHECK(m && out, "null argument");
        for (int k = 0; k < 4; k++) out[k] = m->heat_spec[k];
    });
}

hts_status hts_set_heat_spectrum(hts_mesh *m, const double *in)
{
    return guard([&] {
        ARG_CHECK(m && in, "null argument");
        for (int k = 0; k < 4; k++) ARG_CHECK(std::isfinite(in[k]) && in[k] >= 0.0, "bad spectrum entry");
        ARG_CHECK(in[0] == 0.0 || (in[1] > 0.0 && in[2] > 0.0), "lmax estimates must be > 0");
        for (int k = 0; k < 4; k++) m->heat_spec[k] = in[k];
    });
}

hts_status hts_get_previous_state(hts_mesh *m, hts_field field, int32_t level, double *host, double *dt_prev)
{
    return guard([&] {
        ARG_CHECK(m, "null mesh");
        ARG_CHECK(field == 0 || field == 1, "bad field");
        ARG_CHECK(level == 1 || level == 2, "level must be 1 or 2");
        HTS_HIP(hipSetDevice(m->desc.device));
        const double dt = level == 1 ? m->hist_dt[field] : m->hist_dt2[field];
        if (host && dt > 0.0) {
            DBuf<double> &s = field == 0 ? (level == 1 ? m->Pprev : m->Pprev2) : (level == 1 ? m->Tprev : m->Tprev2);
            HTS_HIP(hipMemcpyAsync(host, s.p, m->nnode * sizeof(double), hipMemcpyDeviceToHost, m->stream));
            HTS_HIP(hipStreamSynchronize(m->stream));
        }
        if (dt_prev) *dt_prev = dt;
    });
}

hts_status hts_get_state(hts_mesh *m, hts_field field, double *host, double *t)
{
    return guard([&] {
        ARG_CHECK(m, "null mesh");
        ARG_CHECK(field == 0 || field == 1, "bad field");
        HTS_HIP(hipSetDevice(m->desc.device));
        if (host) {
            DBuf<double> &s = field == 0 ? m->P : m->T;
            HTS_HIP(hipMemcpyAsync(host, s.p, m->nnode * sizeof(double), hipMemcpyDeviceToHost, m->stream));
            HTS_HIP(hipStreamSynchronize(m->stream));
        }
        if (t) *t = m->t;
    });
}

}  // extern "C"

namespace hts {
hts_status guard_call(const std::function<void()> &f) { return guard(f); }
}
