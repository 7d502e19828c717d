// Host-side data model of libhts: meshes, batches, multigrid hierarchies.
#pragma once
#include <cmath>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/hts.h"
#include "bc.h"
#include "common.h"
#include "mg.h"
#include "vec.h"

namespace hts {

void set_error(const std::string &msg);

// ------------------------------------------------------- device memory
struct Alloc {
    hts_allocator a{};
    hipStream_t s = nullptr;
    void *get(size_t bytes)
    {
        if (bytes == 0) return nullptr;
        void *p = nullptr;
        if (a.alloc) {
            p = a.alloc(bytes, (void *)s, a.ctx);
            if (!p) throw Error(HTS_ERR_NOMEM, "allocator returned null");
        } else {
            if (hipMalloc(&p, bytes) != hipSuccess) throw Error(HTS_ERR_NOMEM, "hipMalloc failed");
        }
        return p;
    }
    void put(void *p)
    {
        if (!p) return;
        if (a.alloc) {
            if (a.free) a.free(p, a.ctx);
        } else {
            (void)hipFree(p);
        }
    }
};

template <typename T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    Alloc *al = nullptr;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n), al(o.al) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept
    {
        if (this != &o) {
            release();
            p = o.p; n = o.n; al = o.al;
            o.p = nullptr; o.n = 0;
        }
        return *this;
    }
    ~DBuf() { release(); }
    void release()
    {
        if (p && al) al->put(p);
        p = nullptr;
        n = 0;
    }
    void alloc(Alloc *a, size_t count)
    {
        if (p && count == n) return;
        release();
        al = a;
        n = count;
        if (count) p = static_cast<T *>(a->get(count * sizeof(T)));
    }
    void zero(hipStream_t s)
    {
        if (n) HTS_HIP(hipMemsetAsync(p, 0, n * sizeof(T), s));
    }
    void upload(Alloc *a, const T *h, size_t count, hipStream_t s)
    {
        alloc(a, count);
        if (count) {
            HTS_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
            HTS_HIP(hipStreamSynchronize(s));
        }
    }
    void upload(Alloc *a, const std::vector<T> &h, hipStream_t s) { upload(a, h.data(), h.size(), s); }
};

inline TimeFnDev to_dev(const hts_timefn &f)
{
    TimeFnDev d{};
    d.kind = f.kind;
    d.c0 = f.c0; d.cx = f.cx; d.cy = f.cy; d.cz = f.cz;
    d.amp = f.amp; d.period = f.period; d.phase = f.phase;
    return d;
}

struct FaceSpec {
    int face, kind;
    hts_timefn tf;
};
struct LineSpec {
    double x, y, z0, z1;
    int kind;
    hts_timefn rate;
    double T_inj;
};
struct ColSpec {
    double x, y, z0, z1;
    hts_timefn tf;
};

// Host-built sparse source rows of one field of one instance.
struct SrcRows {
    std::vector<int64_t> rows;      // instance-local node
    std::vector<int32_t> rowptr;    // size rows+1
    std::vector<SrcEnt> ents;       // src = instance-local source index
    std::vector<SrcDev> srcs;       // inst filled at batch build
};

struct Batch;

}  // namespace hts

struct hts_mesh {
    hts_mesh_desc desc{};
    hts::Alloc alloc;
    hipStream_t stream = nullptr;
    int p = 1;
    int n[3] = {0, 0, 0};     // cells
    int N[3] = {0, 0, 0};     // nodes
    double x0[3] = {0, 0, 0}, L[3] = {0, 0, 0}, h[3] = {0, 0, 0};
    int64_t nnode = 0, ncell = 0;
    // graded (rectilinear) meshes: cell edges and node coordinates per axis
    // (host), cell sizes and node coordinates on the device
    bool graded = false;
    std::vector<double> edge[3], node[3];
    hts::DBuf<double> dh[3], dnode[3], dihz;
    // general hexahedra: node coordinates [nnode][3] (host and device)
    bool general = false;
    std::vector<double> hxyz;
    hts::DBuf<double> xyz;
    double cell_lo(int d, int i) const { return graded ? edge[d][i] : x0[d] + i * h[d]; }
    double cell_h(int d, int i) const { return graded ? edge[d][i + 1] - edge[d][i] : h[d]; }

    // materials
    bool has_mat = false;
    double rho_w = 0, mu_w = 0, c_w = 0, lambda_w = 0, g = 0, B = 0;
    std::vector<double> hk, hlam, hcT;       // cellwise k, lambda, c_T (FP64, host)
    hts::DBuf<double> k64, lam64, cT64;
    hts::DBuf<float> k32, lam32, cT32;

    // boundary data and sources
    std::vector<hts::FaceSpec> bcs[2];
    std::vector<double> vsrc;                // W/m^3 per cell (empty = none)
    std::vector<hts::LineSpec> lines;
    std::vector<hts::ColSpec> cols[2];

    // state
    hts::DBuf<double> P, T;
    double t = 0.0;
    bool has_state[2] = {false, false};
    // the two previous time levels of each field (the states before the last
    // and the second-last committed step) and those steps' sizes; hist_dt 0:
    // level n-1 not known, hist_dt2 0: level n-2 not known
    hts::DBuf<double> Pprev, Tprev, Pprev2, Tprev2;
    double hist_dt[2] = {0.0, 0.0}, hist_dt2[2] = {0.0, 0.0};
    // spectral estimates of the heat preconditioner (they depend on the
    // Darcy flux of the step that made them): dt, lmax of D^-1 A without and
    // with convection, imaginary extent; dt 0: none.  Reused by any batch
    // that builds the heat preconditioner for the same dt.
    double heat_spec[4] = {0.0, 0.0, 0.0, 0.0};

    // derived device data (rebuilt when dirty)
    bool dirty = true;
    int dmask[2] = {0, 0};
    hts::DBuf<int32_t> dcol[2], colspec[2];
    hts::DBuf<hts::TimeFnDev> coltf[2];
    std::vector<int32_t> h_dcol[2], h_colspec[2];
    // injection-line mass operator (heat)
    hts::DBuf<int32_t> lcol;
    hts::DBuf<hts::LineRow> lrows;
    hts::DBuf<hts::LineEnt> lents;
    hts::DBuf<hts::LineCol> lfcol;           // Q1: rows by column and plane (LineFlat)
    hts::DBuf<hts::LineFlat> lflat;
    std::vector<hts::SrcDev> line_srcs;      // coefficient sources (instance-local)
    bool has_lineop = false;
    // time-dependent sources per field
    hts::SrcRows src[2];
    // static loads: pressure: -rho_w g sum_c k_c int dN/dz (scaled by dt*B or 1);
    // heat: sum_c f_c int N (scaled by dt)
    hts::DBuf<double> load[2];

    std::map<std::string, std::shared_ptr<hts::Batch>> batches;   // cached solo batch

    // learned-preconditioner inputs: normalised node log-permeability and
    // the pressure Dirichlet mask (rebuilt after prepare_mesh)
    hts::DBuf<float> nn_feat;
    hts::DBuf<uint8_t> nn_mask;
    double nn_nfree = 0.0;
    bool nn_ready = false;
};

namespace hts {

void prepare_mesh(hts_mesh *m);                 // (re)build derived device data
void forget_batches(hts_mesh *m);               // drop every cached batch that holds m (solve.hip)
bool is_constrained(const hts_mesh *m, int field, int i, int j, int k);   // host, after prepare_mesh
OpDev make_op(const hts_mesh *m, int field, bool fp32, double dt, bool steady, bool mass_only);
// kernel family of a mesh: its degree, or DEGREE_HEX for general hexahedra
inline int kernel_degree(const hts_mesh *m) { return m->general ? DEGREE_HEX : m->p; }
int tile_own_x(int degree, int field);          // owned node columns per tile of the operator kernels, x
int tile_own_y(int degree, int field);          // and y
// node planes per work item of the operator kernels (force > 0: that depth)
int zc_for(const hts_mesh *M, int field, int prec, int64_t tiles, int force);

}  // namespace hts
