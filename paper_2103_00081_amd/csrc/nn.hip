// Learned preconditioner: a 3D convolutional encoder-decoder that maps a
// normalised pressure residual and the node log-permeability to an error
// estimate, trained on (residual, error) pairs harvested from the
// library's own multigrid-CG pressure solves (Eq. 3 systems), and used as the
// preconditioner of flexible CG with the V-cycle as fallback.
//
// Network (levels L, widths c_0..c_{L-1}; every convolution 3x3x3, zero
// padding 1): enc0a in->c0, enc0b c0->c0 (gives e_0); for l = 1..L-1 a
// stride-2 down_l c_{l-1}->c_l and enc_l c_l->c_l (gives e_l); for l = L-2..0
// dec_l c_{l+1}->c_l on the linearly upsampled d_{l+1} (d_{L-1} = e_{L-1}),
// d_l = relu(dec_l(up d_{l+1})) + e_l; out c0->1 without activation.
// Activations and weights are BF16 (channels-last), accumulation FP32, FP32
// master weights with Adam.  Stored channel counts are padded to multiples
// of 8 (input 2 -> 8, output 1 -> 8) with zero weights.
#include <atomic>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <tuple>

#include "internal.h"
#include "nnk.h"
#include "solve.h"

namespace hts {
hts_status guard_call(const std::function<void()> &f);

namespace {

int up8(int c) { return (c + 7) / 8 * 8; }
int up16(int c) { return (c + 15) / 16 * 16; }
int up32(int c) { return (c + 31) / 32 * 32; }

uint16_t host_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFF) ? 0x40 : 0));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

}  // namespace

struct NNLayer {
    int cin = 0, cout = 0, stride = 1, relu = 1;   // logical channels
    int cinp = 0, coutp = 0;                       // stored channels
    int rows = 0, kp = 0, trows = 0, ktp = 0;      // padded weight shapes
    int lin = 0, lout = 0;                         // resolution levels
    DBuf<float> w, b, mw, vw, mb, vb, gw, gb;
    DBuf<uint16_t> wbf, wt;
};

struct NNWork {
    Dims d[4];
    int64_t n[4] = {0, 0, 0, 0};
    DBuf<uint16_t> x0, G, tgt, rbf;
    std::vector<DBuf<uint16_t>> y, dsum, up;
    DBuf<float> out, gy, gA, gB, partial, feat;
    std::vector<DBuf<float>> ge;
    DBuf<double> lpart;
    DBuf<uint8_t> mask;
};

}  // namespace hts

struct hts_nn {
    hts_nn_desc desc{};
    hts::Alloc al;
    hipStream_t s = nullptr;
    int L = 4;
    int ch[4] = {16, 32, 48, 64};
    std::vector<hts::NNLayer> layers;
    std::map<std::tuple<int, int, int>, std::unique_ptr<hts::NNWork>> work;
    int adam_step = 0;
    double gamma = 1.0;   // target scale: network output * gamma ~ error / rms(residual)
    hts::DBuf<double> dgamma;   // gamma on the device (read by the preconditioner's output kernel)
    bool gamma_set = false;   // gamma fixed (first train call, or loaded)
    uint64_t serial = 0;      // unique per network object (keys captured graphs)
    // harvested pairs (all of one node grid); targets of pairs [0, nscaled)
    // are divided by gamma already, later ones are not yet
    hts::Dims dd{};
    int64_t npairs = 0, cap = 0, nscaled = 0;
    std::vector<int> pair_draw;
    std::vector<double> pair_scale;
    hts::DBuf<uint16_t> pr, pt;
    std::vector<hts::DBuf<float>> dfeat;
    std::vector<hts::DBuf<uint8_t>> dmask;
    std::vector<double> dnfree;
};

namespace hts {

// ------------------------------------------------------------- structure
static void build_layers(hts_nn *nn)
{
    const int L = nn->L;
    auto add = [&](int cin, int cout, int stride, int relu, int lin, int lout) {
        NNLayer Ly;
        Ly.cin = cin; Ly.cout = cout; Ly.stride = stride; Ly.relu = relu;
        Ly.cinp = up8(cin); Ly.coutp = up8(cout);
        Ly.rows = up16(Ly.coutp);
        Ly.kp = up32(27 * Ly.cinp);
        Ly.trows = up16(Ly.cinp);
        Ly.ktp = up32(27 * Ly.coutp);
        Ly.lin = lin; Ly.lout = lout;
        nn->layers.push_back(std::move(Ly));
    };
    add(2, nn->ch[0], 1, 1, 0, 0);
    add(nn->ch[0], nn->ch[0], 1, 1, 0, 0);
    for (int l = 1; l < L; l++) {
        add(nn->ch[l - 1], nn->ch[l], 2, 1, l - 1, l);
        add(nn->ch[l], nn->ch[l], 1, 1, l, l);
    }
    for (int l = L - 2; l >= 0; l--) add(nn->ch[l + 1], nn->ch[l], 1, 1, l, l);
    add(nn->ch[0], 1, 1, 0, 0, 0);
    for (NNLayer &Ly : nn->layers) {
        const size_t nw = (size_t)Ly.rows * Ly.kp;
        Ly.w.alloc(&nn->al, nw); Ly.mw.alloc(&nn->al, nw); Ly.vw.alloc(&nn->al, nw); Ly.gw.alloc(&nn->al, nw);
        Ly.b.alloc(&nn->al, Ly.rows); Ly.mb.alloc(&nn->al, Ly.rows); Ly.vb.alloc(&nn->al, Ly.rows);
        Ly.gb.alloc(&nn->al, Ly.rows);
        Ly.wbf.alloc(&nn->al, nw);
        Ly.wt.alloc(&nn->al, (size_t)Ly.trows * Ly.ktp);
        Ly.w.zero(nn->s); Ly.mw.zero(nn->s); Ly.vw.zero(nn->s); Ly.gw.zero(nn->s);
        Ly.b.zero(nn->s); Ly.mb.zero(nn->s); Ly.vb.zero(nn->s); Ly.gb.zero(nn->s);
        Ly.wbf.zero(nn->s); Ly.wt.zero(nn->s);
    }
}

static int64_t n_params(const hts_nn *nn)
{
    int64_t t = 0;
    for (const NNLayer &Ly : nn->layers) t += (int64_t)Ly.cout * Ly.cin * 27 + Ly.cout;
    return t;
}

// BF16 copies and transposes of the FP32 master weights
static void refresh_weights(hts_nn *nn, hipStream_t s)
{
    for (NNLayer &Ly : nn->layers) {
        nn_f32_to_bf16(Ly.w.p, (int64_t)Ly.rows * Ly.kp, Ly.wbf.p, s);
        nn_transpose_w(Ly.wbf.p, Ly.coutp, Ly.cinp, Ly.kp, Ly.wt.p, Ly.ktp, s);
    }
}

// parameters in the exchange layout: per layer W[cout][cin][kz][ky][kx], b[cout]
static void set_params(hts_nn *nn, const double *theta)
{
    int64_t o = 0;
    for (NNLayer &Ly : nn->layers) {
        std::vector<float> w((size_t)Ly.rows * Ly.kp, 0.0f), b((size_t)Ly.rows, 0.0f);
        for (int co = 0; co < Ly.cout; co++)
            for (int ci = 0; ci < Ly.cin; ci++)
                for (int tap = 0; tap < 27; tap++) {
                    const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                    w[(size_t)co * Ly.kp + tap * Ly.cinp + ci] =
                        (float)theta[o + (((int64_t)co * Ly.cin + ci) * 3 + dz) * 9 + dy * 3 + dx];
                }
        o += (int64_t)Ly.cout * Ly.cin * 27;
        for (int co = 0; co < Ly.cout; co++) b[co] = (float)theta[o + co];
        o += Ly.cout;
        HTS_HIP(hipMemcpyAsync(Ly.w.p, w.data(), w.size() * 4, hipMemcpyHostToDevice, nn->s));
        HTS_HIP(hipMemcpyAsync(Ly.b.p, b.data(), b.size() * 4, hipMemcpyHostToDevice, nn->s));
        HTS_HIP(hipStreamSynchronize(nn->s));
    }
    refresh_weights(nn, nn->s);
    HTS_HIP(hipStreamSynchronize(nn->s));
}

// which = 0: parameters, 1: gradients
static void get_params(const hts_nn *nn, double *theta, int which)
{
    int64_t o = 0;
    for (const NNLayer &Ly : nn->layers) {
        std::vector<float> w((size_t)Ly.rows * Ly.kp), b((size_t)Ly.rows);
        HTS_HIP(hipMemcpyAsync(w.data(), which ? Ly.gw.p : Ly.w.p, w.size() * 4, hipMemcpyDeviceToHost, nn->s));
        HTS_HIP(hipMemcpyAsync(b.data(), which ? Ly.gb.p : Ly.b.p, b.size() * 4, hipMemcpyDeviceToHost, nn->s));
        HTS_HIP(hipStreamSynchronize(nn->s));
        for (int co = 0; co < Ly.cout; co++)
            for (int ci = 0; ci < Ly.cin; ci++)
                for (int tap = 0; tap < 27; tap++) {
                    const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                    theta[o + (((int64_t)co * Ly.cin + ci) * 3 + dz) * 9 + dy * 3 + dx] =
                        w[(size_t)co * Ly.kp + tap * Ly.cinp + ci];
                }
        o += (int64_t)Ly.cout * Ly.cin * 27;
        for (int co = 0; co < Ly.cout; co++) theta[o + co] = b[co];
        o += Ly.cout;
    }
}

static void init_params(hts_nn *nn)
{
    std::mt19937_64 rng(nn->desc.seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<double> th((size_t)n_params(nn));
    int64_t o = 0;
    const size_t nl = nn->layers.size();
    for (size_t k = 0; k < nl; k++) {
        const NNLayer &Ly = nn->layers[k];
        const double sd = std::sqrt(2.0 / (27.0 * Ly.cin)) * (k + 1 == nl ? 0.1 : 1.0);
        for (int64_t i = 0; i < (int64_t)Ly.cout * Ly.cin * 27; i++) th[o + i] = sd * nd(rng);
        o += (int64_t)Ly.cout * Ly.cin * 27;
        for (int co = 0; co < Ly.cout; co++) th[o + co] = 0.0;
        o += Ly.cout;
    }
    set_params(nn, th.data());
}

// ------------------------------------------------------------- workspace
static NNWork &workspace(hts_nn *nn, Dims d0)
{
    auto key = std::make_tuple(d0.x, d0.y, d0.z);
    auto it = nn->work.find(key);
    if (it != nn->work.end()) return *it->second;
    auto W = std::make_unique<NNWork>();
    const int L = nn->L;
    W->d[0] = d0;
    for (int l = 1; l < L; l++)
        W->d[l] = Dims{(W->d[l - 1].x - 1) / 2 + 1, (W->d[l - 1].y - 1) / 2 + 1, (W->d[l - 1].z - 1) / 2 + 1};
    for (int l = 0; l < L; l++) W->n[l] = W->d[l].n();
    Alloc *al = &nn->al;
    const int64_t n0 = W->n[0];
    W->x0.alloc(al, (size_t)n0 * 8);
    const size_t nl = nn->layers.size();
    W->y.resize(nl);
    int64_t gmax = 0, pmax = 0, abmax = 0;
    for (size_t k = 0; k + 1 < nl; k++) {
        const NNLayer &Ly = nn->layers[k];
        W->y[k].alloc(al, (size_t)W->n[Ly.lout] * Ly.coutp);
    }
    for (size_t k = 0; k < nl; k++) {
        const NNLayer &Ly = nn->layers[k];
        gmax = std::max(gmax, W->n[Ly.lout] * Ly.coutp);
        pmax = std::max(pmax, (nn_bwd_weight_chunks(W->d[Ly.lout]) + SUM_GROUPS) * (int64_t)Ly.coutp * Ly.kp);
        abmax = std::max(abmax, W->n[Ly.lout] * (int64_t)Ly.coutp);
        abmax = std::max(abmax, W->n[Ly.lin] * (int64_t)Ly.cinp);
    }
    W->dsum.resize(L);
    W->up.resize(L);
    W->ge.resize(L);
    for (int l = 0; l < L; l++) {
        W->ge[l].alloc(al, (size_t)W->n[l] * nn->ch[l]);
        if (l < L - 1) {
            W->dsum[l].alloc(al, (size_t)W->n[l] * nn->ch[l]);
            W->up[l].alloc(al, (size_t)W->n[l] * nn->ch[l + 1]);
        }
    }
    W->G.alloc(al, (size_t)gmax);
    W->gA.alloc(al, (size_t)abmax);
    W->gB.alloc(al, (size_t)abmax);
    W->partial.alloc(al, (size_t)std::max<int64_t>(pmax, (n0 + 511) / 512 * 64));
    W->out.alloc(al, (size_t)n0 * 8);
    W->gy.alloc(al, (size_t)n0 * 8);
    W->lpart.alloc(al, (size_t)nn_loss_blocks(n0));
    W->tgt.alloc(al, (size_t)n0);
    W->rbf.alloc(al, (size_t)n0);
    W->mask.alloc(al, (size_t)n0);
    W->feat.alloc(al, (size_t)n0);
    NNWork &ref = *W;
    nn->work[key] = std::move(W);
    return ref;
}

static const uint16_t *e_of(const NNWork &W, int l) { return W.y[2 * l + 1].p; }
static const uint16_t *d_of(const hts_nn *nn, const NNWork &W, int l)
{
    return l == nn->L - 1 ? e_of(W, l) : W.dsum[l].p;
}

static void conv(hts_nn *nn, NNWork &W, int k, const uint16_t *X, uint16_t *Ybf, float *Yf, hipStream_t s,
                 const int32_t *gate = nullptr)
{
    const NNLayer &Ly = nn->layers[k];
    nn_conv_fwd(X, Ly.cinp, W.d[Ly.lin], Ly.wbf.p, Ly.kp, Ly.b.p, Ly.coutp, W.d[Ly.lout], Ly.stride, Ly.relu, nullptr,
                Ybf, Yf, Ly.coutp, s, gate);
}

// out [n0][8] (FP32, channel 0 meaningful) from x0; gate: optional device
// flag that switches every launch off
static void forward(hts_nn *nn, NNWork &W, hipStream_t s, const int32_t *gate = nullptr)
{
    const int L = nn->L;
    conv(nn, W, 0, W.x0.p, W.y[0].p, nullptr, s, gate);
    conv(nn, W, 1, W.y[0].p, W.y[1].p, nullptr, s, gate);
    for (int l = 1; l < L; l++) {
        conv(nn, W, 2 * l, W.y[2 * l - 1].p, W.y[2 * l].p, nullptr, s, gate);
        conv(nn, W, 2 * l + 1, W.y[2 * l].p, W.y[2 * l + 1].p, nullptr, s, gate);
    }
    for (int l = L - 2; l >= 0; l--) {
        const int k = 3 * L - 2 - l;
        nn_upsample(d_of(nn, W, l + 1), W.d[l + 1], nn->ch[l + 1], W.up[l].p, W.d[l], s, gate);
        conv(nn, W, k, W.up[l].p, W.y[k].p, nullptr, s, gate);
        nn_add_bf16(W.y[k].p, e_of(W, l), W.n[l] * nn->ch[l], W.dsum[l].p, s, gate);
    }
    conv(nn, W, 3 * L - 1, W.dsum[0].p, nullptr, W.out.p, s, gate);
}

// weight and bias gradients from gy (FP32 [n0][8]); acc = add to the stored ones
static void backward(hts_nn *nn, NNWork &W, int acc, hipStream_t s)
{
    const int L = nn->L;
    auto bw = [&](int k, const float *gout, const uint16_t *yrelu, const uint16_t *X, float *gx) {
        NNLayer &Ly = nn->layers[k];
        const int64_t nout = W.n[Ly.lout];
        nn_relu_mask(gout, Ly.relu ? yrelu : nullptr, nout * Ly.coutp, W.G.p, s);
        nn_conv_bwd_weight(W.G.p, Ly.coutp, W.d[Ly.lout], X, Ly.cinp, W.d[Ly.lin], Ly.stride, W.partial.p, Ly.kp,
                           Ly.gw.p, acc, s);
        nn_bias_grad(W.G.p, nout, Ly.coutp, W.partial.p, Ly.gb.p, acc, s);
        if (gx)
            nn_conv_bwd_data(W.G.p, Ly.coutp, W.d[Ly.lout], Ly.wt.p, Ly.ktp, Ly.cinp, W.d[Ly.lin], Ly.stride, gx, s);
    };
    bw(3 * L - 1, W.gy.p, nullptr, W.dsum[0].p, W.gA.p);                      // gA = grad d_0
    for (int l = 0; l <= L - 2; l++) {
        const int k = 3 * L - 2 - l;
        HTS_HIP(hipMemcpyAsync(W.ge[l].p, W.gA.p, sizeof(float) * W.n[l] * nn->ch[l], hipMemcpyDeviceToDevice, s));
        bw(k, W.gA.p, W.y[k].p, W.up[l].p, W.gB.p);                           // gB = grad up_l
        nn_upsample_adj(W.gB.p, W.d[l], nn->ch[l + 1], W.gA.p, W.d[l + 1], s);  // gA = grad d_{l+1}
    }
    HTS_HIP(hipMemcpyAsync(W.ge[L - 1].p, W.gA.p, sizeof(float) * W.n[L - 1] * nn->ch[L - 1],
                           hipMemcpyDeviceToDevice, s));
    for (int l = L - 1; l >= 1; l--) {
        bw(2 * l + 1, W.ge[l].p, W.y[2 * l + 1].p, W.y[2 * l].p, W.gA.p);       // gA = grad of down_l output
        bw(2 * l, W.gA.p, W.y[2 * l].p, W.y[2 * l - 1].p, W.gB.p);             // gB = grad e_{l-1}
        nn_add_f32(W.ge[l - 1].p, W.gB.p, W.n[l - 1] * nn->ch[l - 1], s);
    }
    bw(1, W.ge[0].p, W.y[1].p, W.y[0].p, W.gA.p);
    bw(0, W.gA.p, W.y[0].p, W.x0.p, nullptr);
}

static double loss(hts_nn *nn, NNWork &W, const uint16_t *tgt, const uint8_t *mask, double nfree, hipStream_t s)
{
    const int64_t n0 = W.n[0];
    nn_loss(W.out.p, 8, tgt, mask, n0, 1.0 / std::max(1.0, nfree), W.gy.p, W.lpart.p, s);
    std::vector<double> h((size_t)nn_loss_blocks(n0));
    HTS_HIP(hipMemcpyAsync(h.data(), W.lpart.p, h.size() * 8, hipMemcpyDeviceToHost, s));
    HTS_HIP(hipStreamSynchronize(s));
    double t = 0.0;
    for (double v : h) t += v;
    return t / std::max(1.0, nfree);
}

static void adam(hts_nn *nn, double lr, int batch, hipStream_t s)
{
    nn->adam_step++;
    const float gs = 1.0f / (float)std::max(1, batch);
    for (NNLayer &Ly : nn->layers) {
        nn_adam(Ly.w.p, Ly.mw.p, Ly.vw.p, Ly.gw.p, (int64_t)Ly.rows * Ly.kp, (float)lr, 0.9f, 0.999f, 1e-8f,
                nn->adam_step, gs, Ly.wbf.p, nullptr, s);
        nn_adam(Ly.b.p, Ly.mb.p, Ly.vb.p, Ly.gb.p, Ly.rows, (float)lr, 0.9f, 0.999f, 1e-8f, nn->adam_step, gs, nullptr,
                nullptr, s);
        nn_transpose_w(Ly.wbf.p, Ly.coutp, Ly.cinp, Ly.kp, Ly.wt.p, Ly.ktp, s);
    }
}

// ------------------------------------------------- per-mesh network inputs
// Node feature: mean log10 k of the cells around the node, standardised over
// the mesh; mask: pressure Dirichlet nodes.
static void mesh_inputs(hts_mesh *m, std::vector<float> &feat, std::vector<uint8_t> &mask, double &nfree)
{
    prepare_mesh(m);
    const int64_t nn_ = m->nnode;
    feat.assign((size_t)nn_, 0.0f);
    mask.assign((size_t)nn_, 0);
    std::vector<double> f((size_t)nn_);
    double mean = 0.0;
    for (int k = 0; k < m->N[2]; k++)
        for (int j = 0; j < m->N[1]; j++)
            for (int i = 0; i < m->N[0]; i++) {
                int c0[3], c1[3];
                const int ijk[3] = {i, j, k};
                for (int a = 0; a < 3; a++) {
                    c0[a] = std::max(0, std::min(m->n[a] - 1, (ijk[a] - 1) / m->p));
                    c1[a] = std::max(0, std::min(m->n[a] - 1, ijk[a] / m->p));
                    if (ijk[a] == 0) c0[a] = 0;
                }
                double s = 0.0;
                int cnt = 0;
                for (int cz = c0[2]; cz <= c1[2]; cz++)
                    for (int cy = c0[1]; cy <= c1[1]; cy++)
                        for (int cx = c0[0]; cx <= c1[0]; cx++) {
                            const double kc = m->hk[(size_t)cx + (size_t)m->n[0] * (cy + (size_t)m->n[1] * cz)];
                            s += std::log10(std::max(kc, 1e-300));
                            cnt++;
                        }
                const int64_t v = (int64_t)i + (int64_t)m->N[0] * (j + (int64_t)m->N[1] * k);
                f[v] = s / cnt;
                mean += f[v];
                mask[v] = is_constrained(m, 0, i, j, k) ? 1 : 0;
            }
    mean /= (double)nn_;
    double var = 0.0;
    for (double v : f) var += (v - mean) * (v - mean);
    const double sd = std::sqrt(var / (double)nn_);
    for (int64_t v = 0; v < nn_; v++) feat[v] = sd > 1e-6 ? (float)((f[v] - mean) / sd) : 0.0f;
    nfree = 0.0;
    for (uint8_t b : mask) nfree += b ? 0.0 : 1.0;
}

static void ensure_mesh_inputs(hts_mesh *m)
{
    prepare_mesh(m);
    if (m->nn_ready) return;
    std::vector<float> feat;
    std::vector<uint8_t> mask;
    mesh_inputs(m, feat, mask, m->nn_nfree);
    m->nn_feat.upload(&m->alloc, feat, m->stream);
    m->nn_mask.upload(&m->alloc, mask, m->stream);
    m->nn_ready = true;
}

// --------------------------------------------- preconditioner in a solve
// Network inputs and workspaces of every instance of the batch, so that the
// preconditioner itself allocates nothing (it may be captured in a graph).
void nn_prepare(hts_nn *nn, Batch &B)
{
    for (int i = 0; i < B.n; i++) {
        hts_mesh *m = B.m[i];
        ensure_mesh_inputs(m);
        (void)workspace(nn, Dims{m->N[0], m->N[1], m->N[2]});
    }
}

uint64_t nn_serial(const hts_nn *nn) { return nn->serial; }

// z (instance slice) = gamma rms(r) Net(r / rms(r), feature), zero on
// Dirichlet rows; rms(r)^2 = S[inst][S_RR] / (free nodes).  gate: device
// flag of the instance (0: every launch returns at once, z untouched).
void nn_precondition(hts_nn *nn, Batch &B, int inst, const double *r, double *z, const int32_t *gate)
{
    hts_mesh *m = B.m[inst];
    ensure_mesh_inputs(m);
    NNWork &W = workspace(nn, Dims{m->N[0], m->N[1], m->N[2]});
    const int64_t off = B.off[inst], n = m->nnode;
    const double *rr = B.S.p + (int64_t)inst * NSLOT + S_RR;
    nn_pack_input_dev(r + off, rr, m->nn_nfree, m->nn_feat.p, n, W.x0.p, B.s, gate);
    forward(nn, W, B.s, gate);
    nn_unpack_output_dev(W.out.p, 8, rr, m->nn_nfree, nn->dgamma.p, m->nn_mask.p, n, z + off, B.s, gate);
}

// gamma on the host and on the device
static void set_gamma(hts_nn *nn, double g)
{
    nn->gamma = g;
    nn->dgamma.upload(&nn->al, &nn->gamma, 1, nn->s);
}

}  // namespace hts

using namespace hts;

extern "C" {

hts_status hts_nn_create(const hts_nn_desc *desc, hts_nn **out)
{
    if (out) *out = nullptr;
    return guard_call([&] {
        if (!desc || !out) throw Error(HTS_ERR_ARG, "null argument");
        if (desc->levels < 2 || desc->levels > 4) throw Error(HTS_ERR_ARG, "levels must be 2..4");
        for (int l = 0; l < desc->levels; l++)
            if (desc->channels[l] < 8 || desc->channels[l] > 64 || desc->channels[l] % 8)
                throw Error(HTS_ERR_ARG, "channels must be multiples of 8 in [8, 64]");
        HTS_HIP(hipSetDevice(desc->device));
        auto nn = std::make_unique<hts_nn>();
        nn->desc = *desc;
        nn->s = (hipStream_t)desc->stream;
        nn->al.s = nn->s;
        nn->L = desc->levels;
        for (int l = 0; l < 4; l++) nn->ch[l] = l < desc->levels ? desc->channels[l] : 0;
        build_layers(nn.get());
        init_params(nn.get());
        static std::atomic<uint64_t> next_serial{1};
        nn->serial = next_serial++;
        set_gamma(nn.get(), 1.0);
        *out = nn.release();
    });
}

void hts_nn_destroy(hts_nn *nn)
{
    if (!nn) return;
    (void)hipStreamSynchronize(nn->s);
    delete nn;
}

hts_status hts_nn_num_params(const hts_nn *nn, int64_t *count)
{
    return guard_call([&] {
        if (!nn || !count) throw Error(HTS_ERR_ARG, "null argument");
        *count = n_params(nn);
    });
}

hts_status hts_nn_set_params(hts_nn *nn, const double *theta, int64_t count)
{
    return guard_call([&] {
        if (!nn || !theta) throw Error(HTS_ERR_ARG, "null argument");
        if (count != n_params(nn)) throw Error(HTS_ERR_ARG, "parameter count mismatch");
        set_params(nn, theta);
    });
}

hts_status hts_nn_get_params(const hts_nn *nn, double *theta, int64_t count)
{
    return guard_call([&] {
        if (!nn || !theta) throw Error(HTS_ERR_ARG, "null argument");
        if (count != n_params(nn)) throw Error(HTS_ERR_ARG, "parameter count mismatch");
        get_params(nn, theta, 0);
    });
}

hts_status hts_nn_eval(hts_nn *nn, const int32_t dims[3], const float *input, const float *target,
                       const uint8_t *mask, float *out, double *loss_out, double *grad)
{
    return guard_call([&] {
        if (!nn || !dims || !input || !out) throw Error(HTS_ERR_ARG, "null argument");
        if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) throw Error(HTS_ERR_ARG, "bad dims");
        if ((grad || loss_out) && !target) throw Error(HTS_ERR_ARG, "loss and gradient need a target");
        const Dims d0{dims[0], dims[1], dims[2]};
        NNWork &W = workspace(nn, d0);
        const int64_t n = d0.n();
        std::vector<uint16_t> x((size_t)n * 8, 0);
        for (int64_t v = 0; v < n; v++) {
            x[(size_t)v * 8] = host_bf16(input[2 * v]);
            x[(size_t)v * 8 + 1] = host_bf16(input[2 * v + 1]);
        }
        hipStream_t s = nn->s;
        HTS_HIP(hipMemcpyAsync(W.x0.p, x.data(), x.size() * 2, hipMemcpyHostToDevice, s));
        forward(nn, W, s);
        std::vector<float> y((size_t)n * 8);
        HTS_HIP(hipMemcpyAsync(y.data(), W.out.p, y.size() * 4, hipMemcpyDeviceToHost, s));
        HTS_HIP(hipStreamSynchronize(s));
        for (int64_t v = 0; v < n; v++) out[v] = y[(size_t)v * 8];
        if (!target) return;
        std::vector<uint16_t> t((size_t)n);
        std::vector<uint8_t> mk((size_t)n, 0);
        double nfree = 0.0;
        for (int64_t v = 0; v < n; v++) {
            t[v] = host_bf16(target[v]);
            mk[v] = mask ? mask[v] : 0;
            nfree += mk[v] ? 0.0 : 1.0;
        }
        HTS_HIP(hipMemcpyAsync(W.tgt.p, t.data(), t.size() * 2, hipMemcpyHostToDevice, s));
        HTS_HIP(hipMemcpyAsync(W.mask.p, mk.data(), mk.size(), hipMemcpyHostToDevice, s));
        const double lv = loss(nn, W, W.tgt.p, W.mask.p, nfree, s);
        if (loss_out) *loss_out = lv;
        if (grad) {
            backward(nn, W, 0, s);
            HTS_HIP(hipStreamSynchronize(s));
            get_params(nn, grad, 1);
        }
    });
}

// Single convolution layer on the matrix cores, for verification.  Host
// arrays; x, g BF16 bit patterns channels-last [voxel][channel] with x
// fastest; w BF16 [cout][cin][3][3][3]; outputs FP32.
hts_status hts_nn_conv3d(int32_t op, int32_t cin, int32_t cout, int32_t stride, const int32_t din[3],
                         const uint16_t *x, const uint16_t *w, const float *bias, const uint16_t *g, float *out,
                         float *out_bias, void *stream)
{
    return guard_call([&] {
        if (!din || !w || !out) throw Error(HTS_ERR_ARG, "null argument");
        if (cin < 8 || cout < 8 || cin > 64 || cout > 64 || cin % 8 || cout % 8)
            throw Error(HTS_ERR_ARG, "channels must be multiples of 8 in [8, 64]");
        if (stride != 1 && stride != 2) throw Error(HTS_ERR_ARG, "stride must be 1 or 2");
        if (op < 0 || op > 2) throw Error(HTS_ERR_ARG, "op must be 0, 1 or 2");
        if ((op != 1 && !x) || (op != 0 && !g)) throw Error(HTS_ERR_ARG, "missing input");
        hipStream_t s = (hipStream_t)stream;
        Alloc al;
        al.s = s;
        const Dims di{din[0], din[1], din[2]};
        const Dims dn{(din[0] - 1) / stride + 1, (din[1] - 1) / stride + 1, (din[2] - 1) / stride + 1};
        const int kp = up32(27 * cin), rows = up16(cout), ktp = up32(27 * cout), trows = up16(cin);
        std::vector<uint16_t> wd((size_t)rows * kp, 0);
        for (int co = 0; co < cout; co++)
            for (int ci = 0; ci < cin; ci++)
                for (int tap = 0; tap < 27; tap++) {
                    const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                    wd[(size_t)co * kp + tap * cin + ci] = w[(((size_t)co * cin + ci) * 3 + dz) * 9 + dy * 3 + dx];
                }
        DBuf<uint16_t> W, X, G, Wt;
        DBuf<float> B, Y, P, GB;
        W.upload(&al, wd, s);
        if (op == 0) {
            std::vector<float> bb((size_t)rows, 0.0f);
            if (bias)
                for (int co = 0; co < cout; co++) bb[co] = bias[co];
            B.upload(&al, bb, s);
            X.upload(&al, x, (size_t)di.n() * cin, s);
            Y.alloc(&al, (size_t)dn.n() * cout);
            nn_conv_fwd(X.p, cin, di, W.p, kp, B.p, cout, dn, stride, 0, nullptr, nullptr, Y.p, cout, s);
            HTS_HIP(hipMemcpyAsync(out, Y.p, Y.n * 4, hipMemcpyDeviceToHost, s));
        } else if (op == 1) {
            G.upload(&al, g, (size_t)dn.n() * cout, s);
            Wt.alloc(&al, (size_t)trows * ktp);
            nn_transpose_w(W.p, cout, cin, kp, Wt.p, ktp, s);
            Y.alloc(&al, (size_t)di.n() * cin);
            nn_conv_bwd_data(G.p, cout, dn, Wt.p, ktp, cin, di, stride, Y.p, s);
            HTS_HIP(hipMemcpyAsync(out, Y.p, Y.n * 4, hipMemcpyDeviceToHost, s));
        } else {
            G.upload(&al, g, (size_t)dn.n() * cout, s);
            X.upload(&al, x, (size_t)di.n() * cin, s);
            P.alloc(&al, (size_t)std::max<int64_t>((nn_bwd_weight_chunks(dn) + SUM_GROUPS) * cout * kp, 1));
            Y.alloc(&al, (size_t)cout * kp);
            nn_conv_bwd_weight(G.p, cout, dn, X.p, cin, di, stride, P.p, kp, Y.p, 0, s);
            std::vector<float> gw((size_t)cout * kp);
            HTS_HIP(hipMemcpyAsync(gw.data(), Y.p, gw.size() * 4, hipMemcpyDeviceToHost, s));
            HTS_HIP(hipStreamSynchronize(s));
            for (int co = 0; co < cout; co++)
                for (int ci = 0; ci < cin; ci++)
                    for (int tap = 0; tap < 27; tap++) {
                        const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                        out[(((size_t)co * cin + ci) * 3 + dz) * 9 + dy * 3 + dx] =
                            gw[(size_t)co * kp + tap * cin + ci];
                    }
            if (out_bias) {
                GB.alloc(&al, (size_t)cout);
                nn_bias_grad(G.p, dn.n(), cout, P.p, GB.p, 0, s);
                HTS_HIP(hipMemcpyAsync(out_bias, GB.p, (size_t)cout * 4, hipMemcpyDeviceToHost, s));
            }
        }
        HTS_HIP(hipStreamSynchronize(s));
    });
}

hts_status hts_nn_adam(int64_t n, int32_t step, double lr, double gscale, float *w, float *m, float *v,
                       const float *g, uint16_t *wbf, void *stream)
{
    return guard_call([&] {
        if (n < 0 || step < 1 || !(lr > 0.0) || !std::isfinite(gscale)) throw Error(HTS_ERR_ARG, "bad arguments");
        if (n > 0 && (!w || !m || !v || !g)) throw Error(HTS_ERR_ARG, "null argument");
        if (n == 0) return;
        hipStream_t s = (hipStream_t)stream;
        Alloc al;
        al.s = s;
        DBuf<float> W, M, V, G;
        DBuf<uint16_t> B;
        W.upload(&al, w, (size_t)n, s);
        M.upload(&al, m, (size_t)n, s);
        V.upload(&al, v, (size_t)n, s);
        G.upload(&al, g, (size_t)n, s);
        if (wbf) B.alloc(&al, (size_t)n);
        nn_adam(W.p, M.p, V.p, G.p, n, (float)lr, 0.9f, 0.999f, 1e-8f, step, (float)gscale, wbf ? B.p : nullptr,
                nullptr, s);
        HTS_HIP(hipMemcpyAsync(w, W.p, (size_t)n * 4, hipMemcpyDeviceToHost, s));
        HTS_HIP(hipMemcpyAsync(m, M.p, (size_t)n * 4, hipMemcpyDeviceToHost, s));
        HTS_HIP(hipMemcpyAsync(v, V.p, (size_t)n * 4, hipMemcpyDeviceToHost, s));
        if (wbf) HTS_HIP(hipMemcpyAsync(wbf, B.p, (size_t)n * 2, hipMemcpyDeviceToHost, s));
        HTS_HIP(hipStreamSynchronize(s));
    });
}

hts_status hts_nn_time_forward(hts_nn *nn, const int32_t dims[3], int32_t reps, double *ms_per_forward,
                               double *flop_per_forward)
{
    return guard_call([&] {
        if (!nn || !dims || reps < 1 || !ms_per_forward) throw Error(HTS_ERR_ARG, "bad arguments");
        const Dims d0{dims[0], dims[1], dims[2]};
        NNWork &W = workspace(nn, d0);
        hipStream_t s = nn->s;
        // input: a smooth nonzero pattern (the time does not depend on values)
        std::vector<float> ones((size_t)d0.n(), 1.0f);
        DBuf<float> f;
        f.upload(&nn->al, ones, s);
        nn_f32_to_bf16(f.p, d0.n(), W.rbf.p, s);
        nn_pack_input_bf(W.rbf.p, f.p, d0.n(), W.x0.p, s);
        forward(nn, W, s);   // warm
        hipEvent_t a, b;
        HTS_HIP(hipEventCreate(&a));
        HTS_HIP(hipEventCreate(&b));
        HTS_HIP(hipEventRecord(a, s));
        for (int r = 0; r < reps; r++) forward(nn, W, s);
        HTS_HIP(hipEventRecord(b, s));
        HTS_HIP(hipEventSynchronize(b));
        float ms = 0.0f;
        HTS_HIP(hipEventElapsedTime(&ms, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        *ms_per_forward = ms / reps;
        if (flop_per_forward) {
            // 2 flops per multiply-add of every 3x3x3 convolution (logical channels)
            double fl = 0.0;
            for (const NNLayer &Ly : nn->layers) fl += 2.0 * 27.0 * Ly.cin * Ly.cout * (double)W.n[Ly.lout];
            *flop_per_forward = fl;
        }
    });
}

hts_status hts_nn_harvest(hts_nn *nn, hts_mesh *const *meshes, int32_t n_draws, int32_t n_steps, double dt,
                          int32_t pairs_per_solve)
{
    return guard_call([&] {
        if (!nn || !meshes || n_draws < 1 || n_steps < 1 || !(dt > 0.0) || pairs_per_solve < 1)
            throw Error(HTS_ERR_ARG, "bad harvest arguments");
        const Dims d0{meshes[0]->N[0], meshes[0]->N[1], meshes[0]->N[2]};
        for (int d = 0; d < n_draws; d++) {
            if (!meshes[d]) throw Error(HTS_ERR_ARG, "null mesh");
            if (meshes[d]->N[0] != d0.x || meshes[d]->N[1] != d0.y || meshes[d]->N[2] != d0.z)
                throw Error(HTS_ERR_ARG, "all harvest meshes must have the same node grid");
            if (!meshes[d]->has_state[0]) throw Error(HTS_ERR_STATE, "pressure state not set");
        }
        if (nn->npairs > 0 && (nn->dd.x != d0.x || nn->dd.y != d0.y || nn->dd.z != d0.z))
            throw Error(HTS_ERR_ARG, "harvest grid differs from the pairs already held");
        nn->dd = d0;
        const int64_t n = d0.n();
        // capacity: every inner solve of every step, up to pairs_per_solve each,
        // with room for two inner solves per step
        const int64_t want = nn->npairs + (int64_t)n_draws * n_steps * pairs_per_solve * 2;
        if (want > nn->cap) {
            DBuf<uint16_t> r2, t2;
            r2.alloc(&nn->al, (size_t)want * n);
            t2.alloc(&nn->al, (size_t)want * n);
            if (nn->npairs) {
                HTS_HIP(hipMemcpyAsync(r2.p, nn->pr.p, (size_t)nn->npairs * n * 2, hipMemcpyDeviceToDevice, nn->s));
                HTS_HIP(hipMemcpyAsync(t2.p, nn->pt.p, (size_t)nn->npairs * n * 2, hipMemcpyDeviceToDevice, nn->s));
                HTS_HIP(hipStreamSynchronize(nn->s));
            }
            nn->pr = std::move(r2);
            nn->pt = std::move(t2);
            nn->cap = want;
        }
        hts_solver_opts o;
        hts_default_opts(&o);
        o.mode = HTS_MODE_FP64;
        o.rtol = 1e-10;
        o.max_iter = 200;
        o.extrapolate = 0;   // plain warm starts: the march does not keep time levels
        for (int d = 0; d < n_draws; d++) {
            hts_mesh *m = meshes[d];
            HTS_HIP(hipSetDevice(m->desc.device));
            const int draw = (int)nn->dfeat.size();
            {
                std::vector<float> feat;
                std::vector<uint8_t> mask;
                double nfree = 0.0;
                mesh_inputs(m, feat, mask, nfree);
                nn->dfeat.emplace_back();
                nn->dmask.emplace_back();
                nn->dfeat.back().upload(&nn->al, feat, nn->s);
                nn->dmask.back().upload(&nn->al, mask, nn->s);
                nn->dnfree.push_back(nfree);
            }
            auto Bp = solo_batch(m);
            Batch &B = *Bp;
            B.gather_state();
            const double t0 = m->t;
            // the march below advances the batch's pressure, which is the
            // mesh's own state for a single mesh: keep it and put it back
            DBuf<double> psave;
            psave.alloc(B.al, (size_t)n);
            HTS_HIP(hipMemcpyAsync(psave.p, B.Pn.p, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, B.s));
            auto restore = [&] {
                (void)hipMemcpyAsync(B.Pn.p, psave.p, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, B.s);
                (void)hipStreamSynchronize(B.s);
            };
            DBuf<double> iters, e, r;
            DBuf<float> tmp;
            iters.alloc(B.al, (size_t)(o.max_iter + 1) * n);
            e.alloc(B.al, (size_t)n);
            r.alloc(B.al, (size_t)n);
            tmp.alloc(B.al, (size_t)n);
            int nit = 0;
            B.cg_hook = [&](const double *x, int k) {
                if (k <= o.max_iter) {
                    HTS_HIP(hipMemcpyAsync(iters.p + (size_t)k * n, x, (size_t)n * 8, hipMemcpyDeviceToDevice, B.s));
                    nit = std::max(nit, k + 1);
                }
            };
            B.inner_hook = [&](const Tables &A, const double *xs) {
                // pick pairs_per_solve iterates evenly over 0 .. nit-1
                const int K = nit;
                nit = 0;
                if (K < 1) return;
                const int np = std::min(K, pairs_per_solve);
                std::vector<int32_t> one(1, 1);
                B.set_active(one);
                VecCtx v = B.vctx(false);
                for (int q = 0; q < np && nn->npairs < nn->cap; q++) {
                    const int k = np == 1 ? 0 : (int)((int64_t)q * (K - 1) / (np - 1));
                    vcopy<double>(v, xs, e.p);
                    vaxpby<double>(v, -1.0, -1, iters.p + (size_t)k * n, 1.0, -1, e.p);
                    EpiArgs<double> ep{};
                    B.apply_op<double>(A, EPI_STORE, true, e.p, r.p, ep);
                    vdot<double>(v, r.p, r.p, e.p, B.partial.p);
                    vreduce(B.rch, B.partial.p, 2, RED_STORE2, S_TMP2, B.S.p, B.active.p, 0, 0.0, nullptr, B.s);
                    B.download_S();
                    const double rr = B.hS[S_TMP2];
                    if (!(rr > 0.0) || !std::isfinite(rr)) continue;
                    // (r, e) -> (r / rms r, e / rms r), both BF16
                    const double nf = nn->dnfree[draw];
                    const double sc = std::sqrt(nf / rr);
                    vaxpby<double>(v, sc, -1, r.p, 0.0, -1, r.p);
                    vaxpby<double>(v, sc, -1, e.p, 0.0, -1, e.p);
                    vdot<double>(v, e.p, e.p, nullptr, B.partial.p);
                    vreduce(B.rch, B.partial.p, 2, RED_STORE, S_TMP3, B.S.p, B.active.p, 0, 0.0, nullptr, B.s);
                    B.download_S();
                    const double ee = B.hS[S_TMP3];
                    if (!std::isfinite(ee)) continue;
                    vconvert<double, float>(v, 1.0, -1, r.p, tmp.p);
                    nn_f32_to_bf16(tmp.p, n, nn->pr.p + (size_t)nn->npairs * n, B.s);
                    vconvert<double, float>(v, 1.0, -1, e.p, tmp.p);
                    nn_f32_to_bf16(tmp.p, n, nn->pt.p + (size_t)nn->npairs * n, B.s);
                    HTS_HIP(hipStreamSynchronize(B.s));
                    nn->pair_draw.push_back(draw);
                    nn->pair_scale.push_back(std::sqrt(ee / nf));
                    nn->npairs++;
                }
            };
            try {
                for (int st = 0; st < n_steps; st++) {
                    FieldStats fs = B.solve_pressure(dt, false, o);
                    if (fs.status[0] != HTS_OK) throw Error(fs.status[0], "harvest pressure solve failed");
                    std::vector<int32_t> one(1, 1);
                    B.set_active(one);
                    vcopy<double>(B.vctx(false), B.P1.p, B.Pn.p);
                    m->t += dt;
                }
            } catch (...) {
                B.cg_hook = nullptr;
                B.inner_hook = nullptr;
                m->t = t0;
                restore();
                throw;
            }
            B.cg_hook = nullptr;
            B.inner_hook = nullptr;
            m->t = t0;
            restore();
            HTS_HIP(hipStreamSynchronize(B.s));
        }
    });
}

hts_status hts_nn_train(hts_nn *nn, int32_t epochs, double lr, int32_t batch, int32_t val_draws,
                        hts_train_stats *out)
{
    return guard_call([&] {
        if (!nn || epochs < 0 || !(lr > 0.0) || batch < 1 || val_draws < 0) throw Error(HTS_ERR_ARG, "bad arguments");
        if (nn->npairs < 1) throw Error(HTS_ERR_STATE, "no harvested pairs");
        const int ndraw = (int)nn->dfeat.size();
        if (val_draws >= ndraw) throw Error(HTS_ERR_ARG, "no training draws left");
        const int first_val = ndraw - val_draws;
        std::vector<int64_t> tr, va;
        for (int64_t i = 0; i < nn->npairs; i++) (nn->pair_draw[i] < first_val ? tr : va).push_back(i);
        if (tr.empty()) throw Error(HTS_ERR_STATE, "no training pairs");
        // target scale: the median error-to-residual ratio of the training
        // pairs, fixed once; every pair's target is divided by it exactly once
        if (!nn->gamma_set) {
            std::vector<double> sc;
            for (int64_t i : tr) sc.push_back(nn->pair_scale[i]);
            std::nth_element(sc.begin(), sc.begin() + sc.size() / 2, sc.end());
            const double g = sc[sc.size() / 2];
            set_gamma(nn, g > 0.0 && std::isfinite(g) ? g : 1.0);
            nn->gamma_set = true;
        }
        if (nn->nscaled < nn->npairs) {
            nn_scale_bf16(nn->pt.p + (size_t)nn->nscaled * nn->dd.n(), (nn->npairs - nn->nscaled) * nn->dd.n(),
                          (float)(1.0 / nn->gamma), nn->s);
            nn->nscaled = nn->npairs;
        }
        hipStream_t s = nn->s;
        NNWork &W = workspace(nn, nn->dd);
        const int64_t n = nn->dd.n();
        auto sample = [&](int64_t i) {
            const int d = nn->pair_draw[i];
            nn_pack_input_bf(nn->pr.p + (size_t)i * n, nn->dfeat[d].p, n, W.x0.p, s);
            forward(nn, W, s);
            return loss(nn, W, nn->pt.p + (size_t)i * n, nn->dmask[d].p, nn->dnfree[d], s);
        };
        std::mt19937_64 rng(nn->desc.seed ^ 0x5eedULL);
        hts_train_stats st{};
        st.pairs = (int32_t)nn->npairs;
        for (int ep = 0; ep < epochs; ep++) {
            std::shuffle(tr.begin(), tr.end(), rng);
            double tot = 0.0;
            for (size_t b0 = 0; b0 < tr.size(); b0 += batch) {
                const size_t b1 = std::min(tr.size(), b0 + batch);
                for (size_t j = b0; j < b1; j++) {
                    tot += sample(tr[j]);
                    backward(nn, W, j > b0 ? 1 : 0, s);
                }
                adam(nn, lr, (int)(b1 - b0), s);
            }
            const double mean = tot / (double)tr.size();
            if (ep == 0) st.loss_first = mean;
            st.loss_last = mean;
            st.epochs_done = ep + 1;
        }
        double vt = 0.0;
        for (int64_t i : va) vt += sample(i);
        st.val_loss = va.empty() ? 0.0 : vt / (double)va.size();
        HTS_HIP(hipStreamSynchronize(s));
        if (out) *out = st;
    });
}

hts_status hts_nn_save(const hts_nn *nn, const char *path)
{
    return guard_call([&] {
        if (!nn || !path) throw Error(HTS_ERR_ARG, "null argument");
        std::vector<double> th((size_t)n_params(nn));
        get_params(nn, th.data(), 0);
        FILE *f = std::fopen(path, "wb");
        if (!f) throw Error(HTS_ERR_ARG, "cannot open file for writing");
        const char magic[8] = {'H', 'T', 'S', 'N', 'N', '0', '0', '1'};
        int32_t hdr[6] = {nn->L, nn->ch[0], nn->ch[1], nn->ch[2], nn->ch[3], 0};
        int64_t cnt = (int64_t)th.size();
        bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 6, f) == 6 &&
                  std::fwrite(&nn->gamma, 8, 1, f) == 1 && std::fwrite(&cnt, 8, 1, f) == 1 &&
                  std::fwrite(th.data(), 8, th.size(), f) == th.size();
        ok = (std::fclose(f) == 0) && ok;
        if (!ok) throw Error(HTS_ERR_ARG, "write failed");
    });
}

hts_status hts_nn_load(hts_nn *nn, const char *path)
{
    return guard_call([&] {
        if (!nn || !path) throw Error(HTS_ERR_ARG, "null argument");
        FILE *f = std::fopen(path, "rb");
        if (!f) throw Error(HTS_ERR_ARG, "cannot open file");
        char magic[8];
        int32_t hdr[6];
        double gamma = 1.0;
        int64_t cnt = 0;
        bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "HTSNN001", 8) == 0 &&
                  std::fread(hdr, 4, 6, f) == 6 && std::fread(&gamma, 8, 1, f) == 1 && std::fread(&cnt, 8, 1, f) == 1;
        ok = ok && hdr[0] == nn->L && hdr[1] == nn->ch[0] && hdr[2] == nn->ch[1] && hdr[3] == nn->ch[2] &&
             hdr[4] == nn->ch[3] && cnt == n_params(nn);
        std::vector<double> th;
        if (ok) {
            th.resize((size_t)cnt);
            ok = std::fread(th.data(), 8, th.size(), f) == th.size();
        }
        std::fclose(f);
        if (!ok) throw Error(HTS_ERR_ARG, "not a network file of this architecture");
        set_params(nn, th.data());
        // targets already divided by the previous gamma take the loaded one
        if (nn->nscaled > 0 && gamma != nn->gamma)
            nn_scale_bf16(nn->pt.p, nn->nscaled * nn->dd.n(), (float)(nn->gamma / gamma), nn->s);
        set_gamma(nn, gamma);
        nn->gamma_set = true;
        HTS_HIP(hipStreamSynchronize(nn->s));
    });
}

}  // extern "C"
