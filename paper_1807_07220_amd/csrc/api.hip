// Host orchestration of the C ABI declared in include/tgms.h.
//
// Setup (paper section 5, Step 2): block factors -> snapshots (section 4.1)
// -> block Gram matrices -> pencils, eigenproblems and selection (section
// 4.2) -> divergence-free coarse basis, its SPD matrix, stream functions and
// FP64 Cholesky -> smoother patch factors -> coarse RT0 operator of the
// preprocessing.  Solve (Steps 1, 3, 4): preprocessing (section 3), PCG in
// stream-function coordinates with the two-grid preconditioner (section 5),
// v = vbar + C psi, pressure.
#include <algorithm>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <string>

#include "common.h"
#include "d3.h"
#include "band.h"
#include "patch.h"

namespace tgms {
void bnd_faces(tgms_ctx* c, const double* g, double* gb);

hipEvent_t take_event(tgms_ctx* c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        HIP_OK(hipEventCreate(&e));
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// Event pairs around launches when profiling (launches are then never captured).
ProfScope::ProfScope(tgms_ctx* ctx, int kid) : c(ctx), id(kid) {
    if (!c->prof) return;
    e1 = take_event(c);
    HIP_OK(hipEventRecord(e1, c->stream));
}

ProfScope::~ProfScope() {
    if (!c->prof || !e1) return;
    hipEvent_t e2 = take_event(c);
    (void)hipEventRecord(e2, c->stream);
    c->prof_rec.push_back({id, c->prof_iter, e1, e2});
}

// order the library stream after the work queued on the caller's stream
void enter(tgms_ctx* c) {
    HIP_OK(hipEventRecord(c->ev_enter, c->user_stream));
    HIP_OK(hipStreamWaitEvent(c->stream, c->ev_enter, 0));
}

}  // namespace tgms

namespace {
struct DevPool {
    std::mutex mu;
    std::map<int, std::multimap<size_t, void*>> blocks;  // free blocks by size, per device
    std::map<int, size_t> cached;
};
DevPool& dev_pool() {
    static DevPool* p = new DevPool();  // never destroyed: no HIP calls at static destruction
    return *p;
}
constexpr size_t POOL_CAP = 16ull << 30;  // most bytes kept per device
}  // namespace

void* tgms::dev_alloc(size_t bytes, size_t* got) {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    DevPool& P = dev_pool();
    {
        std::lock_guard<std::mutex> lock(P.mu);
        auto& fl = P.blocks[dev];
        auto it = fl.lower_bound(bytes);
        // a cached block, unless it is much larger than asked for
        if (it != fl.end() && it->first <= bytes + bytes / 4 + (1u << 20)) {
            void* p = it->second;
            *got = it->first;
            P.cached[dev] -= it->first;
            fl.erase(it);
            return p;
        }
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        // return the cached blocks of this device to the runtime and try again
        std::lock_guard<std::mutex> lock(P.mu);
        for (auto& kv : P.blocks[dev]) (void)hipFree(kv.second);
        P.blocks[dev].clear();
        P.cached[dev] = 0;
        HIP_OK(hipMalloc(&p, bytes));
    }
    *got = bytes;
    return p;
}

void tgms::dev_free(void* p, size_t bytes) {
    if (!p) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipFree(p);
        return;
    }
    DevPool& P = dev_pool();
    std::lock_guard<std::mutex> lock(P.mu);
    if (P.cached[dev] + bytes > POOL_CAP) {
        (void)hipFree(p);
        return;
    }
    P.blocks[dev].emplace(bytes, p);
    P.cached[dev] += bytes;
}

namespace {

thread_local std::string g_last_error;

struct Timer {
    hipEvent_t a, b;
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st) {
        HIP_OK(hipEventCreate(&a));
        HIP_OK(hipEventCreate(&b));
        HIP_OK(hipEventRecord(a, s));
    }
    double ms() {
        HIP_OK(hipEventRecord(b, s));
        HIP_OK(hipEventSynchronize(b));
        float t = 0;
        HIP_OK(hipEventElapsedTime(&t, a, b));
        HIP_OK(hipEventDestroy(a));
        HIP_OK(hipEventDestroy(b));
        return t;
    }
};

// the elapsed time between two events recorded on a stream (read after both)
struct SpanTimer {
    hipEvent_t a = nullptr, b = nullptr;
    void start(hipStream_t s) {
        HIP_OK(hipEventCreate(&a));
        HIP_OK(hipEventCreate(&b));
        HIP_OK(hipEventRecord(a, s));
    }
    void stop(hipStream_t s) { HIP_OK(hipEventRecord(b, s)); }
    double ms() {
        if (!a || !b) return 0.0;
        HIP_OK(hipEventSynchronize(b));
        float t = 0;
        HIP_OK(hipEventElapsedTime(&t, a, b));
        return t;
    }
    ~SpanTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

template <typename F>
tgms_status guarded(F&& f) {
    try {
        f();
        return TGMS_OK;
    } catch (const TgmsError& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return TGMS_E_DEVICE;
    }
}

// Extreme eigenvalues of the symmetric tridiagonal Lanczos matrix by bisection (Sturm counts).
double lanczos_cond(const std::vector<double>& al, const std::vector<double>& be) {
    const int k = (int)al.size();
    if (k == 0) return 1.0;
    std::vector<double> d(k), e(k, 0.0);
    for (int i = 0; i < k; ++i) {
        d[i] = 1.0 / al[i] + (i > 0 ? be[i - 1] / al[i - 1] : 0.0);
        if (i + 1 < k && i < (int)be.size()) e[i] = std::sqrt(std::fabs(be[i])) / al[i];
    }
    double lo = d[0], hi = d[0];
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + std::fabs(e[i]);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
    }
    auto count_below = [&](double x) {
        int cnt = 0;
        double q = d[0] - x;
        if (q < 0) ++cnt;
        for (int i = 1; i < k; ++i) {
            if (q == 0) q = 1e-300;
            q = d[i] - x - e[i - 1] * e[i - 1] / q;
            if (q < 0) ++cnt;
        }
        return cnt;
    };
    auto kth = [&](int idx) {
        double a = lo, b = hi;
        for (int it = 0; it < 200; ++it) {
            const double m = 0.5 * (a + b);
            if (count_below(m) > idx)
                b = m;
            else
                a = m;
        }
        return 0.5 * (a + b);
    };
    const double mn = kth(0), mx = kth(k - 1);
    return mn > 0 ? mx / mn : INFINITY;
}

// z = B_TG g (paper section 5): pre-smoothing, coarse correction, post-smoothing,
// with the residual recomputed after each.  g: the right-hand side in the
// preconditioner's precision (T), gd: the same right-hand side in FP64 (the
// residuals are formed in FP64 from it); z: FP64 output.  With dots, the final
// gather also forms the PCG scalars from gd (and gold for the flexible variant).
// The variants of section 5's cycle, unfused: m = c->msteps pre- and post-smoothing steps
// with the residual recomputed after each (z += S(g - K z)), and the two-level additive
// Schwarz form z = S g + P g (c->additive).  The iterate of the cycle is kept in FP64
// (vt2), the residual formed in FP64 (vt) and rounded to the preconditioner's precision;
// the last gather forms the PCG's partial sums.
template <typename T>
void twogrid_variant(tgms_ctx* c, const T* g, const double* gd, double* z, const double* gold, bool dots,
                     bool first) {
    const double* sc = dots ? c->sc : nullptr;
    const long long nv = (long long)c->nx * c->ny;
    const T* w = sizeof(T) == 8 ? (const T*)c->patW : (const T*)c->patW32;
    double* z1 = c->vt2;
    double* tmp = c->vt3;
    double* td = c->vt;
    T* tT = sizeof(T) == 8 ? (T*)c->vt : (T*)c->ft;
    auto to_T = [&](const double* x) -> const T* {  // x in the preconditioner's precision
        if constexpr (sizeof(T) == 8) return (const T*)x;
        tgms::cast_d2f(c, nv, x, c->ft);
        return (const T*)c->ft;
    };
    auto smooth_add = [&](const T* rhs, bool last) {
        // z1 += S rhs (the last post-smoothing gathers into z with the PCG sums instead)
        tgms::smooth_patches<T>(c, rhs, sc);
        if (last) {
            const T* zin;
            if constexpr (sizeof(T) == 8) {
                zin = (const T*)z1;
            } else {
                tgms::cast_d2f(c, nv, z1, c->ft2);
                zin = (const T*)c->ft2;
            }
            tgms::gather_final<T>(c, w, zin, z, dots ? gd : nullptr, gold, dots, first);
        } else {
            tgms::gather_final<T>(c, w, nullptr, tmp, nullptr, nullptr, false, false);
            tgms::axpy(c, nv, 1.0, tmp, z1);
        }
    };
    if (c->additive) {
        // z = S g + P g
        tgms::smooth_patches<T>(c, g, sc);
        T* zc = sizeof(T) == 8 ? (T*)c->vt2 : (T*)c->ft2;
        tgms::coarse_apply<T>(c, to_T(gd), zc, false, sc);
        tgms::gather_final<T>(c, w, (const T*)zc, z, dots ? gd : nullptr, gold, dots, first);
        return;
    }
    const int m = c->msteps;
    tgms::zero(c, z1, sizeof(double) * nv);
    for (int k = 0; k < m; ++k) {  // pre-smoothing
        if (k == 0) {
            smooth_add(g, false);
        } else {
            tgms::vertex_residual(c, gd, z1, td);
            smooth_add(to_T(td), false);
        }
    }
    // coarse correction of the residual
    tgms::vertex_residual(c, gd, z1, td);
    if constexpr (sizeof(T) == 8) {
        tgms::coarse_apply<double>(c, td, z1, true, sc);
    } else {
        tgms::coarse_apply<float>(c, to_T(td), c->ft2, false, sc);
        tgms::cast_f2d(c, nv, c->ft2, tmp);
        tgms::axpy(c, nv, 1.0, tmp, z1);
    }
    for (int k = 0; k < m; ++k) {  // post-smoothing
        tgms::vertex_residual(c, gd, z1, td);
        smooth_add(to_T(td), k == m - 1);
    }
    (void)tT;
}

// With fu, the PCG update runs first and forms the right-hand side g (gd = fu->gout in
// FP64; for an FP32 preconditioner its rounding, in fg).
template <typename T>
void twogrid(tgms_ctx* c, const T* g, const double* gd, double* z, const double* gold, bool dots, bool first,
             const FusedUpdate* fu = nullptr) {
    if (fu) {
        T* gT = sizeof(T) == 8 ? nullptr : (T*)c->fg;
        tgms::pcg_update<T>(c, *fu, gT);
        g = sizeof(T) == 8 ? (const T*)fu->gout : gT;
    }
    if (c->msteps != 1 || c->additive) {
        twogrid_variant<T>(c, g, gd, z, gold, dots, first);
        return;
    }
    const double* sc = dots ? c->sc : nullptr;
    T *w, *z1, *z2, *t;
    if constexpr (sizeof(T) == 8) {
        w = (T*)c->patW;
        z1 = (T*)c->vt2;
        z2 = (T*)c->vt3;
        t = (T*)c->vt;
    } else {
        w = (T*)c->patW32;
        z1 = (T*)c->fz;
        z2 = (T*)c->ft2;
        t = (T*)c->ft;
    }
    tgms::smooth_patches<T>(c, g, sc);
    tgms::gather_res_restrict<T>(c, w, gd, z1, t, tgms::coarse_cy<T>(c), sc);
    // the coarse solution prolonged, z2 = z1 + W c, and the second smoothing's right-hand
    // side g - K z2 (into t, whose restriction the coarse solve has consumed)
    PreResidual<T> pr;
    pr.z1 = z1;
    pr.z1p = z2;
    pr.c = tgms::coarse_solve<T>(c, sc);
    if constexpr (sizeof(T) == 8)
        pr.W = (const T*)c->W;
    else
        pr.W = (const T*)c->W32;
    pr.mu = c->mu;
    pr.unk = c->blk_unk;
    pr.nunk = c->blk_nu;
    pr.g = gd;
    pr.a = c->a;
    pr.sx2 = c->sx * c->sx;
    pr.sy2 = c->sy * c->sy;
    tgms::prolong_residual<T>(c, pr, t, sc);
    tgms::smooth_patches<T>(c, t, sc);
    tgms::gather_final<T>(c, w, z2, z, dots ? gd : nullptr, gold, dots, first);
}

// probes: which = 0 smoother, 1 coarse correction, 2 two-grid; g, z FP64 vertex arrays
void precond(tgms_ctx* c, int which, const double* g, double* z) {
    const long long nv = (long long)c->nx * c->ny;
    if (c->precision == 0) {
        if (which == 0) {
            tgms::smooth_patches<double>(c, g, nullptr);
            tgms::gather_final<double>(c, c->patW, nullptr, z, nullptr, nullptr, false, false);
        } else if (which == 1) {
            tgms::coarse_apply<double>(c, g, z, false, nullptr);
        } else {
            twogrid<double>(c, g, g, z, nullptr, false, false);
        }
    } else {
        tgms::cast_d2f(c, nv, g, c->fg);
        if (which == 0) {
            tgms::smooth_patches<float>(c, c->fg, nullptr);
            tgms::gather_final<float>(c, c->patW32, nullptr, z, nullptr, nullptr, false, false);
        } else if (which == 1) {
            tgms::coarse_apply<float>(c, c->fg, c->fz, false, nullptr);
            tgms::cast_f2d(c, nv, c->fz, z);
        } else {
            twogrid<float>(c, c->fg, g, z, nullptr, false, false);
        }
    }
}

}  // namespace

void tgms::twogrid_probe(tgms_ctx* c) { precond(c, 2, c->vz, c->vq); }

namespace {

// Coarse unknowns (the zero-flux modes of every face, then one stream function per
// interior coarse vertex), the unknowns touching each block (slots, ordered by id) and
// their CSR inverse, and the description of each slot's combination of the face
// modes (meta, read by k_fill_td, which forms Td on the device from YQ).  All of it is
// written into `pack` and uploaded with one copy; `pack` must outlive that copy.  Returns
// the device address of meta.
int* build_coarse_numbering(tgms_ctx* c, std::vector<int>& pack) {
    const int Nx = c->Nx, Ny = c->Ny, nex = c->nex, nblk = c->nblk;
    const int* cnt = c->counts_h.data();
    // Numbering in the row-major order of the unknowns' positions on the coarse grid, in
    // doubled coordinates: vertex (I, J) at (2I, 2J), the zero-flux modes of x-face (I, J)
    // at (2I, 2J + 1), of y-face (I, J) at (2I + 1, 2J).  Unknowns couple only through a
    // shared block, so the matrix is banded with a half-bandwidth of about Nx + 1 unknowns
    // (block tridiagonal for the cyclic-reduction Cholesky).  Without zero-flux modes the
    // vertices come in row-major order.
    std::vector<int> zstart(c->ne, -1), vtx((size_t)(Nx + 1) * (Ny + 1), -1);
    int next = 0;
    for (int J = 0; J <= Ny; ++J) {
        // doubled row 2J: vertices (I, J) and the y-faces (I, J) between them
        for (int I = 0; I <= Nx; ++I) {
            if (I >= 1 && I <= Nx - 1 && J >= 1 && J <= Ny - 1) vtx[(size_t)J * (Nx + 1) + I] = next++;
            if (I < Nx && J >= 1 && J <= Ny - 1) {
                const int f = nex + (J - 1) * Nx + I;
                zstart[f] = next;
                next += cnt[f] - 1;
            }
        }
        if (J == Ny) break;
        // doubled row 2J + 1: the interior x-faces (I, J) of block row J
        for (int I = 1; I <= Nx - 1; ++I) {
            const int f = J * (Nx - 1) + I - 1;
            zstart[f] = next;
            next += cnt[f] - 1;
        }
    }
    c->nv = (Nx - 1) * (Ny - 1);
    c->ncs = next;
    const int ncs = next;
    auto vid = [&](int I, int J) { return (I <= 0 || I >= Nx || J <= 0 || J >= Ny) ? -1 : vtx[(size_t)J * (Nx + 1) + I]; };
    // faces of block (I, J): 0 left (x-face I), 1 right (x-face I + 1), 2 bottom
    // (y-face J), 3 top (y-face J + 1); -1 on the domain boundary
    auto faces = [&](int I, int J, int face[4]) {
        face[0] = I > 0 ? J * (Nx - 1) + I - 1 : -1;
        face[1] = I + 1 < Nx ? J * (Nx - 1) + I : -1;
        face[2] = J > 0 ? nex + (J - 1) * Nx + I : -1;
        face[3] = J + 1 < Ny ? nex + J * Nx + I : -1;
    };
    int mu = 1;
    for (int J = 0; J < Ny; ++J)
        for (int I = 0; I < Nx; ++I) {
            int face[4], n = 0;
            faces(I, J, face);
            for (int s = 0; s < 4; ++s)
                if (face[s] >= 0) n += cnt[face[s]] - 1;
            n += (vid(I, J) >= 0) + (vid(I + 1, J) >= 0) + (vid(I, J + 1) >= 0) + (vid(I + 1, J + 1) >= 0);
            mu = std::max(mu, n);
        }
    c->mu = mu;
    // pack: meta (11 words per slot), slot ids, slot counts, CSR pointers and entries,
    // slot corners; each part starts on a 256-byte boundary
    const size_t nslot = (size_t)nblk * mu;
    auto up = [](size_t n) { return (n + 63) & ~(size_t)63; };
    const size_t o_meta = 0, o_unk = up(nslot * 11), o_nu = o_unk + up(nslot), o_ptr = o_nu + up(nblk),
                 o_flat = o_ptr + up((size_t)ncs + 1), o_zc = o_flat + up(std::max(nslot, (size_t)1));
    pack.assign(o_zc + up(nslot), 0);
    int* meta = pack.data() + o_meta;
    int* unk = pack.data() + o_unk;
    int* nu = pack.data() + o_nu;
    int* ptr = pack.data() + o_ptr;
    int* flat = pack.data() + o_flat;
    int* zc = pack.data() + o_zc;
    // Slots of a block in increasing id, i.e. in the doubled-coordinate raster: vertex
    // (I, J), bottom face modes, vertex (I + 1, J), left face modes, right face modes,
    // vertex (I, J + 1), top face modes, vertex (I + 1, J + 1).  A face mode k >= 1 is its
    // own slot; a corner vertex's slot combines the carriers (k = 0) of the block's two
    // faces meeting there, in face order, with sign +1 where the vertex is the face's
    // first end (left/right faces: the upper vertex; bottom/top: the left one) and -1
    // where it is the second.  `corner` is the vertex's local index in the (bx+1) x (by+1)
    // grid of the block, counted from the diagonally opposite corner.
    const int bx = c->bx, by = c->by;
    int cband = 0;
    for (int J = 0; J < Ny; ++J)
        for (int I = 0; I < Nx; ++I) {
            const int b = J * Nx + I;
            int face[4];
            faces(I, J, face);
            int u = 0;
            auto slot = [&](int id, int corner, int n) -> int* {
                unk[(size_t)b * mu + u] = id;
                zc[(size_t)b * mu + u] = corner;
                int* mm = meta + ((size_t)b * mu + u) * 11;
                mm[0] = id;
                mm[1] = corner;
                mm[2] = n;
                ++u;
                return mm;
            };
            auto modes = [&](int s) {
                const int f = face[s];
                if (f < 0) return;
                for (int k = 1; k < cnt[f]; ++k) {
                    int* mm = slot(zstart[f] + k - 1, 0, 1);
                    mm[3] = f;
                    mm[4] = s;
                    mm[5] = k;
                    mm[6] = 1;
                }
            };
            // vertex slot: carriers of faces s0 and s1 with signs g0, g1
            auto vertex = [&](int v, int corner, int s0, int g0, int s1, int g1) {
                if (v < 0) return;
                int* mm = slot(v, corner, 2);
                mm[3] = face[s0];
                mm[4] = s0;
                mm[5] = 0;
                mm[6] = g0;
                mm[7] = face[s1];
                mm[8] = s1;
                mm[9] = 0;
                mm[10] = g1;
            };
            vertex(vid(I, J), by * (bx + 1) + bx, 0, -1, 2, 1);
            modes(2);
            vertex(vid(I + 1, J), by * (bx + 1), 1, -1, 2, -1);
            modes(0);
            modes(1);
            vertex(vid(I, J + 1), bx, 0, 1, 3, 1);
            modes(3);
            vertex(vid(I + 1, J + 1), 0, 1, 1, 3, -1);
            nu[b] = u;
            if (u > 0) cband = std::max(cband, unk[(size_t)b * mu + u - 1] - unk[(size_t)b * mu]);
            for (int q = 0; q < u; ++q) ++ptr[unk[(size_t)b * mu + q] + 1];
        }
    // half-bandwidth of the coarse matrix: unknowns couple only within a block
    c->cband = cband;
    for (int q = 0; q < ncs; ++q) ptr[q + 1] += ptr[q];
    std::vector<int> fill(ptr, ptr + ncs);
    for (int b = 0; b < nblk; ++b)  // blocks in increasing order: the accumulation order
        for (int q = 0; q < nu[b]; ++q) flat[fill[unk[(size_t)b * mu + q]]++] = b * mu + q;
    int* d = c->alloc<int>(pack.size());
    HIP_OK(hipMemcpyAsync(d, pack.data(), sizeof(int) * pack.size(), hipMemcpyHostToDevice, c->stream));
    c->blk_unk = d + o_unk;
    c->blk_nu = d + o_nu;
    c->unk_ptr = d + o_ptr;
    c->unk_ent = d + o_flat;
    c->zcd = d + o_zc;
    return d + o_meta;
}

// Coarse RT0 vertex stiffness K_H = C_H^T A_H0 C_H (dense, host-assembled from the per-block Grams).
// coarse RT0 stream-function stiffness (preprocessing, section 3) and its inverse
// The cyclic-reduction Cholesky is taken for systems larger than the one-launch explicit
// inverse serves (or whose FP32 inverse would lose accuracy) when their band fits the
// factor kernel; `which` (tgms_options.coarse_factor): 0 that choice, 1 always the dense
// inverse, 2 cyclic reduction wherever the band fits.
bool use_bcr(const tgms_ctx* c, int n, int band, bool fp32) {
    if (c->coarse_factor == 1 || n <= 0) return false;
    if (band + 1 > tgms::bcr_max_block(c)) return false;
    if (c->coarse_factor == 2) return true;
    return fp32 || n > tgms::symv_acc_max();
}

// Coarse RT0 vertex stiffness K_H = C_H^T A_H0 C_H (9-point: half-bandwidth Nx in the
// row-major vertex order) and its factorisation, on the calling stream.
void build_rt0_stiffness(tgms_ctx* c) {
    const int nv = c->nv;
    if (!c->KH) c->KH = c->alloc<double>((size_t)nv * nv);
    tgms::zero(c, c->KH, sizeof(double) * (size_t)nv * nv);
    tgms::rt0_stiffness(c, c->AH0, c->KH);
    if (use_bcr(c, nv, c->Nx, false)) {
        tgms::bcr_factor(c, c->KH, nv, std::max(c->Nx, 1), c->kb, false);
        if (tgms::bcr_failed(c, c->kb)) throw TgmsError{TGMS_E_INVAL, "coarse RT0 operator is not positive definite"};
    } else {
        tgms::dense_spd_inverse(c, c->KH, nv);
    }
}

// Factorisation of the coarse SPD matrix c->Ac (assembled): the cyclic-reduction Cholesky
// of its band, or the dense Cholesky inverse (in place, with the explicit inverse for a
// small FP64 system and an FP32 copy for the FP32 preconditioner).
void factor_coarse(tgms_ctx* c) {
    const long long n2 = (long long)c->ncs * c->ncs;
    if (use_bcr(c, c->ncs, c->cband, c->precision != 0)) {
        tgms::bcr_factor(c, c->Ac, c->ncs, std::max(c->cband, 1), c->cb, c->precision != 0, true);
        if (tgms::bcr_failed(c, c->cb)) throw TgmsError{TGMS_E_INVAL, "coarse operator is not positive definite"};
        return;
    }
    c->cb = Bcr{};
    if (!c->precision && c->ncs <= tgms::symv_acc_max() && !c->Acf) c->Acf = c->alloc<double>(n2);
    tgms::dense_spd_inverse(c, c->Ac, c->ncs, c->Acf);
    if (c->precision) {
        if (!c->Ac32) c->Ac32 = c->alloc<float>(n2);
        tgms::cast_d2f(c, n2, c->Ac, c->Ac32);
    }
}

// The coarse matrix of the RT0 coarse space: the coarse vertex stiffness over the
// bilinear stream functions (exactly W^T K W for the W of tgms::rt0_coarse_W), from
// Grams of the current cell weights formed on the calling stream.
void rt0_coarse_matrix(tgms_ctx* c) {
    if (!c->AH0c) c->AH0c = c->alloc<double>((size_t)c->nblk * 6);
    tgms::coarse_rt0_blocks(c, c->AH0c);
    tgms::zero(c, c->Ac, sizeof(double) * (size_t)c->ncs * c->ncs);
    tgms::rt0_stiffness(c, c->AH0c, c->Ac);
}

// What tgms_save writes and tgms_load reads back: the permeability as the setup saw it
// (kappa^{-1}), the current cell weights (after mobility updates), and the adaptive
// coarse space: basis counts, eigenvalues and each face's kept modes (in snapshot
// coefficients, recombined into the unit-flux carrier and zero-flux modes).
struct Artefact {
    int nx = 0, ny = 0, bx = 0, by = 0, overlap = 0, precision = 0, coarse_space = 0, mobility = 0, ne = 0, jmax = 0;
    double eta = 0, tol = 0, H = 0;
    std::vector<double> kinv, a, eigs, YQ;
    std::vector<int> counts;
};

void rebuild_operator(tgms_ctx* c);

// art: a saved context to restore (kappa unused; the coarse space is read, not solved for)
void setup_impl(const tgms_grid* grid, const double* kappa, double eig_tol, const tgms_options* opt,
                tgms_ctx** out, const Artefact* art = nullptr) {
    if (!grid || (!kappa && !art) || !out) throw TgmsError{TGMS_E_INVAL, "null argument"};
    tgms_options o;
    tgms_default_options(&o);
    if (opt) o = *opt;
    if (grid->dim == 3) {
        if (art) throw TgmsError{TGMS_E_UNSUPPORTED, "saved contexts are two-dimensional"};
        auto* c = new tgms_ctx();
        try {
            c->user_stream = (hipStream_t)o.stream;
            HIP_OK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            HIP_OK(hipEventCreateWithFlags(&c->ev_enter, hipEventDisableTiming));
            tgms::enter(c);
            tgms3::setup3(c, grid, kappa, eig_tol, &o);
        } catch (...) {
            tgms_destroy(c);
            throw;
        }
        *out = c;
        return;
    }
    if (grid->dim != 2 || grid->nz > 1 || grid->bz > 1)
        throw TgmsError{TGMS_E_INVAL, "dim must be 2 (with nz and bz 0 or 1)"};
    const int nx = grid->nx, ny = grid->ny, bx = grid->bx, by = grid->by;
    if (nx <= 0 || ny <= 0 || bx <= 0 || by <= 0 || nx % bx || ny % by)
        throw TgmsError{TGMS_E_INVAL, "grid sizes must be positive and divisible by the block size"};
    if (!(eig_tol > 0) || !(o.eta > 0)) throw TgmsError{TGMS_E_INVAL, "bad tolerance or eta"};
    // Without oversampling the smoother never touches the fine fluxes across block
    // edges; the coarse space spans only part of them, so the two-grid preconditioner
    // is singular on the divergence-free fields and PCG stops at a wrong solution.
    if (o.overlap < 1) throw TgmsError{TGMS_E_INVAL, "overlap must be at least 1"};
    if (bx < 3 || by < 3 || nx / bx < 2 || ny / by < 2)
        throw TgmsError{TGMS_E_UNSUPPORTED, "need blocks of at least 3x3 cells and at least 2x2 blocks"};
    if (o.overlap >= std::min(bx, by)) throw TgmsError{TGMS_E_UNSUPPORTED, "overlap must be smaller than a block"};
    if (std::max(bx, by) > 64) throw TgmsError{TGMS_E_UNSUPPORTED, "blocks wider than 64 cells"};
    const int ex = std::min(bx + 2 * o.overlap, nx), ey = std::min(by + 2 * o.overlap, ny);
    if (ex > 33) throw TgmsError{TGMS_E_UNSUPPORTED, "smoother patches wider than 33 cells"};
    (void)ey;
    if (o.warm_start < 0 || o.warm_start > 2) throw TgmsError{TGMS_E_INVAL, "warm_start must be 0, 1 or 2"};
    if (o.smoother_staging < -1 || o.smoother_staging > 1)
        throw TgmsError{TGMS_E_INVAL, "smoother_staging must be -1, 0 or 1"};
    if (o.rows_per_thread != 0 && o.rows_per_thread != 1 && o.rows_per_thread != 4)
        throw TgmsError{TGMS_E_INVAL, "rows_per_thread must be 0, 1 or 4"};
    if (o.coarse_space < 0 || o.coarse_space > 2) throw TgmsError{TGMS_E_INVAL, "coarse_space must be 0, 1 or 2"};
    if (o.coarse_factor < 0 || o.coarse_factor > 2) throw TgmsError{TGMS_E_INVAL, "coarse_factor must be 0, 1 or 2"};
    if (o.smooth_steps < 1 || o.smooth_steps > 16) throw TgmsError{TGMS_E_INVAL, "smooth_steps must lie in [1, 16]"};
    if (o.additive != 0 && o.additive != 1) throw TgmsError{TGMS_E_INVAL, "additive must be 0 or 1"};
    if (o.force_counts && (o.warm_start != 0 || o.coarse_space != 0))
        throw TgmsError{TGMS_E_INVAL, "force_counts needs the dense eigensolve of the adaptive space"};
    if (o.coarse_space != 0 && o.warm_start != 0)
        throw TgmsError{TGMS_E_INVAL, "the MsFEM and RT0 coarse spaces solve no eigenproblem to warm-start"};
    if (art) {
        o.warm_start = 0;
        o.force_counts = nullptr;
    }
    if (o.warm_start == 2) {
        if (!o.cnn_weights) throw TgmsError{TGMS_E_INVAL, "warm_start 2 needs cnn_weights"};
        if (bx != by || !tgms::cnn_shape_ok(2 * bx, bx))
            throw TgmsError{TGMS_E_UNSUPPORTED, "the network warm start needs square blocks of at most 16 x 16 cells"};
    }
    auto* c = new tgms_ctx();
    // second stream (default priority) for the preprocessing's coarse RT0 inverse, which
    // runs concurrently with the spectral setup; declared before the queued inverse so
    // that the inverse's clean-up still finds it
    struct Side {
        hipStream_t s = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, ez = nullptr;
        ~Side() {
            if (s) (void)hipStreamSynchronize(s);
            if (ez) (void)hipEventDestroy(ez);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (e2) (void)hipEventDestroy(e2);
            if (s) (void)hipStreamDestroy(s);
        }
    } side;
    tgms::DenseInvAsync kh_inv;
    SpanTimer pat_timer;     // the smoother factorisation on the second stream
    // the main stream's phases, read after the final synchronisation (no waits between)
    SpanTimer snap_timer, eig_timer, coarse_timer;
    int* pat_fail = nullptr;
    int* blk_fail = nullptr;  // the block factorisation (checked at the end)
    try {
        // All work runs on a stream of the library's own (default priority); each call
        // first waits for what the caller queued on its stream (NULL: the null stream)
        // and returns after synchronising, so results are visible on every stream.
        c->user_stream = (hipStream_t)o.stream;
        HIP_OK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        HIP_OK(hipEventCreateWithFlags(&c->ev_enter, hipEventDisableTiming));
        tgms::enter(c);
        c->nx = nx; c->ny = ny; c->bx = bx; c->by = by;
        c->Nx = nx / bx; c->Ny = ny / by; c->nblk = c->Nx * c->Ny;
        c->nex = (c->Nx - 1) * c->Ny;
        c->ne = c->nex + c->Nx * (c->Ny - 1);
        c->jmax = std::max(bx, by);
        c->hx = 1.0 / nx; c->hy = 1.0 / ny;
        c->sx = 1.0 / c->hy; c->sy = 1.0 / c->hx;
        c->H = o.s_scale > 0 ? o.s_scale : std::sqrt(bx * c->hx * by * c->hy);
        c->coarse_space = o.coarse_space;
        c->coarse_factor = o.coarse_factor;
        c->msteps = o.smooth_steps;
        c->additive = o.additive ? 1 : 0;
        c->eig_bad = c->alloc<int>(1);
        c->eta = o.eta; c->tol = eig_tol; c->overlap = o.overlap; c->precision = o.precision ? 1 : 0;
        c->graph_failed = o.graphs == 0;  // never capture: launch every kernel directly
        c->warm = o.warm_start;
        c->rq_tol = o.rq_tol > 0 ? o.rq_tol : 1e-6;
        c->nfx = (nx + 1) * ny; c->nfy = nx * (ny + 1); c->nf = c->nfx + c->nfy;
        c->nfk = by * (bx + 1) + (by + 1) * bx;
        c->ncol = 4 * c->jmax;
        const long long ncell = (long long)nx * ny;
        {
            int dev = 0, v = 0;
            HIP_OK(hipGetDevice(&dev));
            if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
                c->lds_max = v;
        }
        Timer total(c->stream);
        c->kinv = c->alloc<double>(ncell);
        c->a = c->alloc<double>(ncell);
        if (art) {
            HIP_OK(hipMemcpyAsync(c->kinv, art->kinv.data(), sizeof(double) * ncell, hipMemcpyHostToDevice, c->stream));
            tgms::weights_from_kinv(c);
        } else {
            int* bad = c->alloc<int>(1);
            tgms::cell_weights(c, kappa, bad);
            int hbad = 0;
            HIP_OK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
            HIP_OK(hipStreamSynchronize(c->stream));
            if (hbad) throw TgmsError{TGMS_E_INVAL, "permeability must be finite and positive"};
        }
        if (o.force_counts) {
            for (int f = 0; f < c->ne; ++f) {
                const int J = f < c->nex ? by : bx, l = o.force_counts[f];
                if (l < 1 || l > J) throw TgmsError{TGMS_E_INVAL, "force_counts entries must lie in [1, J_i]"};
            }
            c->force = c->alloc<int>(c->ne);
            HIP_OK(hipMemcpyAsync(c->force, o.force_counts, sizeof(int) * c->ne, hipMemcpyHostToDevice, c->stream));
        }
        // block factors
        c->blk_m = bx - 1;
        c->blk_n = (bx - 1) * (by - 1);
        c->blk_b = bx;
        c->blkL = c->alloc<double>((size_t)c->nblk * btri_size(bx - 1, by - 1));
        c->blkS = c->alloc<double>((size_t)c->nblk * c->blk_n);
        // the coarse RT0 stiffness of the preprocessing (section 3) and its inverse go to a
        // second stream, joined before the end of the coarse phase; they are queued after the
        // block factorisation is launched, so that the GPU works while the host queues them
        c->nv = (c->Nx - 1) * (c->Ny - 1);
        c->AH0 = c->alloc<double>((size_t)c->nblk * 6);
        c->KH = c->alloc<double>((size_t)c->nv * c->nv);
        HIP_OK(hipStreamCreateWithFlags(&side.s, hipStreamNonBlocking));
        HIP_OK(hipEventCreateWithFlags(&side.e0, hipEventDisableTiming));
        HIP_OK(hipEventCreateWithFlags(&side.e1, hipEventDisableTiming));
        HIP_OK(hipEventCreateWithFlags(&side.e2, hipEventDisableTiming));
        HIP_OK(hipEventCreateWithFlags(&side.ez, hipEventDisableTiming));
        // The smoother's patch table and the large spectral buffers are allocated with
        // their upload and clearing queued on the second stream ahead of its other work
        // (they depend on nothing queued before), where they run during the block
        // factorisation; the snapshots wait for the clearing (event ez).
        const bool gram_mfma = tgms::gram_uses_mfma(c);
        const size_t nvk = (size_t)(bx + 1) * (by + 1);
        {
            const hipStream_t main_stream = c->stream;
            struct Restore {
                tgms_ctx* c;
                hipStream_t s;
                ~Restore() { c->stream = s; }
            } restore{c, main_stream};
            c->stream = side.s;
            // the smoother's patch table, uploaded first on this stream (a copy from pageable
            // memory holds the host until the stream reaches it)
            c->patch_h.resize(c->nblk);
            long long off = 0, voff = 0;
            std::set<int> widths;
            for (int J = 0; J < c->Ny; ++J)
                for (int I = 0; I < c->Nx; ++I) {
                    Rect& r = c->patch_h[J * c->Nx + I];
                    r.i0 = std::max(I * bx - o.overlap, 0);
                    r.i1 = std::min((I + 1) * bx + o.overlap, nx);
                    r.j0 = std::max(J * by - o.overlap, 0);
                    r.j1 = std::min((J + 1) * by + o.overlap, ny);
                    const int m = r.i1 - r.i0 - 1, n = m * (r.j1 - r.j0 - 1);
                    r.off = off;
                    r.voff = voff;
                    off += (tw_size(m, r.j1 - r.j0 - 1) + 3) & ~3LL;  // 16-byte aligned factors
                    c->pat_fmax = std::max(c->pat_fmax, tw_size(m, r.j1 - r.j0 - 1));
                    voff += n;
                    c->pat_nmax = std::max(c->pat_nmax, n);
                    c->pat_hmax = std::max(c->pat_hmax, r.j1 - r.j0 - 1);
                    c->pat_bmax = std::max(c->pat_bmax, m + 1);
                    widths.insert(m);
                }
            // the kernels take fixed-width paths for up to two distinct row widths
            c->pat_m1 = *widths.rbegin();
            c->pat_m2 = widths.size() == 1 ? c->pat_m1 : widths.size() == 2 ? *widths.begin() : -1;
            c->pat_pool = off;
            c->pat_vpool = voff;
            c->patch = c->alloc<Rect>(c->nblk);
            HIP_OK(hipMemcpyAsync(c->patch, c->patch_h.data(), sizeof(Rect) * c->nblk, hipMemcpyHostToDevice,
                                  c->stream));
            // snapshots (A Psi is the snapshot solves' scratch until the Gram products),
            // A_K Psi for the Gram kernel without matrix cores (the path integrals of the
            // coarse assembly reuse it: nblk * (bx+1)(by+1) * ncol) and the Grams
            c->Psi = c->alloc<double>((size_t)c->nblk * c->ncol * c->nfk);
            c->APsi = c->alloc<double>((size_t)c->nblk * c->ncol * (gram_mfma ? nvk : (size_t)c->nfk));
            c->G = c->alloc<double>((size_t)c->nblk * c->ncol * c->ncol);
            HIP_OK(hipEventRecord(side.ez, side.s));
            // the rest of this stream's work reads what the main stream has queued so far
            HIP_OK(hipEventRecord(side.e0, main_stream));
            HIP_OK(hipStreamWaitEvent(side.s, side.e0, 0));
        }
        double* YQd = nullptr;
        {
            snap_timer.start(c->stream);
            blk_fail = c->alloc<int>(1);
            tgms::factor_blocks(c, blk_fail);
            // snapshots + Gram (queued before the coarse RT0 inverse on the second stream:
            // queueing that inverse's few hundred launches takes the host milliseconds,
            // which these kernels then cover)
            HIP_OK(hipStreamWaitEvent(c->stream, side.ez, 0));
            if (c->coarse_space != 2) {  // the RT0 coarse space needs no snapshots
                tgms::snapshots(c, c->APsi, (long long)c->ncol * (gram_mfma ? (long long)nvk : (long long)c->nfk));
                tgms::gram(c);
            }
            {
                const hipStream_t main_stream = c->stream;
                struct Restore {
                    tgms_ctx* c;
                    hipStream_t s;
                    ~Restore() { c->stream = s; }
                } restore{c, main_stream};
                c->stream = side.s;
                // smoother patches (section 5): factorised first on this second stream,
                // concurrently with the spectral setup on the main one (the patch matrices
                // depend on the cell weights only); the patch table is up already.  The
                // coarse RT0 operator of the preprocessing follows (its factor is needed
                // only at the end of the coarse phase); with it first, the patch factor
                // ended later and held the 8 x 8-block setup 0.5 ms longer.
                const long long off = c->pat_pool, voff = c->pat_vpool;
                c->patL = c->alloc<double>(off);
                c->patW = c->alloc<double>(voff);
                if (c->precision) {
                    c->patL32 = c->alloc<float>(off);
                    c->patW32 = c->alloc<float>(voff);
                }
                // a vertex is covered by its own block's patch and, when blocks are at least
                // twice the overlap, by at most one neighbour per direction: four slots
                c->slots = bx >= 2 * o.overlap && by >= 2 * o.overlap;
                if (c->slots) {
                    c->patW4 = c->alloc<double>(4 * (size_t)ncell);  // zero: slots no patch covers stay zero
                    if (c->precision) c->patW4_32 = c->alloc<float>(4 * (size_t)ncell);
                }
                pat_fail = c->alloc<int>(1);
                pat_timer.start(side.s);
                // two workgroups per CU: the spectral setup on the main stream keeps CUs to
                // run on
                int cus = 0, dev = 0;
                HIP_OK(hipGetDevice(&dev));
                if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
                tgms::factor_patches_launch(c, pat_fail, 2 * cus);
                pat_timer.stop(side.s);
                // the coarse RT0 stiffness of the preprocessing and its factor
                tgms::coarse_rt0_blocks(c, c->AH0);
                tgms::rt0_stiffness(c, c->AH0, c->KH);
                if (use_bcr(c, c->nv, c->Nx, false))
                    tgms::bcr_factor(c, c->KH, c->nv, std::max(c->Nx, 1), c->kb, false);  // checked at the join
                else
                    tgms::dense_spd_inverse_begin(c, c->KH, c->nv, kh_inv);
                HIP_OK(hipEventRecord(side.e1, side.s));
                // the pressure's DCT matrices and the solve workspaces, cleared on this
                // stream too (the host queues them while the spectral kernels run)
                // pressure: orthonormal DCT-II matrices and the 1D Neumann eigenvalues
                c->Qx = c->alloc<double>((size_t)nx * nx);
                c->lamx = c->alloc<double>(nx);
                c->Qy = c->alloc<double>((size_t)ny * ny);
                c->lamy = c->alloc<double>(ny);
                tgms::dct_matrix(c, nx, c->Qx, c->lamx);
                tgms::dct_matrix(c, ny, c->Qy, c->lamy);
                // solve workspaces
                const long long nvtx = ncell;
                c->vx = c->alloc<double>(nvtx); c->vg = c->alloc<double>(nvtx); c->vz = c->alloc<double>(nvtx);
                c->vp = c->alloc<double>(nvtx); c->vq = c->alloc<double>(nvtx); c->vt = c->alloc<double>(nvtx);
                c->vt2 = c->alloc<double>(nvtx); c->vt3 = c->alloc<double>(nvtx); c->vgold = c->alloc<double>(nvtx);
                c->vg2 = c->alloc<double>(nvtx);
                c->fg = c->alloc<float>(nvtx); c->fz = c->alloc<float>(nvtx); c->ft = c->alloc<float>(nvtx);
                c->ft2 = c->alloc<float>(nvtx);
                c->fbar = c->alloc<double>(c->nf); c->fu = c->alloc<double>(c->nf); c->fF = c->alloc<double>(c->nf);
                c->cellw = c->alloc<double>(ncell); c->cellw2 = c->alloc<double>(std::max<long long>(ncell, 2 * c->nblk));
                c->blkbuf = c->alloc<double>(2 * (size_t)c->nblk);
                c->sc = c->alloc<double>(SC_COUNT);
                c->part = c->alloc<double>(3 * (size_t)tgms::pcg_tiles(c));
                c->part2 = c->alloc<double>((size_t)tgms::pcg_tiles(c));
                tgms::allow_fused_lds(c);
                c->vp1 = c->alloc<double>(nvtx);
                c->cflux = c->alloc<double>(2 * ((size_t)c->Ny * (c->Nx + 1) + (size_t)(c->Ny + 1) * c->Nx));
                c->svec = c->alloc<double>((size_t)c->nv + 1);
                c->svec2 = c->alloc<double>(2 * (size_t)c->nv + 1);
                HIP_OK(hipHostMalloc((void**)&c->red_h, SC_COUNT * sizeof(double), hipHostMallocDefault));
                HIP_OK(hipEventRecord(side.e2, side.s));
            }
            snap_timer.stop(c->stream);
            // the eigenproblems' buffers, queued while the spectral kernels run
            c->eigs = c->alloc<double>((size_t)c->ne * c->jmax);
            c->counts = c->alloc<int>(c->ne);
            c->Y = c->alloc<double>((size_t)c->ne * c->jmax * c->jmax);
            YQd = c->alloc<double>((size_t)c->ne * c->jmax * c->jmax);
            c->YQ = YQd;
            if (!art && c->coarse_space != 2 && c->warm) c->wstat = c->alloc<int>(c->ne);
            // the block factorisation, checked once the GPU has reached this point (before
            // the spectral problems use the snapshots)
            int hb = 0;
            HIP_OK(hipMemcpyAsync(&hb, blk_fail, sizeof(int), hipMemcpyDeviceToHost, c->stream));
            HIP_OK(hipStreamSynchronize(c->stream));
            if (hb) throw TgmsError{TGMS_E_INVAL, "local stream-function matrix is not positive definite"};
        }
        // pencils and eigenproblems
        if (art) {
            // the coarse space of the saved context
            Timer t(c->stream);
            HIP_OK(hipMemcpyAsync(c->eigs, art->eigs.data(), sizeof(double) * art->eigs.size(), hipMemcpyHostToDevice,
                                  c->stream));
            HIP_OK(hipMemcpyAsync(c->counts, art->counts.data(), sizeof(int) * c->ne, hipMemcpyHostToDevice, c->stream));
            HIP_OK(hipMemcpyAsync(YQd, art->YQ.data(), sizeof(double) * art->YQ.size(), hipMemcpyHostToDevice,
                                  c->stream));
            c->t_eig_ms = t.ms();
        } else if (c->coarse_space == 2) {
            // RT0: one coarse function per face, no eigenproblem
            std::vector<int> ones(c->ne, 1);
            HIP_OK(hipMemcpyAsync(c->counts, ones.data(), sizeof(int) * c->ne, hipMemcpyHostToDevice, c->stream));
        } else {
            eig_timer.start(c->stream);
            const float* Y0 = nullptr;
            if (c->warm == 2) {
                // network inputs of every face and the initial blocks [ne][8][b]
                Timer tc(c->stream);
                float* Xw = c->alloc<float>((size_t)c->ne * 2 * bx * bx);
                float* Yw = c->alloc<float>((size_t)c->ne * tgms::cnn_kout() * bx);
                tgms::cnn_windows(c, Xw);
                tgms::cnn_infer_bf16(c->stream, o.cnn_weights, Xw, c->ne, 2 * bx, bx, Yw);
                Y0 = Yw;
                c->t_cnn_ms = tc.ms();
            }
            tgms::pencil_eig_q(c, YQd, Y0, nullptr);
            eig_timer.stop(c->stream);
            HIP_OK(hipMemcpyAsync(&c->eig_unconverged, c->eig_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        }
        {
            coarse_timer.start(c->stream);
            c->counts_h.resize(c->ne);
            HIP_OK(hipMemcpyAsync(c->counts_h.data(), c->counts, sizeof(int) * c->ne, hipMemcpyDeviceToHost, c->stream));
            if (c->warm) {
                c->wstat_h.resize(c->ne);
                HIP_OK(hipMemcpyAsync(c->wstat_h.data(), c->wstat, sizeof(int) * c->ne, hipMemcpyDeviceToHost,
                                      c->stream));
            }
            HIP_OK(hipStreamSynchronize(c->stream));
            for (int w : c->wstat_h)
                if (w >= 0) {
                    ++c->warm_accepted;
                    c->warm_iters += w;
                }
            std::vector<int> pack;  // host side of the numbering upload, kept until the timer's synchronisation
            int* metad = build_coarse_numbering(c, pack);
            if (c->coarse_space != 2) {
                // the first coarse kernel as soon as the numbering is up (the GPU waits for the host here)
                c->Td = c->alloc<double>((size_t)c->nblk * c->ncol * c->mu);
                tgms::fill_td(c, metad, YQd, c->Td);
            }
            c->W = c->alloc<double>((size_t)c->nblk * bx * by * c->mu);
            if (c->precision) c->W32 = c->alloc<float>((size_t)c->nblk * bx * by * c->mu);
            c->Ac = c->alloc<double>((size_t)c->ncs * c->ncs);
            if (c->coarse_space == 2) {
                tgms::rt0_coarse_W(c);
                rt0_coarse_matrix(c);
            } else {
                tgms::coarse_local_run(c, c->Td, c->zcd);
            }
            c->cy = c->alloc<double>((size_t)c->nblk * c->mu);
            c->cvec = c->alloc<double>(2 * (size_t)c->ncs + 1);
            c->cvec2 = c->alloc<double>((size_t)c->ncs + 1);
            c->cy32 = c->alloc<float>((size_t)c->nblk * c->mu);
            c->cvec32 = c->alloc<float>(2 * (size_t)c->ncs + 1);
            c->cvec2_32 = c->alloc<float>((size_t)c->ncs + 1);
            factor_coarse(c);
            // coarse RT0 for the preprocessing: join the second stream
            HIP_OK(hipStreamWaitEvent(c->stream, side.e1, 0));
            tgms::dense_spd_inverse_end(kh_inv);
            if (c->kb.nb > 0 && tgms::bcr_failed(c, c->kb))
                throw TgmsError{TGMS_E_INVAL, "coarse RT0 operator is not positive definite"};
            coarse_timer.stop(c->stream);
        }
        // smoother patches: join the second stream and check the factorisation
        {
            HIP_OK(hipStreamWaitEvent(c->stream, side.e2, 0));
            int h = 0;
            HIP_OK(hipMemcpyAsync(&h, pat_fail, sizeof(int), hipMemcpyDeviceToHost, c->stream));
            HIP_OK(hipStreamSynchronize(c->stream));
            c->t_smoother_ms = pat_timer.ms();
            if (h) throw TgmsError{TGMS_E_INVAL, "smoother patch matrix is not positive definite"};
        }
        if (art && art->mobility) {
            // the saved context had its mobility updated: its weights, and every factor
            // built from them
            HIP_OK(hipMemcpyAsync(c->a, art->a.data(), sizeof(double) * ncell, hipMemcpyHostToDevice, c->stream));
            c->mobility_updated = true;
            rebuild_operator(c);
        }
        if (o.autotune) tgms::autotune(c, o.tune_cache);
        if (o.smoother_staging >= 0) c->smooth_staged = o.smoother_staging;
        if (o.rows_per_thread == 1 || o.rows_per_thread == 4) c->rpt = o.rows_per_thread;
        HIP_OK(hipStreamSynchronize(c->stream));
        c->t_setup_ms = total.ms();
        c->t_snap_ms = snap_timer.ms();
        if (eig_timer.a) c->t_eig_ms = eig_timer.ms();
        c->t_coarse_ms = coarse_timer.ms();
        *out = c;
    } catch (...) {
        if (side.s) (void)hipStreamSynchronize(side.s);  // its work writes into the context's buffers
        tgms_destroy(c);
        throw;
    }
}

// Mobility update with the coarse space kept (paper section 6.2: the basis built for
// the initial permeability is reused while the mobility changes).  The operator
// becomes A(lambda) with cell weights |c| / (lambda kappa); every factor that
// depends on it is rebuilt: block factors (preprocessing), the block Gram
// matrices of the fixed snapshots and the coarse SPD matrix over the fixed
// basis, its Cholesky inverse, the coarse RT0 operator and the smoother patches.
// every factor built from the cell weights c->a, with the coarse basis kept
void rebuild_operator(tgms_ctx* c) {
    tgms::factor_blocks(c);
    if (c->coarse_space == 2) {
        rt0_coarse_matrix(c);
    } else {
        tgms::gram(c);
        tgms::zero(c, c->Ac, sizeof(double) * (size_t)c->ncs * c->ncs);
        tgms::coarse_local_run(c, c->Td, c->zcd);
    }
    factor_coarse(c);
    tgms::coarse_rt0_blocks(c, c->AH0);
    build_rt0_stiffness(c);
    tgms::factor_patches(c);
    HIP_OK(hipStreamSynchronize(c->stream));
}

void update_mobility_impl(tgms_ctx* c, const double* lambda) {
    if (!c || !lambda) throw TgmsError{TGMS_E_INVAL, "null argument"};
    tgms::enter(c);
    if (c->dim == 3) {
        tgms3::update_mobility3(c, lambda);
        return;
    }
    // the new weights go to a scratch array first: an invalid field leaves the context as it was
    int* bad = c->alloc_scratch_int();
    tgms::mobility_weights(c, lambda, bad, c->cellw2);
    int hbad = 0;
    HIP_OK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (hbad) throw TgmsError{TGMS_E_INVAL, "mobility must be finite and positive"};
    tgms::copy(c, (long long)c->nx * c->ny, c->cellw2, c->a);
    c->mobility_updated = true;
    rebuild_operator(c);
}

// keep_history: read the PCG's alpha, beta back to the host (for tgms_last_cond)
void solve_impl(tgms_ctx* c, const double* F, const double* g_bnd, double rtol, int maxit, double* u, double* p,
                int* iters, double* relres, tgms_status* st, bool keep_history = true) {
    if (!c || !F || !u) throw TgmsError{TGMS_E_INVAL, "null argument"};
    if (!(rtol >= 0) || maxit < 0) throw TgmsError{TGMS_E_INVAL, "bad rtol or maxit"};
    tgms::enter(c);
    if (c->dim == 3) {
        if (g_bnd) throw TgmsError{TGMS_E_UNSUPPORTED, "on the cube only the no-flow boundary (g_bnd NULL)"};
        tgms3::solve3(c, F, rtol, maxit, u, p, iters, relres, st);
        if (*st == TGMS_E_NOTCONV) g_last_error = "PCG did not converge within maxit";
        if (*st == TGMS_E_BREAKDOWN) g_last_error = "PCG breakdown";
        return;
    }
    const long long nv = (long long)c->nx * c->ny;
    // Step 1: preprocessing
    tgms::preprocess(c, F, g_bnd, c->fbar, c->cellw2);
    // u0 = vbar + g_bnd (boundary entries), g = -C^T A u0
    tgms::bnd_faces(c, g_bnd, c->fF);
    tgms::axpy(c, c->nf, 1.0, c->fbar, c->fF);
    tgms::curlT_A_faces(c, c->fF, c->vg, -1.0);
    // Step 3: PCG in stream-function coordinates with its scalars on the device.
    // Two iterations (the search direction alternates between two buffers) are
    // captured once as a HIP graph and replayed; the kernels of iterations queued
    // after convergence return at once, so the host reads the scalars only every
    // four iterations.  With profiling on, the kernels are launched directly (four
    // iterations per check as well) and each event pair is tagged with its
    // iteration, so that launches of iterations after convergence are not counted.
    const bool flexible = c->precision != 0;
    if (c->hist_cap < maxit + 2) {
        c->hist = c->alloc<double>(2 * (size_t)(maxit + 2));
        c->hist_cap = maxit + 2;
        if (c->iter_graph) {
            (void)hipGraphExecDestroy(c->iter_graph);
            c->iter_graph = nullptr;
        }
    }
    const size_t prof_first = c->prof_rec.size(), ev_first = c->ev_used;
    tgms::zero(c, c->vx, sizeof(double) * nv);
    tgms::zero(c, c->vp, sizeof(double) * nv);
    tgms::zero(c, c->vp1, sizeof(double) * nv);
    for (int k = 0; k < SC_COUNT; ++k) c->red_h[k] = 0.0;
    c->red_h[SC_RTOL2] = rtol * rtol;
    c->red_h[SC_MAXIT] = maxit;
    c->red_h[SC_FLEX] = flexible ? 1.0 : 0.0;
    HIP_OK(hipMemcpyAsync(c->sc, c->red_h, SC_COUNT * sizeof(double), hipMemcpyHostToDevice, c->stream));
    // z_0 = B_TG g_0, rho_0 = g.z, |z_0|^2
    c->prof_iter = 0;
    if (flexible) {
        tgms::cast_d2f(c, nv, c->vg, c->fg);
        twogrid<float>(c, c->fg, c->vg, c->vz, nullptr, true, true);
    } else {
        twogrid<double>(c, c->vg, c->vg, c->vz, nullptr, true, true);
    }
    // The update x += alpha p, g -= alpha q runs ahead of the preconditioning; it reads
    // g from one buffer and writes the new g to the other (gin / gout alternate with the
    // search direction; gin is also the old residual the flexible beta needs).
    auto iteration = [&](const double* pin, double* pout, double* gin, double* gout) {
        tgms::dir_apply(c, c->vz, pin, pout, c->vq);
        const FusedUpdate fu{c->part2, c->nred, c->sc, c->hist, pout, c->vq, c->vx, gin, gout};
        if (flexible)
            twogrid<float>(c, nullptr, gout, c->vz, gin, true, false, &fu);
        else
            twogrid<double>(c, nullptr, gout, c->vz, nullptr, true, false, &fu);
    };
    double* const gA = c->vg;
    double* const gB = c->vg2;
    const bool use_graph = !c->prof && !c->graph_failed;
    if (use_graph && !c->iter_graph) {
        hipGraph_t graph = nullptr;
        bool ok = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            try {
                iteration(c->vp, c->vp1, gA, gB);
                iteration(c->vp1, c->vp, gB, gA);
            } catch (...) {
                ok = false;
            }
            ok = (hipStreamEndCapture(c->stream, &graph) == hipSuccess) && ok;
        }
        if (ok && graph && hipGraphInstantiate(&c->iter_graph, graph, nullptr, nullptr, 0) != hipSuccess) {
            c->iter_graph = nullptr;
            ok = false;
        }
        if (graph) (void)hipGraphDestroy(graph);
        if (!ok) {
            c->graph_failed = true;
            (void)hipGetLastError();
        }
    }
    const bool graph = use_graph && c->iter_graph;
    c->last_graph = graph ? 1 : 0;
    auto read_sc = [&]() {
        HIP_OK(hipMemcpyAsync(c->red_h, c->sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_OK(hipStreamSynchronize(c->stream));
    };
    read_sc();
    int launched = 0;  // iterations queued so far
    while (c->red_h[SC_DONE] == 0.0) {
        if (graph) {
            HIP_OK(hipGraphLaunch(c->iter_graph, c->stream));
            HIP_OK(hipGraphLaunch(c->iter_graph, c->stream));
            launched += 4;
        } else {
            for (int l = 0; l < 4; ++l) {
                c->prof_iter = ++launched;
                if (launched % 2)
                    iteration(c->vp, c->vp1, gA, gB);
                else
                    iteration(c->vp1, c->vp, gB, gA);
            }
        }
        // the last queued iteration's scalars (the next iteration would finalise them)
        tgms::finalize(c, false);
        read_sc();
    }
    c->prof_iter = -1;
    if (c->prof) {
        // keep the timings of the launches that belong to iterations that ran
        const int ran = (int)c->red_h[SC_IT] + (c->red_h[SC_FLAG] != 0.0 ? 1 : 0);
        for (size_t k = prof_first; k < c->prof_rec.size(); ++k) {
            const auto& r = c->prof_rec[k];
            if (r.iter > ran) continue;
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, r.e1, r.e2));
            c->prof_acc_ms[r.id] += ms;
            c->prof_acc_n[r.id] += 1;
        }
        c->prof_rec.resize(prof_first);
        c->ev_used = ev_first;
    }
    const int it = (int)c->red_h[SC_IT];
    const double rel = std::sqrt(c->red_h[SC_REL2]);
    *st = TGMS_OK;
    if (c->red_h[SC_FLAG] != 0.0)
        *st = TGMS_E_BREAKDOWN;
    else if (c->red_h[SC_Z02] > 0.0 && rel > rtol)
        *st = TGMS_E_NOTCONV;
    c->alphas.clear();
    c->betas.clear();
    if (it > 0 && keep_history) {
        std::vector<double> h(2 * (size_t)it);
        HIP_OK(hipMemcpyAsync(h.data(), c->hist, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
        HIP_OK(hipStreamSynchronize(c->stream));
        for (int k = 0; k < it; ++k) {
            c->alphas.push_back(h[2 * k]);
            if (k + 1 < it) c->betas.push_back(h[2 * k + 1]);
        }
    }
    // Step 4: v = vbar + g + C psi
    tgms::curl_add(c, c->vx, c->fF, u);
    if (p) tgms::pressure(c, u, p);
    HIP_OK(hipStreamSynchronize(c->stream));
    if (iters) *iters = it;
    if (relres) *relres = rel;
    if (*st != TGMS_OK) {
        g_last_error = (*st == TGMS_E_NOTCONV) ? "PCG did not converge within maxit" : "PCG breakdown";
    }
}

}  // namespace

// ---------------------------------------------------------------- allocation-free solve
// The PCG's device scalars, the per-workgroup partial sums of its reductions and its
// alpha / beta history live here for tgms_solve_noalloc instead of in buffers of the
// context.  One copy per device, kept until the process ends.  Host code uses the
// device address from hipGetSymbolAddress (kept per device in g_scratch_ptr), never
// the array's name.
static constexpr long long kScratchDoubles = 65536;  // 512 KB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {nullptr};

// the current device's copy of the scratch array (looked up on its first use)
double* device_scratch() {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw TgmsError{TGMS_E_DEVICE, "device ordinal out of range"};
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = (double*)ptr;
    }
    return g_scratch_ptr[dev];
}

long long noalloc_need(const tgms_ctx* c, int maxit) {
    return SC_COUNT + 4LL * tgms::pcg_tiles(const_cast<tgms_ctx*>(c)) + 2LL * ((long long)maxit + 2);
}

void solve_noalloc_impl(tgms_ctx* c, const double* F, const double* g_bnd, double rtol, int maxit, double* u,
                        double* p, int* iters, double* relres, tgms_status* st) {
    if (!c || !F || !u) throw TgmsError{TGMS_E_INVAL, "null argument"};
    if (maxit < 0 || noalloc_need(c, maxit) > kScratchDoubles)
        throw TgmsError{TGMS_E_INVAL, "maxit outside [0, " +
                                          std::to_string((kScratchDoubles - noalloc_need(c, 0)) / 2) +
                                          "] for the allocation-free solve"};
    double* base = device_scratch();
    // the context's own buffers are swapped for the scratch array for this call
    struct Swap {
        tgms_ctx* c;
        double *sc, *part, *part2, *hist;
        int hist_cap;
        bool graph_failed, prof;
        ~Swap() {
            c->sc = sc;
            c->part = part;
            c->part2 = part2;
            c->hist = hist;
            c->hist_cap = hist_cap;
            c->graph_failed = graph_failed;
            c->prof = prof;
        }
    } swap{c, c->sc, c->part, c->part2, c->hist, c->hist_cap, c->graph_failed, c->prof};
    const long long nt = tgms::pcg_tiles(c);
    c->sc = base;
    c->part = base + SC_COUNT;
    c->part2 = c->part + 3 * nt;
    c->hist = c->part2 + nt;
    c->hist_cap = maxit + 2;  // the history fits: no allocation in the solve
    c->graph_failed = true;   // direct launches (instantiating a graph allocates)
    c->prof = false;          // no event pairs (they come from a growing pool)
    tgms::enter(c);
    tgms::zero(c, base, sizeof(double) * (size_t)noalloc_need(c, maxit));  // a fill kernel
    solve_impl(c, F, g_bnd, rtol, maxit, u, p, iters, relres, st, false);
}

constexpr char kMagic[8] = {'T', 'G', 'M', 'S', 'C', 'S', '0', '1'};

struct FileHeader {
    char magic[8];
    int32_t version, nx, ny, bx, by, overlap, precision, coarse_space, mobility, ne, jmax, pad;
    double eta, tol, H;
};

void save_impl(const tgms_ctx* c, const char* path) {
    tgms_ctx* cc = const_cast<tgms_ctx*>(c);
    const long long ncell = (long long)c->nx * c->ny;
    const size_t nq = (size_t)c->ne * c->jmax * c->jmax;
    Artefact a;
    a.kinv.resize(ncell);
    a.a.resize(ncell);
    a.eigs.resize((size_t)c->ne * c->jmax);
    a.YQ.resize(nq);
    HIP_OK(hipMemcpyAsync(a.kinv.data(), c->kinv, sizeof(double) * ncell, hipMemcpyDeviceToHost, cc->stream));
    HIP_OK(hipMemcpyAsync(a.a.data(), c->a, sizeof(double) * ncell, hipMemcpyDeviceToHost, cc->stream));
    HIP_OK(hipMemcpyAsync(a.eigs.data(), c->eigs, sizeof(double) * a.eigs.size(), hipMemcpyDeviceToHost, cc->stream));
    HIP_OK(hipMemcpyAsync(a.YQ.data(), c->YQ, sizeof(double) * nq, hipMemcpyDeviceToHost, cc->stream));
    HIP_OK(hipStreamSynchronize(cc->stream));
    FileHeader h{};
    std::memcpy(h.magic, kMagic, 8);
    h.version = 1;
    h.nx = c->nx; h.ny = c->ny; h.bx = c->bx; h.by = c->by;
    h.overlap = c->overlap; h.precision = c->precision; h.coarse_space = c->coarse_space;
    h.mobility = c->mobility_updated ? 1 : 0;
    h.ne = c->ne; h.jmax = c->jmax;
    h.eta = c->eta; h.tol = c->tol; h.H = c->H;
    FILE* f = std::fopen(path, "wb");
    if (!f) throw TgmsError{TGMS_E_INVAL, std::string("cannot open ") + path + " for writing"};
    bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1;
    ok = ok && std::fwrite(a.kinv.data(), sizeof(double), ncell, f) == (size_t)ncell;
    ok = ok && std::fwrite(a.a.data(), sizeof(double), ncell, f) == (size_t)ncell;
    ok = ok && std::fwrite(c->counts_h.data(), sizeof(int), c->ne, f) == (size_t)c->ne;
    ok = ok && std::fwrite(a.eigs.data(), sizeof(double), a.eigs.size(), f) == a.eigs.size();
    ok = ok && std::fwrite(a.YQ.data(), sizeof(double), nq, f) == nq;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) throw TgmsError{TGMS_E_INVAL, std::string("writing ") + path + " failed"};
}

void load_impl(const char* path, const tgms_options* opt, tgms_ctx** out) {
    FILE* f = std::fopen(path, "rb");
    if (!f) throw TgmsError{TGMS_E_INVAL, std::string("cannot open ") + path};
    struct Closer {
        FILE* f;
        ~Closer() { std::fclose(f); }
    } closer{f};
    FileHeader h{};
    if (std::fread(&h, sizeof(h), 1, f) != 1 || std::memcmp(h.magic, kMagic, 8) != 0 || h.version != 1)
        throw TgmsError{TGMS_E_INVAL, std::string(path) + " is not a saved tgms context (version 1)"};
    if (h.nx <= 0 || h.ny <= 0 || h.bx <= 0 || h.by <= 0 || h.nx % h.bx || h.ny % h.by || h.ne < 0 || h.jmax <= 0 ||
        (long long)h.nx * h.ny > (1ll << 31))
        throw TgmsError{TGMS_E_INVAL, std::string(path) + ": inconsistent sizes"};
    const int Nx = h.nx / h.bx, Ny = h.ny / h.by;
    if (h.ne != (Nx - 1) * Ny + Nx * (Ny - 1) || h.jmax != std::max(h.bx, h.by))
        throw TgmsError{TGMS_E_INVAL, std::string(path) + ": inconsistent sizes"};
    Artefact a;
    const long long ncell = (long long)h.nx * h.ny;
    const size_t nq = (size_t)h.ne * h.jmax * h.jmax;
    a.kinv.resize(ncell);
    a.a.resize(ncell);
    a.counts.resize(h.ne);
    a.eigs.resize((size_t)h.ne * h.jmax);
    a.YQ.resize(nq);
    bool ok = std::fread(a.kinv.data(), sizeof(double), ncell, f) == (size_t)ncell;
    ok = ok && std::fread(a.a.data(), sizeof(double), ncell, f) == (size_t)ncell;
    ok = ok && std::fread(a.counts.data(), sizeof(int), h.ne, f) == (size_t)h.ne;
    ok = ok && std::fread(a.eigs.data(), sizeof(double), a.eigs.size(), f) == a.eigs.size();
    ok = ok && std::fread(a.YQ.data(), sizeof(double), nq, f) == nq;
    if (!ok) throw TgmsError{TGMS_E_INVAL, std::string(path) + " is truncated"};
    for (int e = 0; e < h.ne; ++e) {
        const int J = e < (Nx - 1) * Ny ? h.by : h.bx;
        if (a.counts[e] < 1 || a.counts[e] > J) throw TgmsError{TGMS_E_INVAL, std::string(path) + ": bad basis count"};
    }
    for (long long k = 0; k < ncell; ++k)
        if (!(a.kinv[k] > 0.0) || !(a.kinv[k] < INFINITY) || !(a.a[k] > 0.0) || !(a.a[k] < INFINITY))
            throw TgmsError{TGMS_E_INVAL, std::string(path) + ": bad cell weights"};
    a.mobility = h.mobility;
    tgms_options o;
    tgms_default_options(&o);
    if (opt) o = *opt;
    o.eta = h.eta;
    o.overlap = h.overlap;
    o.precision = h.precision;
    o.s_scale = h.H;
    o.coarse_space = h.coarse_space;
    o.warm_start = 0;
    o.force_counts = nullptr;
    tgms_grid g{2, h.nx, h.ny, 1, h.bx, h.by, 1};
    setup_impl(&g, nullptr, h.tol, &o, out, &a);
}


tgms_transport_params transport_params(const tgms_transport_params* prm, int nx, int ny, int nz) {
    tgms_transport_params t;
    tgms_default_transport(&t);
    if (prm) t = *prm;
    if (!(t.phi > 0) || !(t.mu_w > 0) || !(t.mu_o > 0) || !(t.tol > 0) || t.max_outer < 0 || !std::isfinite(t.phi) ||
        !std::isfinite(t.mu_w) || !std::isfinite(t.mu_o))
        throw TgmsError{TGMS_E_INVAL, "transport parameters: phi, mu_w, mu_o and tol must be positive and finite"};
    if (t.max_outer == 0) t.max_outer = 8 * (nx + ny + std::max(nz, 1));
    return t;
}

tgms::TransportResult transport_checked(hipStream_t st, int nx, int ny, int nz, const double* u, const double* q,
                                        double* s, double dt, const tgms_transport_params& t) {
    if (nx < 1 || ny < 1 || nz < 0 || !u || !q || !s) throw TgmsError{TGMS_E_INVAL, "transport: bad sizes or null argument"};
    if (!(dt > 0) || !std::isfinite(dt)) throw TgmsError{TGMS_E_INVAL, "transport: dt must be positive"};
    return tgms::transport_step(st, nx, ny, nz, u, q, s, t.phi, dt, t.mu_w, t.mu_o, t.tol, t.max_outer);
}

void impes_impl(tgms_ctx* c, const double* F, double* s, int steps, double dt, int pressure_every,
                const tgms_transport_params* prm, double rtol, int maxit, double* u, int* pcg_iters,
                tgms_status* st) {
    if (!c || !F || !s) throw TgmsError{TGMS_E_INVAL, "null argument"};
    if (steps < 0 || pressure_every < 1) throw TgmsError{TGMS_E_INVAL, "steps >= 0 and pressure_every >= 1"};
    const int nz = c->dim == 3 ? c->d3->g.n[2] : 1;
    const tgms_transport_params t = transport_params(prm, c->nx, c->ny, nz);
    tgms::enter(c);
    const long long nc = (long long)c->nx * c->ny * nz;
    const long long nfaces = c->dim == 3 ? c->d3->g.nf : (long long)c->nf;
    size_t got = 0;
    const size_t bytes = sizeof(double) * ((size_t)nfaces + 2 * (size_t)nc);
    double* w = (double*)tgms::dev_alloc(bytes, &got);
    struct Free {
        double* p;
        size_t b;
        hipStream_t st;
        ~Free() {
            (void)hipStreamSynchronize(st);
            tgms::dev_free(p, b);
        }
    } fr{w, got, c->stream};
    double* uu = u ? u : w;
    double* lam = w + nfaces;
    double* pp = lam + nc;
    int np = 0;
    for (int k = 0; k < steps; ++k) {
        if (k % pressure_every == 0) {
            tgms::total_mobility(c->stream, s, nc, t.mu_w, t.mu_o, lam);
            update_mobility_impl(c, lam);
            int it = 0;
            double rr = 0.0;
            tgms_status sst = TGMS_OK;
            solve_impl(c, F, nullptr, rtol, maxit, uu, pp, &it, &rr, &sst);
            if (pcg_iters) pcg_iters[np] = it;
            ++np;
            if (sst != TGMS_OK) {
                *st = sst;
                return;
            }
        }
        const tgms::TransportResult r = transport_checked(c->stream, c->nx, c->ny, nz, uu, F, s, dt, t);
        if (!r.converged) throw TgmsError{TGMS_E_NOTCONV, "transport: the step did not converge within max_outer"};
    }
}
}  // namespace

// ---------------------------------------------------------------- C ABI
extern "C" {

void tgms_default_options(tgms_options* opt) {
    if (!opt) return;
    opt->eta = 0.2;
    opt->overlap = 2;
    opt->precision = 0;
    opt->s_scale = 1.0;
    opt->stream = nullptr;
    opt->graphs = 1;
    opt->autotune = 1;
    opt->tune_cache = nullptr;
    opt->warm_start = 0;
    opt->cnn_weights = nullptr;
    opt->rq_tol = 1e-6;
    opt->smoother_staging = -1;
    opt->rows_per_thread = 0;
    opt->force_counts = nullptr;
    opt->coarse_space = 0;
    opt->coarse_factor = 0;
    opt->smooth_steps = 1;
    opt->additive = 0;
}

tgms_status tgms_setup(const tgms_grid* grid, const double* kappa, double eig_tol, const tgms_options* opt,
                       tgms_ctx** out) {
    if (out) *out = nullptr;
    return guarded([&] { setup_impl(grid, kappa, eig_tol, opt, out); });
}

tgms_status tgms_solve(tgms_ctx* ctx, const double* F, const double* g_bnd, double rtol, int maxit, double* u,
                       double* p, int* iters, double* relres) {
    tgms_status st = TGMS_OK;
    tgms_status r = guarded([&] { solve_impl(ctx, F, g_bnd, rtol, maxit, u, p, iters, relres, &st); });
    return r != TGMS_OK ? r : st;
}

tgms_status tgms_solve_noalloc(tgms_ctx* ctx, const double* F, const double* g_bnd, double rtol, int maxit,
                               double* u, double* p, int* iters, double* relres) {
    if (ctx && ctx->dim == 3) {
        g_last_error = "solve_noalloc: not available on the cube";
        return TGMS_E_UNSUPPORTED;
    }
    tgms_status st = TGMS_OK;
    tgms_status r = guarded([&] { solve_noalloc_impl(ctx, F, g_bnd, rtol, maxit, u, p, iters, relres, &st); });
    return r != TGMS_OK ? r : st;
}

tgms_status tgms_update_mobility(tgms_ctx* ctx, const double* lambda) {
    return guarded([&] { update_mobility_impl(ctx, lambda); });
}

tgms_status tgms_info(const tgms_ctx* c, tgms_info_t* info) {
    if (!c || !info) {
        g_last_error = "null argument";
        return TGMS_E_INVAL;
    }
    int sum = 0;
    for (int v : c->counts_h) sum += v;
    info->n_coarse_faces = c->ne;
    info->n_blocks = c->nblk;
    info->dim = sum + c->nblk + 1;
    info->n_coarse_spd = c->ncs;
    info->t_setup_ms = c->t_setup_ms;
    info->t_snap_ms = c->t_snap_ms;
    info->t_eig_ms = c->t_eig_ms;
    info->t_coarse_ms = c->t_coarse_ms;
    info->t_smoother_ms = c->t_smoother_ms;
    info->lds_max = c->lds_max;
    info->pcg_graph = c->last_graph;
    info->tuned = c->tuned;
    info->nred = c->nred;
    info->smooth_staged = c->smooth_staged;
    info->warm_accepted = c->warm_accepted;
    info->warm_iters = c->warm_iters;
    info->t_cnn_ms = c->t_cnn_ms;
    info->rows_per_thread = c->rpt;
    info->eig_unconverged = c->eig_unconverged;
    info->coarse_space = c->coarse_space;
    info->nx = c->nx;
    info->ny = c->ny;
    info->bx = c->bx;
    info->by = c->by;
    info->precision = c->precision;
    info->coarse_block = c->cb.nb > 0 ? c->cb.bs : 0;
    info->rt0_block = c->kb.nb > 0 ? c->kb.bs : 0;
    return TGMS_OK;
}

tgms_status tgms_probe_pencil(tgms_ctx* c, double* D, double* S) {
    if (c && c->dim == 3) {
        g_last_error = "probe_pencil: not available on the cube";
        return TGMS_E_UNSUPPORTED;
    }
    if (!c || !D || !S) {
        g_last_error = "null argument";
        return TGMS_E_INVAL;
    }
    if (c->coarse_space == 2) {
        g_last_error = "the RT0 coarse space forms no snapshots or pencils";
        return TGMS_E_INVAL;
    }
    return guarded([&] {
        tgms::enter(c);
        tgms::pencil_probe(c, D, S);
        HIP_OK(hipStreamSynchronize(c->stream));
    });
}

void tgms_trim_device_cache(void) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    DevPool& P = dev_pool();
    std::lock_guard<std::mutex> lock(P.mu);
    for (auto& kv : P.blocks[dev]) (void)hipFree(kv.second);
    P.blocks[dev].clear();
    P.cached[dev] = 0;
}

tgms_status tgms_save(const tgms_ctx* c, const char* path) {
    if (c && c->dim == 3) {
        g_last_error = "save: not available on the cube";
        return TGMS_E_UNSUPPORTED;
    }
    if (!c || !path) {
        g_last_error = "null argument";
        return TGMS_E_INVAL;
    }
    return guarded([&] { save_impl(c, path); });
}

tgms_status tgms_load(const char* path, const tgms_options* opt, tgms_ctx** out) {
    if (out) *out = nullptr;
    if (!path || !out) {
        g_last_error = "null argument";
        return TGMS_E_INVAL;
    }
    return guarded([&] { load_impl(path, opt, out); });
}

tgms_status tgms_get_warm_status(const tgms_ctx* c, int* wstat) {
    if (!c || !wstat) {
        g_last_error = "null argument";
        return TGMS_E_INVAL;
    }
    if (!c->warm) {
        g_last_error = "the context was set up without a warm start";
        return TGMS_E_INVAL;
    }
    std::copy(c->wstat_h.begin(), c->wstat_h.end(), wstat);
    return TGMS_OK;
}

int tgms_cnn_nparams(void) { return tgms::cnn_nparams(); }

size_t tgms_cnn_train_workspace(int n, int H, int W) {
    if (n < 1 || !tgms::cnn_shape_ok(H, W)) return 0;
    return tgms::cnn_train_workspace(n, H, W);
}

tgms_status tgms_cnn_forward(const float* params, const float* X, int n, int H, int W, float* Y, void* stream) {
    if (!params || !X || !Y || n < 1 || !tgms::cnn_shape_ok(H, W)) {
        g_last_error = "bad argument (null pointer, n < 1, or H, W outside [1, 64] with H * W <= 512)";
        return TGMS_E_INVAL;
    }
    return guarded([&] {
        tgms::cnn_forward((hipStream_t)stream, params, X, n, H, W, Y, nullptr);
        HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    });
}

tgms_status tgms_cnn_infer(const float* params, const float* X, int n, int H, int W, float* Y, void* stream) {
    if (!params || !X || !Y || n < 1 || !tgms::cnn_shape_ok(H, W)) {
        g_last_error = "bad argument (null pointer, n < 1, or H, W outside [1, 64] with H * W <= 512)";
        return TGMS_E_INVAL;
    }
    return guarded([&] {
        tgms::cnn_infer_bf16((hipStream_t)stream, params, X, n, H, W, Y);
        HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    });
}

tgms_status tgms_cnn_train_step(float* params, float* adam_m, float* adam_v, int t, float lr, const float* X,
                                const float* V, int n, int H, int W, int k, float* work, double* loss, void* stream) {
    if (!params || !adam_m || !adam_v || !X || !V || !work || t < 1 || !(lr > 0) || n < 1 ||
        !tgms::cnn_shape_ok(H, W) || k < 1 || k > tgms::cnn_kout() || k > W) {
        g_last_error = "bad argument";
        return TGMS_E_INVAL;
    }
    return guarded([&] {
        const double L = tgms::cnn_train_step((hipStream_t)stream, params, adam_m, adam_v, t, lr, X, V, n, H, W, k,
                                              work);
        if (loss) *loss = L;
    });
}

tgms_status tgms_cnn_samples(tgms_ctx* c, float* X, float* V) {
    if (c && c->dim == 3) {
        g_last_error = "cnn_samples: not available on the cube";
        return TGMS_E_UNSUPPORTED;
    }
    if (!c || !X || !V) {
        g_last_error = "null argument";
        return TGMS_E_INVAL;
    }
    if (c->bx != c->by || !tgms::cnn_shape_ok(2 * c->bx, c->bx)) {
        g_last_error = "network samples need square blocks of at most 16 x 16 cells";
        return TGMS_E_UNSUPPORTED;
    }
    if (c->mobility_updated) {
        g_last_error = "network samples describe the setup permeability; not available after a mobility update";
        return TGMS_E_INVAL;
    }
    return guarded([&] {
        tgms::enter(c);
        tgms::cnn_windows(c, X);
        // the dense solve of every face again (same results as setup's), keeping the targets
        // (into scratch outputs: the context's own spectral results stay as set up)
        const int warm = c->warm;
        double* eigs = c->eigs;
        int* counts = c->counts;
        double* Y = c->Y;
        std::vector<DeviceBuf> tmp(4);
        auto get = [&](DeviceBuf& b, size_t bytes) {
            HIP_OK(hipMalloc(&b.p, bytes));
            b.bytes = bytes;
            return b.p;
        };
        auto release = [&] {
            for (auto& b : tmp)
                if (b.p) (void)hipFree(b.p);
            c->eigs = eigs;
            c->counts = counts;
            c->Y = Y;
            c->warm = warm;
        };
        try {
            const size_t nq = (size_t)c->ne * c->jmax * c->jmax;
            c->eigs = (double*)get(tmp[0], sizeof(double) * c->ne * c->jmax);
            c->counts = (int*)get(tmp[1], sizeof(int) * c->ne);
            c->Y = (double*)get(tmp[2], sizeof(double) * nq);
            double* Qd = (double*)get(tmp[3], sizeof(double) * nq);
            c->warm = 0;
            tgms::pencil_eig_q(c, Qd, nullptr, V);
            HIP_OK(hipStreamSynchronize(c->stream));
        } catch (...) {
            (void)hipStreamSynchronize(c->stream);
            release();
            throw;
        }
        release();
    });
}

tgms_status tgms_get_counts(const tgms_ctx* c, int* counts) {
    if (!c || !counts) {
        g_last_error = "null argument";
        return TGMS_E_INVAL;
    }
    std::copy(c->counts_h.begin(), c->counts_h.end(), counts);
    return TGMS_OK;
}

tgms_status tgms_get_eigs(const tgms_ctx* c, double* eigs) {
    if (!c || !eigs) {
        g_last_error = "null argument";
        return TGMS_E_INVAL;
    }
    if (c->dim == 3) {
        std::copy(c->d3->eigs_h.begin(), c->d3->eigs_h.end(), eigs);
        return TGMS_OK;
    }
    return guarded([&] {
        HIP_OK(hipMemcpyAsync(eigs, c->eigs, sizeof(double) * c->ne * c->jmax, hipMemcpyDeviceToHost, c->stream));
        HIP_OK(hipStreamSynchronize(c->stream));
    });
}

tgms_status tgms_last_cond(const tgms_ctx* c, double* cond) {
    if (!c || !cond) {
        g_last_error = "null argument";
        return TGMS_E_INVAL;
    }
    *cond = lanczos_cond(c->alphas, c->betas);
    return TGMS_OK;
}

tgms_status tgms_profile(tgms_ctx* c, int enable) {
    if (c && c->dim == 3) {
        g_last_error = "profile: not available on the cube";
        return TGMS_E_UNSUPPORTED;
    }
    if (!c) {
        g_last_error = "null argument";
        return TGMS_E_INVAL;
    }
    return guarded([&] {
        HIP_OK(hipStreamSynchronize(c->stream));
        c->prof = enable != 0;
        c->prof_rec.clear();
        c->ev_used = 0;
        for (int k = 0; k < tgms::PK_COUNT; ++k) {
            c->prof_acc_ms[k] = 0.0;
            c->prof_acc_n[k] = 0;
        }
    });
}

tgms_status tgms_time_smoother(tgms_ctx* c, int reps, double* avg_ms) {
    if (!c || !avg_ms || reps < 1 || reps > 100000) {
        g_last_error = "bad argument";
        return TGMS_E_INVAL;
    }
    return guarded([&] {
        tgms::enter(c);
        const bool prof = c->prof;
        c->prof = false;
        auto body = [&] {
            if (c->dim == 3)
                tgms3::smooth_patches3(c);
            else if (c->precision != 0)
                tgms::smooth_patches<float>(c, c->fz, nullptr);
            else
                tgms::smooth_patches<double>(c, c->vz, nullptr);
        };
        hipEvent_t a, b;
        HIP_OK(hipEventCreate(&a));
        HIP_OK(hipEventCreate(&b));
        body();  // warm-up
        HIP_OK(hipEventRecord(a, c->stream));
        for (int r = 0; r < reps; ++r) body();
        HIP_OK(hipEventRecord(b, c->stream));
        HIP_OK(hipEventSynchronize(b));
        float ms = 0.f;
        HIP_OK(hipEventElapsedTime(&ms, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        c->prof = prof;
        *avg_ms = ms / reps;
    });
}

tgms_status tgms_time_dir_apply(tgms_ctx* c, int reps, double* avg_ms) {
    if (c && c->dim == 3) {
        g_last_error = "time_dir_apply: not available on the cube";
        return TGMS_E_UNSUPPORTED;
    }
    if (!c || !avg_ms || reps < 1 || reps > 100000) {
        g_last_error = "bad argument";
        return TGMS_E_INVAL;
    }
    return guarded([&] {
        tgms::enter(c);
        const bool prof = c->prof;
        c->prof = false;
        // scalars for a plain update: not done, nothing pending, beta = 1/2 (a solve
        // sets every scalar again before it reads one)
        for (int k = 0; k < SC_COUNT; ++k) c->red_h[k] = 0.0;
        c->red_h[SC_BETA] = 0.5;
        HIP_OK(hipMemcpyAsync(c->sc, c->red_h, SC_COUNT * sizeof(double), hipMemcpyHostToDevice, c->stream));
        auto body = [&] { tgms::dir_apply(c, c->vz, c->vp, c->vp1, c->vq); };
        hipEvent_t a, b;
        HIP_OK(hipEventCreate(&a));
        HIP_OK(hipEventCreate(&b));
        body();  // warm-up
        HIP_OK(hipEventRecord(a, c->stream));
        for (int r = 0; r < reps; ++r) body();
        HIP_OK(hipEventRecord(b, c->stream));
        HIP_OK(hipEventSynchronize(b));
        float ms = 0.f;
        HIP_OK(hipEventElapsedTime(&ms, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        c->prof = prof;
        *avg_ms = ms / reps;
    });
}

tgms_status tgms_profile_get(tgms_ctx* c, int kernel, int* launches, double* total_ms) {
    if (c && c->dim == 3) {
        g_last_error = "profile_get: not available on the cube";
        return TGMS_E_UNSUPPORTED;
    }
    if (!c || !launches || !total_ms || kernel < 0 || kernel >= tgms::PK_COUNT) {
        g_last_error = "bad argument";
        return TGMS_E_INVAL;
    }
    return guarded([&] {
        HIP_OK(hipStreamSynchronize(c->stream));
        int n = c->prof_acc_n[kernel];
        double t = c->prof_acc_ms[kernel];
        for (auto& r : c->prof_rec) {
            if (r.id != kernel) continue;
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, r.e1, r.e2));
            t += ms;
            ++n;
        }
        *launches = n;
        *total_ms = t;
    });
}

void tgms_default_transport(tgms_transport_params* prm) {
    if (!prm) return;
    prm->phi = 0.2;
    prm->mu_w = 1.0;
    prm->mu_o = 5.0;
    prm->tol = 1e-12;
    prm->max_outer = 0;
}

tgms_status tgms_total_mobility(const double* s, long long n, const tgms_transport_params* prm, double* lambda,
                                void* stream) {
    return guarded([&] {
        if (n < 0 || (n > 0 && (!s || !lambda))) throw TgmsError{TGMS_E_INVAL, "bad size or null argument"};
        const tgms_transport_params t = transport_params(prm, 1, 1, 1);
        if (n > 0) tgms::total_mobility((hipStream_t)stream, s, n, t.mu_w, t.mu_o, lambda);
    });
}

tgms_status tgms_transport_step(int nx, int ny, int nz, const double* u, const double* q, double* s, double dt,
                                const tgms_transport_params* prm, void* stream, long long* outer, double* residual) {
    tgms_status st = TGMS_OK;
    tgms_status r = guarded([&] {
        const tgms_transport_params t = transport_params(prm, nx, ny, nz);
        const tgms::TransportResult res = transport_checked((hipStream_t)stream, nx, ny, nz, u, q, s, dt, t);
        if (outer) *outer = res.sweeps;
        if (residual) *residual = res.residual;
        if (!res.converged) {
            g_last_error = "transport: the step did not converge within max_outer";
            st = TGMS_E_NOTCONV;
        }
    });
    return r != TGMS_OK ? r : st;
}

tgms_status tgms_impes(tgms_ctx* ctx, const double* F, double* s, int steps, double dt, int pressure_every,
                       const tgms_transport_params* prm, double rtol, int maxit, double* u, int* pcg_iters) {
    tgms_status st = TGMS_OK;
    tgms_status r =
        guarded([&] { impes_impl(ctx, F, s, steps, dt, pressure_every, prm, rtol, maxit, u, pcg_iters, &st); });
    return r != TGMS_OK ? r : st;
}

void tgms_destroy(tgms_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->d3) tgms3::destroy3(c);
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->iter_graph) (void)hipGraphExecDestroy(c->iter_graph);
    for (auto& b : c->owned) tgms::dev_free(b.p, b.bytes);
    if (c->red_h) (void)hipHostFree(c->red_h);
    if (c->ev_enter) (void)hipEventDestroy(c->ev_enter);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char* tgms_last_error(void) { return g_last_error.c_str(); }

tgms_status tgms_apply_A(tgms_ctx* c, const double* x, double* y) {
    if (!c || !x || !y) {
        g_last_error = "null argument";
        return TGMS_E_INVAL;
    }
    return guarded([&] {
        tgms::enter(c);
        if (c->dim == 3)
            tgms3::apply_A3(c, x, y);
        else
            tgms::faces_A_probe(c, x, y);
        HIP_OK(hipStreamSynchronize(c->stream));
    });
}

tgms_status tgms_preprocess(tgms_ctx* c, const double* F, const double* g_bnd, double* vbar) {
    if (!c || !F || !vbar) {
        g_last_error = "null argument";
        return TGMS_E_INVAL;
    }
    return guarded([&] {
        tgms::enter(c);
        if (c->dim == 3) {
            if (g_bnd) throw TgmsError{TGMS_E_UNSUPPORTED, "on the cube only the no-flow boundary (g_bnd NULL)"};
            tgms3::preprocess3(c, F, vbar);
        } else {
            tgms::preprocess(c, F, g_bnd, vbar, c->cellw2);
        }
        HIP_OK(hipStreamSynchronize(c->stream));
    });
}

tgms_status tgms_apply_precond(tgms_ctx* c, int which, const double* r, double* z) {
    if (!c || !r || !z || which < 0 || which > 2) {
        g_last_error = "bad argument";
        return TGMS_E_INVAL;
    }
    return guarded([&] {
        tgms::enter(c);
        if (c->dim == 3) {
            tgms3::apply_precond3(c, which, r, z);
            return;
        }
        tgms::curlT(c, r, c->vgold);
        precond(c, which, c->vgold, c->vq);
        tgms::curl_add(c, c->vq, nullptr, z);
        HIP_OK(hipStreamSynchronize(c->stream));
    });
}

}  // extern "C"
