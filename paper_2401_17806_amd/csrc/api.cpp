// C ABI entry points: argument checking, host-side mesh setup (Section 3.1), reference
// operators (Section 3.4), device buffers and the CG driver (Section 3.3).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <mutex>
#include <thread>
#include <vector>

#include "sld_internal.h"
#include "state_internal.h"

namespace {
thread_local std::string g_err;

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Graph capture on one thread and device setup or teardown on another must not overlap: the
// runtime rejects synchronous copies and may serialise frees against a capturing stream.  Every
// capture, and every create/destroy that touches device memory, holds this lock.
std::mutex& device_setup_mutex() {
    static std::mutex mu;
    return mu;
}

// Host -> device uploads and clears during setup run on a private non-blocking stream (never
// the legacy null stream), then wait for it.
struct Uploader {
    hipStream_t s = nullptr;
    hipError_t err = hipSuccess;
    Uploader() { err = hipStreamCreateWithFlags(&s, hipStreamNonBlocking); }
    ~Uploader() {
        if (s) (void)hipStreamDestroy(s);
    }
    void copy(void* dst, const void* src, size_t bytes) {
        if (err == hipSuccess && bytes) err = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    }
    void zero(void* dst, size_t bytes) {
        if (err == hipSuccess && bytes) err = hipMemsetAsync(dst, 0, bytes, s);
    }
    hipError_t finish() {
        if (err == hipSuccess) err = hipStreamSynchronize(s);
        return err;
    }
};

template <class T>
void dfree(T* p) {
    if (p) (void)hipFree(p);
}

template <class T>
hipError_t dalloc(T** p, size_t count) {
    return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (count ? count : 1));
}

void free_mesh(sld_mesh_s* m) {
    if (!m) return;
    dfree(m->geo);
    dfree(m->nbr);
    dfree(m->edges);
    dfree(m->tedges);
    dfree(m->halo_pad);
    dfree(m->perm);
    dfree(m->geo_i);
    dfree(m->geo_nb);
    dfree(m->nbr_i);
    delete m;
}

// Drop one reference; the last one frees host tables and device memory.
void release_mesh(sld_mesh_s* m) {
    if (m->refs.fetch_sub(1) != 1) return;
    if (m->device < 0) {
        free_mesh(m);
        return;
    }
    DeviceGuard dg(m->device);
    std::lock_guard<std::mutex> lk(device_setup_mutex());
    free_mesh(m);
}

template <int P>
size_t ops_size() { return sizeof(RefOps<P>); }

int build_ops(int p, void** host, size_t* bytes) {
    int rc = 0;
    switch (p) {
#define SLD_OPS_CASE(PP)                                          \
    case PP: {                                                    \
        RefOps<PP>* o = new (std::nothrow) RefOps<PP>();          \
        if (!o) return -1;                                        \
        rc = build_refops<PP>(o);                                 \
        *host = o;                                                \
        *bytes = sizeof(RefOps<PP>);                              \
    } break;
        SLD_OPS_CASE(1)
        SLD_OPS_CASE(2)
        SLD_OPS_CASE(3)
        SLD_OPS_CASE(4)
#undef SLD_OPS_CASE
        default:
            return -2;
    }
    return rc;
}

// float copy of the operators (built on the host, uploaded once)
template <int P>
int build_sl_p(std::vector<unsigned char>* out) {
    out->assign(sizeof(SlOps<P>), 0);
    return build_slops<P>(reinterpret_cast<SlOps<P>*>(out->data()));
}

int build_sl(int p, std::vector<unsigned char>* out) {
    switch (p) {
        case 1: return build_sl_p<1>(out);
        case 2: return build_sl_p<2>(out);
        case 3: return build_sl_p<3>(out);
        case 4: return build_sl_p<4>(out);
        default: return 1;
    }
}

size_t ops32_bytes(int p) {
    switch (p) {
        case 1: return sizeof(RefOps32<1>);
        case 2: return sizeof(RefOps32<2>);
        case 3: return sizeof(RefOps32<3>);
        case 4: return sizeof(RefOps32<4>);
        default: return 0;
    }
}

void round_ops(int p, const void* in, void* out) {
    switch (p) {
        case 1: round_refops<1>(*static_cast<const RefOps<1>*>(in), static_cast<RefOps32<1>*>(out)); break;
        case 2: round_refops<2>(*static_cast<const RefOps<2>*>(in), static_cast<RefOps32<2>*>(out)); break;
        case 3: round_refops<3>(*static_cast<const RefOps<3>*>(in), static_cast<RefOps32<3>*>(out)); break;
        case 4: round_refops<4>(*static_cast<const RefOps<4>*>(in), static_cast<RefOps32<4>*>(out)); break;
        default: break;
    }
}

void free_ops_host(int p, void* h) {
    switch (p) {
        case 1: delete static_cast<RefOps<1>*>(h); break;
        case 2: delete static_cast<RefOps<2>*>(h); break;
        case 3: delete static_cast<RefOps<3>*>(h); break;
        case 4: delete static_cast<RefOps<4>*>(h); break;
        default: break;
    }
}

const double* ops_w(const sld_disc_s* d) {
    switch (d->p) {
        case 1: return static_cast<const RefOps<1>*>(d->ops_host)->w;
        case 2: return static_cast<const RefOps<2>*>(d->ops_host)->w;
        case 3: return static_cast<const RefOps<3>*>(d->ops_host)->w;
        case 4: return static_cast<const RefOps<4>*>(d->ops_host)->w;
        default: return nullptr;
    }
}

void free_disc(sld_disc_s* d) {
    if (!d) return;
    CgWork& w = d->cg;
    dfree(w.x);
    dfree(w.e);
    for (int k = 0; k < 2; ++k) {
        dfree(w.r[k]);
        dfree(w.q[k]);
        dfree(w.d[k]);
    }
    dfree(w.b);
    dfree(w.part);
    dfree(w.part_s);
    for (int k = 0; k < 2; ++k) {
        dfree(w.r32[k]);
        dfree(w.q32[k]);
        dfree(w.d32[k]);
    }
    dfree(w.e32);
    dfree(w.part32);
    dfree(w.scal_in);
    if (w.host_scal_in) (void)hipHostFree(w.host_scal_in);
    if (w.graph32) (void)hipGraphExecDestroy(w.graph32);
    dfree(d->ops32_dev);
    dfree(d->sl_dev);
    dfree(d->mx_dev);
    dfree(w.scal);
    dfree(w.wall_i);
    if (w.graph) (void)hipGraphExecDestroy(w.graph);
    if (w.graph_shift) (void)hipGraphExecDestroy(w.graph_shift);
    if (w.capture) (void)hipStreamDestroy(w.capture);
    if (w.host_scal) (void)hipHostFree(w.host_scal);
    for (hipEvent_t e : w.events) (void)hipEventDestroy(e);
    dfree(d->ops_dev);
    free_ops_host(d->p, d->ops_host);
    delete d;
}

#define SLD_REQUIRE(cond, code, msg) \
    do {                             \
        if (!(cond)) {               \
            sld_set_error(msg);      \
            return code;             \
        }                            \
    } while (0)

}  // namespace

void sld_set_error(const std::string& msg) { g_err = msg; }

extern "C" {

const char* sld_last_error(void) { return g_err.c_str(); }

int32_t sld_abi_version(void) { return 3; }

sld_status sld_mesh_create(const double* xy, int64_t nv, const int32_t* tri, int64_t ne,
                           const double* period, int32_t device, sld_mesh* out) {
    SLD_REQUIRE(out, SLD_E_INVALID, "sld_mesh_create: out is NULL");
    *out = nullptr;
    SLD_REQUIRE(xy && tri, SLD_E_INVALID, "sld_mesh_create: xy or tri is NULL");
    SLD_REQUIRE(nv >= 3 && ne >= 1, SLD_E_INVALID, "sld_mesh_create: need nv >= 3 and ne >= 1");
    SLD_REQUIRE(ne < (int64_t(1) << 28), SLD_E_BUDGET, "sld_mesh_create: ne must be < 2^28");
    if (period) {
        SLD_REQUIRE(std::isfinite(period[0]) && std::isfinite(period[1]) && period[0] > 0 &&
                        period[1] > 0,
                    SLD_E_INVALID, "sld_mesh_create: period must be positive and finite");
    }
    if (device != -1) {
        int ndev = 0;
        SLD_HIP_CHECK(hipGetDeviceCount(&ndev));
        SLD_REQUIRE(device >= 0 && device < ndev, SLD_E_INVALID,
                    "sld_mesh_create: bad device ordinal");
    }

    sld_mesh_s* m = new (std::nothrow) sld_mesh_s();
    SLD_REQUIRE(m, SLD_E_NOMEM, "sld_mesh_create: host allocation failed");
    m->device = device;
    m->ne = ne;
    m->nv = nv;
    m->periodic = period != nullptr;
    try {
        m->P.resize(size_t(ne) * 6);
        std::vector<double4> geo(ne);
        double area = 0;
        for (int64_t i = 0; i < ne; ++i) {
            int32_t v[3] = {tri[3 * i], tri[3 * i + 1], tri[3 * i + 2]};
            for (int k = 0; k < 3; ++k) {
                if (v[k] < 0 || v[k] >= nv) {
                    free_mesh(m);
                    sld_set_error("sld_mesh_create: vertex id out of range in triangle " +
                                  std::to_string(i));
                    return SLD_E_MESH;
                }
            }
            double x0 = xy[2 * v[0]], y0 = xy[2 * v[0] + 1];
            double px[3], py[3];
            for (int k = 0; k < 3; ++k) {
                double x = xy[2 * v[k]], y = xy[2 * v[k] + 1];
                if (period) {
                    x -= period[0] * std::nearbyint((x - x0) / period[0]);
                    y -= period[1] * std::nearbyint((y - y0) / period[1]);
                }
                px[k] = x;
                py[k] = y;
                m->P[6 * i + 2 * k] = x;
                m->P[6 * i + 2 * k + 1] = y;
            }
            double e1x = px[1] - px[0], e1y = py[1] - py[0];
            double e2x = px[2] - px[0], e2y = py[2] - py[0];
            double det = e1x * e2y - e1y * e2x;
            if (!(det > 0) || !std::isfinite(det)) {
                free_mesh(m);
                sld_set_error("sld_mesh_create: triangle " + std::to_string(i) +
                              " has non-positive area (vertices must be counter-clockwise)");
                return SLD_E_MESH;
            }
            area += 0.5 * det;
            geo[i] = make_double4(e1x, e1y, e2x, e2y);
        }
        m->area_total = area;

        // edges in order of first appearance
        std::unordered_map<uint64_t, int32_t> edge_of;
        edge_of.reserve(size_t(ne) * 2);
        std::vector<int4> nbr(ne, make_int4(-1, -1, -1, 0));
        std::vector<int4> tedges(ne, make_int4(0, 0, 0, 0));
        m->tedge.assign(size_t(ne) * 3, -1);
        for (int64_t i = 0; i < ne; ++i) {
            for (int al = 0; al < 3; ++al) {
                uint32_t va = (uint32_t)tri[3 * i + al], vb = (uint32_t)tri[3 * i + (al + 1) % 3];
                if (va == vb) {
                    free_mesh(m);
                    sld_set_error("sld_mesh_create: degenerate edge in triangle " + std::to_string(i));
                    return SLD_E_MESH;
                }
                uint64_t key = va < vb ? (uint64_t(va) << 32 | vb) : (uint64_t(vb) << 32 | va);
                auto it = edge_of.find(key);
                int32_t j;
                if (it == edge_of.end()) {
                    j = (int32_t)m->left.size();
                    edge_of.emplace(key, j);
                    m->left.push_back((int32_t)i);
                    m->right.push_back(-1);
                    m->alpha_l.push_back(al);
                    m->alpha_r.push_back(-1);
                } else {
                    j = it->second;
                    int32_t l = m->left[j], all = m->alpha_l[j];
                    if (m->right[j] != -1) {
                        free_mesh(m);
                        sld_set_error("sld_mesh_create: non-manifold edge (more than two triangles)");
                        return SLD_E_MESH;
                    }
                    if ((uint32_t)tri[3 * l + all] != vb || (uint32_t)tri[3 * l + (all + 1) % 3] != va) {
                        free_mesh(m);
                        sld_set_error("sld_mesh_create: inconsistent orientation across an edge");
                        return SLD_E_MESH;
                    }
                    if (l == (int32_t)i) {
                        free_mesh(m);
                        sld_set_error("sld_mesh_create: an edge joins a triangle to itself");
                        return SLD_E_MESH;
                    }
                    m->right[j] = (int32_t)i;
                    m->alpha_r[j] = al;
                }
                m->tedge[3 * i + al] = j;
            }
        }
        m->nd = (int64_t)m->left.size();
        std::vector<int4> edges(m->nd);
        m->shift.assign(size_t(m->nd) * 2, 0.0);
        for (int64_t j = 0; j < m->nd; ++j) {
            int32_t l = m->left[j], r = m->right[j], al = m->alpha_l[j], ar = m->alpha_r[j];
            edges[j] = make_int4(l, r, al, ar);
            int* nl = al == 0 ? &nbr[l].x : (al == 1 ? &nbr[l].y : &nbr[l].z);
            int* tl = al == 0 ? &tedges[l].x : (al == 1 ? &tedges[l].y : &tedges[l].z);
            *nl = pack_nbr(r, ar);
            *tl = int(2 * j);
            if (r >= 0) {
                int* nr = ar == 0 ? &nbr[r].x : (ar == 1 ? &nbr[r].y : &nbr[r].z);
                int* tr = ar == 0 ? &tedges[r].x : (ar == 1 ? &tedges[r].y : &tedges[r].z);
                *nr = pack_nbr(l, al);
                *tr = int(2 * j + 1);
                // r's copy of B (its vertex ar) minus l's copy of B (l's vertex al+1)
                for (int c = 0; c < 2; ++c) {
                    double sB = m->P[6 * r + 2 * ar + c] - m->P[6 * l + 2 * ((al + 1) % 3) + c];
                    double sA = m->P[6 * r + 2 * ((ar + 1) % 3) + c] - m->P[6 * l + 2 * al + c];
                    double tol = 1e-9 * (1.0 + std::fabs(m->P[6 * l + 2 * al + c]));
                    if (std::fabs(sA - sB) > tol || (!period && std::fabs(sA) > tol)) {
                        free_mesh(m);
                        sld_set_error("sld_mesh_create: neighbouring triangles disagree on an edge "
                                      "(triangle larger than half a period?)");
                        return SLD_E_MESH;
                    }
                    m->shift[2 * j + c] = sB;
                }
            }
        }
        // internal order: Morton curve over (periodically wrapped) centroids
        std::vector<int> perm(ne), inv(ne);
        {
            double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
            std::vector<double> cx(ne), cy(ne);
            for (int64_t i = 0; i < ne; ++i) {
                double c[2];
                for (int k = 0; k < 2; ++k) {
                    c[k] = (m->P[6 * i + k] + m->P[6 * i + 2 + k] + m->P[6 * i + 4 + k]) / 3.0;
                    if (period) c[k] -= period[k] * std::floor(c[k] / period[k]);
                    lo[k] = std::min(lo[k], c[k]);
                    hi[k] = std::max(hi[k], c[k]);
                }
                cx[i] = c[0];
                cy[i] = c[1];
            }
            std::vector<std::pair<uint32_t, int>> key(ne);
            for (int64_t i = 0; i < ne; ++i) {
                uint32_t q[2];
                const double c[2] = {cx[i], cy[i]};
                for (int k = 0; k < 2; ++k) {
                    const double span = hi[k] > lo[k] ? hi[k] - lo[k] : 1.0;
                    q[k] = (uint32_t)std::min(65535.0, std::floor((c[k] - lo[k]) / span * 65536.0));
                }
                uint32_t code = 0;
                for (int bit = 0; bit < 16; ++bit)
                    code |= ((q[0] >> bit) & 1u) << (2 * bit) | ((q[1] >> bit) & 1u) << (2 * bit + 1);
                key[i] = {code, (int)i};
            }
            std::sort(key.begin(), key.end());
            for (int64_t i = 0; i < ne; ++i) {
                perm[i] = key[i].second;
                inv[key[i].second] = (int)i;
            }
        }
        std::vector<double4> geo_i(ne);
        std::vector<int4> nbr_i(ne);
        for (int64_t i = 0; i < ne; ++i) {
            const int c = perm[i];
            geo_i[i] = geo[c];
            int v[3] = {nbr[c].x, nbr[c].y, nbr[c].z};
            for (int al = 0; al < 3; ++al) v[al] = v[al] < 0 ? -1 : pack_nbr(inv[v[al] >> 2], v[al] & 3);
            nbr_i[i] = make_int4(v[0], v[1], v[2], 0);
        }
        // the neighbour's geometry across each local edge (zeros on a wall), so that the CG
        // iteration reads it without first reading the neighbour's id
        std::vector<double4> geo_nb(size_t(ne) * 3);
        for (int64_t i = 0; i < ne; ++i) {
            const int v[3] = {nbr_i[i].x, nbr_i[i].y, nbr_i[i].z};
            for (int al = 0; al < 3; ++al)
                geo_nb[size_t(i) * 3 + al] = v[al] < 0 ? make_double4(0, 0, 0, 0) : geo_i[v[al] >> 2];
        }
        // tiles of kTriPerBlock consecutive (internal) triangles: halo lists and local slots
        const int64_t ntiles = (ne + kTriPerBlock - 1) / kTriPerBlock;
        std::vector<int> halo_off(ntiles + 1, 0), halo_ids;
        halo_ids.reserve(size_t(ne));
        for (int64_t t = 0; t < ntiles; ++t) {
            const int64_t i0 = t * kTriPerBlock, i1 = std::min<int64_t>(ne, i0 + kTriPerBlock);
            std::vector<int> ext;
            for (int64_t i = i0; i < i1; ++i)
                for (int al = 0; al < 3; ++al) {
                    const int nb = al == 0 ? nbr_i[i].x : (al == 1 ? nbr_i[i].y : nbr_i[i].z);
                    if (nb < 0) continue;
                    const int r = nb >> 2;
                    if (r < i0 || r >= i1) ext.push_back(r);
                }
            std::sort(ext.begin(), ext.end());
            ext.erase(std::unique(ext.begin(), ext.end()), ext.end());
            if ((int)ext.size() + kTriPerBlock >= kSlotWall) {
                free_mesh(m);
                sld_set_error("sld_mesh_create: a tile's halo is too large");
                return SLD_E_MESH;
            }
            for (int64_t i = i0; i < i1; ++i) {
                int slots[3];
                for (int al = 0; al < 3; ++al) {
                    const int nb = al == 0 ? nbr_i[i].x : (al == 1 ? nbr_i[i].y : nbr_i[i].z);
                    if (nb < 0) {
                        slots[al] = kSlotWall;
                        continue;
                    }
                    const int r = nb >> 2;
                    if (r >= i0 && r < i1) slots[al] = int(r - i0);
                    else
                        slots[al] = kTriPerBlock +
                                    int(std::lower_bound(ext.begin(), ext.end(), r) - ext.begin());
                }
                nbr_i[i].w = slots[0] | (slots[1] << 10) | (slots[2] << 20);
            }
            m->hmax = std::max<int>(m->hmax, (int)ext.size());
            halo_ids.insert(halo_ids.end(), ext.begin(), ext.end());
            halo_off[t + 1] = (int)halo_ids.size();
        }
        m->halo_total = (int64_t)halo_ids.size();
        // fixed-stride copy of the halo lists (hmax entries per tile, -1 padded) so that a
        // tile's halo ids are addressable without first reading its offset
        const int hstride = std::max(m->hmax, 1);
        std::vector<int> halo_pad(size_t(ntiles) * hstride, -1);
        for (int64_t t = 0; t < ntiles; ++t)
            for (int k = halo_off[t]; k < halo_off[t + 1]; ++k)
                halo_pad[size_t(t) * hstride + (k - halo_off[t])] = halo_ids[k];
        if (device == -1) {
            *out = m;  // host-only handle: tables and node queries, no device work
            return SLD_OK;
        }
        DeviceGuard dg(device);
        if (!dg.ok) {
            free_mesh(m);
            sld_set_error("sld_mesh_create: hipSetDevice failed");
            return SLD_E_HIP;
        }
        std::lock_guard<std::mutex> lk(device_setup_mutex());
        Uploader up;
        hipError_t e = up.err;
        if (e == hipSuccess) e = dalloc(&m->geo, ne);
        if (e == hipSuccess) e = dalloc(&m->nbr, ne);
        if (e == hipSuccess) e = dalloc(&m->tedges, ne);
        if (e == hipSuccess) e = dalloc(&m->edges, m->nd);
        if (e == hipSuccess) e = dalloc(&m->perm, ne);
        if (e == hipSuccess) e = dalloc(&m->geo_i, ne);
        if (e == hipSuccess) e = dalloc(&m->geo_nb, size_t(ne) * 3);
        if (e == hipSuccess) e = dalloc(&m->nbr_i, ne);
        if (e == hipSuccess) e = dalloc(&m->halo_pad, halo_pad.size());
        if (e == hipSuccess) {
            up.copy(m->perm, perm.data(), sizeof(int) * ne);
            up.copy(m->geo_i, geo_i.data(), sizeof(double4) * ne);
            up.copy(m->geo_nb, geo_nb.data(), sizeof(double4) * geo_nb.size());
            up.copy(m->nbr_i, nbr_i.data(), sizeof(int4) * ne);
            up.copy(m->halo_pad, halo_pad.data(), sizeof(int) * halo_pad.size());
            up.copy(m->geo, geo.data(), sizeof(double4) * ne);
            up.copy(m->nbr, nbr.data(), sizeof(int4) * ne);
            up.copy(m->tedges, tedges.data(), sizeof(int4) * ne);
            up.copy(m->edges, edges.data(), sizeof(int4) * m->nd);
            e = up.finish();
        }
        if (e != hipSuccess) {
            free_mesh(m);
            sld_set_error(std::string("sld_mesh_create: device setup failed: ") + hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? SLD_E_NOMEM : SLD_E_HIP;
        }
    } catch (const std::bad_alloc&) {
        free_mesh(m);
        sld_set_error("sld_mesh_create: host allocation failed");
        return SLD_E_NOMEM;
    }
    *out = m;
    return SLD_OK;
}

sld_status sld_mesh_counts(sld_mesh m, int64_t* ne, int64_t* nd, int64_t* nv) {
    SLD_REQUIRE(m, SLD_E_INVALID, "sld_mesh_counts: NULL mesh");
    if (ne) *ne = m->ne;
    if (nd) *nd = m->nd;
    if (nv) *nv = m->nv;
    return SLD_OK;
}

sld_status sld_mesh_edges(sld_mesh m, int32_t* left, int32_t* right, int32_t* alpha_left,
                          int32_t* alpha_right) {
    SLD_REQUIRE(m, SLD_E_INVALID, "sld_mesh_edges: NULL mesh");
    const size_t n = size_t(m->nd) * sizeof(int32_t);
    if (left) std::memcpy(left, m->left.data(), n);
    if (right) std::memcpy(right, m->right.data(), n);
    if (alpha_left) std::memcpy(alpha_left, m->alpha_l.data(), n);
    if (alpha_right) std::memcpy(alpha_right, m->alpha_r.data(), n);
    return SLD_OK;
}

void sld_mesh_destroy(sld_mesh m) {
    if (m) release_mesh(m);
}

sld_status sld_disc_create(sld_mesh m, int32_t p, uint32_t flags, sld_disc* out) {
    SLD_REQUIRE(out, SLD_E_INVALID, "sld_disc_create: out is NULL");
    *out = nullptr;
    SLD_REQUIRE(m, SLD_E_INVALID, "sld_disc_create: NULL mesh");
    SLD_REQUIRE(p >= 1 && p <= 4, SLD_E_INVALID, "sld_disc_create: degree p must be in 1..4");
    SLD_REQUIRE(flags == 0, SLD_E_INVALID, "sld_disc_create: flags must be 0");
    sld_disc_s* d = new (std::nothrow) sld_disc_s();
    SLD_REQUIRE(d, SLD_E_NOMEM, "sld_disc_create: host allocation failed");
    d->mesh = m;
    d->p = p;
    d->nphi = (p + 1) * (p + 2) / 2;
    d->npsi = (p + 1) * (p + 1);
    int rc = build_ops(p, &d->ops_host, &d->ops_bytes);
    if (rc != 0) {
        free_disc(d);
        sld_set_error("sld_disc_create: reference operator construction failed");
        return rc == -1 ? SLD_E_NOMEM : SLD_E_INVALID;
    }
    if (m->device < 0) {
        m->refs.fetch_add(1);
        *out = d;  // host-only: reference operators and node queries only
        return SLD_OK;
    }
    DeviceGuard dg(m->device);
    const size_t nv = size_t(m->ne) * d->nphi;
    CgWork& w = d->cg;
    bool front = false;
    int G = cg_grid_for(d, &front);
    w.front = front;
    if (const char* gcap = std::getenv("SLD_CG_GRID")) {  // debugging aid: grid size cap
        const int cap = std::atoi(gcap);
        if (cap > 0 && cap < G) G = (cap + 7) & ~7;
    }
    // the MFMA operator serves meshes without wall edges (SLD_MX=0 in the environment turns it
    // off, a debugging aid).  When the library's default FP64 iteration is the MFMA one (or
    // SLD_MX_GRID=1, a debugging aid for measuring it), its CG kernel sets the grid: as many
    // blocks as stay resident (a multiple of 8), or one tile per block on smaller meshes.  The
    // grid is shared by every CG kernel of the disc (the dot partials are laid out by it).
    w.mx_ok = m->periodic;
    if (const char* mx = std::getenv("SLD_MX"))
        if (std::atoi(mx) == 0) w.mx_ok = false;
    bool mx_grid = kAutoMx64;
    if (const char* mg = std::getenv("SLD_MX_GRID")) mx_grid = std::atoi(mg) != 0;
    if (w.mx_ok) {
        // (resident blocks of the MFMA kernels, both word sizes: zero when the tile's LDS does
        // not fit, and then the disc keeps the vector-unit kernels)
        int cus = 0;
        const int per = mx_blocks_per_cu(d, false);
        if (per <= 0 || mx_blocks_per_cu(d, true) <= 0 ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess ||
            cus <= 0) {
            w.mx_ok = false;
        } else if (mx_grid) {
            const int64_t tiles = (m->ne + kTriPerBlock - 1) / kTriPerBlock;
            int64_t g = std::min<int64_t>(tiles, (int64_t)per * cus);
            g = std::min<int64_t>(g, kCgMaxGrid);
            G = (int)((g + 7) & ~int64_t(7));
        }
    }
    if (const char* gcap = std::getenv("SLD_CG_GRID")) {
        const int cap = std::atoi(gcap);
        if (cap > 0 && cap < G) G = (cap + 7) & ~7;
    }
    w.grid = G;
    w.grid32 = cg_grid32_for(d, G, w.front);
    if (const char* g32 = std::getenv("SLD_CG_GRID32")) {  // debugging aid: FP32 grid
        const int v = std::atoi(g32);
        if (v >= G) w.grid32 = (v + 7) & ~7;
    }
    const int GP = std::max(G, w.grid32);  // partial sums laid out by either grid
    if (const char* sx = std::getenv("SLD_CG_STREAM_X"))  // debugging aid: force x streaming
        w.stream_x = std::atoi(sx) != 0 ? 1 : 0;
    std::lock_guard<std::mutex> lk(device_setup_mutex());
    Uploader up;
    std::vector<unsigned char> h32(ops32_bytes(p));
    round_ops(p, d->ops_host, h32.data());
    std::vector<unsigned char> hsl;
    if (build_sl(p, &hsl) != 0) {
        free_disc(d);
        sld_set_error("sld_disc_create: semi-Lagrangian projection data failed to build");
        return SLD_E_INVALID;
    }
    std::vector<unsigned char> hmx(mx_tab_bytes(p));
    if (build_mx_tables(p, d->ops_host, hmx.data()) != 0) {
        free_disc(d);
        sld_set_error("sld_disc_create: MFMA operand tables failed to build");
        return SLD_E_INVALID;
    }
    hipError_t e = up.err;
    if (e == hipSuccess) e = hipMalloc(&d->ops_dev, d->ops_bytes);
    if (e == hipSuccess) e = hipMalloc(&d->ops32_dev, h32.size());
    if (e == hipSuccess) e = hipMalloc(&d->mx_dev, hmx.size());
    if (e == hipSuccess) e = hipMalloc(&d->sl_dev, hsl.size());
    if (e == hipSuccess) e = dalloc(&w.x, nv);
    if (e == hipSuccess) e = dalloc(&w.e, nv);
    for (int k = 0; k < 2; ++k) {
        if (e == hipSuccess) e = dalloc(&w.r[k], nv);
        if (e == hipSuccess) e = dalloc(&w.q[k], nv);
        if (e == hipSuccess) e = dalloc(&w.d[k], nv);
    }
    if (e == hipSuccess) e = dalloc(&w.b, nv);
    if (e == hipSuccess) e = dalloc(&w.part, size_t(8) * G);
    if (e == hipSuccess) e = dalloc(&w.part_s, size_t(2) * GP);
    if (e == hipSuccess) e = dalloc(&w.scal, CgScalars::NSCAL);
    if (e == hipSuccess) e = dalloc(&w.wall_i, size_t(m->ne));
    for (int k = 0; k < 2; ++k) {
        if (e == hipSuccess) e = dalloc(&w.r32[k], nv);
        if (e == hipSuccess) e = dalloc(&w.q32[k], nv);
        if (e == hipSuccess) e = dalloc(&w.d32[k], nv);
    }
    if (e == hipSuccess) e = dalloc(&w.e32, nv);
    if (e == hipSuccess) e = dalloc(&w.part32, size_t(8) * GP);
    if (e == hipSuccess) e = dalloc(&w.scal_in, CgScalars::NSCAL);
    if (e == hipSuccess) {
        up.copy(d->ops_dev, d->ops_host, d->ops_bytes);
        up.copy(d->ops32_dev, h32.data(), h32.size());
        up.copy(d->sl_dev, hsl.data(), hsl.size());
        up.copy(d->mx_dev, hmx.data(), hmx.size());
        up.zero(w.scal, CgScalars::NSCAL * sizeof(double));
        up.zero(w.wall_i, size_t(m->ne));
        up.zero(w.scal_in, CgScalars::NSCAL * sizeof(double));
        e = up.finish();
    }
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&w.host_scal_in), CgScalars::NSCAL * sizeof(double),
                          hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&w.capture, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&w.host_scal), 3 * CgScalars::NSCAL * sizeof(double),
                          hipHostMallocDefault);
    if (e != hipSuccess) {
        free_disc(d);
        sld_set_error(std::string("sld_disc_create: device allocation failed: ") + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? SLD_E_NOMEM : SLD_E_HIP;
    }
    m->refs.fetch_add(1);
    *out = d;
    return SLD_OK;
}

}  // extern "C"

namespace {

template <int P>
sld_status ref_operator_p(const sld_disc_s* d, int which, int alpha, std::vector<double>* v) {
    const RefOps<P>& R = *reinterpret_cast<const RefOps<P>*>(d->ops_host);
    auto put = [&](const double* a, size_t n) { v->assign(a, a + n); };
    constexpr int N = RefOps<P>::NPHI, NE = P + 1;
    switch (which) {
        case 0: put(&R.S[0][0][0], size_t(3) * N * N); break;
        case 1: put(&R.Sh[alpha][0][0][0], size_t(3) * N * N); break;
        case 2: put(&R.E[alpha][0][0][0], size_t(2) * NE * N); break;
        case 3: put(&R.Pt[alpha][0][0][0], size_t(2) * N * NE); break;
        case 4: put(&R.C[0][0], size_t(NE) * NE); break;
        case 5: put(&R.M1[0][0], size_t(NE) * NE); break;
        case 6: put(&R.w[0], size_t(N)); break;
        case 7:
        case 8: {
            SlOps<P> sl;
            if (build_slops<P>(&sl) != 0) {
                sld_set_error("sld_ref_operator: semi-Lagrangian rule failed to build");
                return SLD_E_INVALID;
            }
            if (which == 7) put(&sl.pts[0][0], size_t(SlOps<P>::NG) * 2);
            else put(&sl.proj[0][0], size_t(N) * SlOps<P>::NG);
        } break;
        case 9: put(&R.Mref[0][0], size_t(N) * N); break;
        case 10: put(&R.Ldm[alpha][0][0], size_t(N) * N); break;
        default:
            sld_set_error("sld_ref_operator: which must be in 0..10");
            return SLD_E_INVALID;
    }
    return SLD_OK;
}

}  // namespace

extern "C" {

sld_status sld_ref_operator(sld_disc d, int32_t which, int32_t alpha, double* host_out,
                            int64_t cap, int64_t* count) {
    SLD_REQUIRE(d && count, SLD_E_INVALID, "sld_ref_operator: NULL argument");
    SLD_REQUIRE(alpha >= 0 && alpha <= 2, SLD_E_INVALID, "sld_ref_operator: alpha must be 0..2");
    std::vector<double> v;
    sld_status st = SLD_E_INVALID;
    switch (d->p) {
        case 1: st = ref_operator_p<1>(d, which, alpha, &v); break;
        case 2: st = ref_operator_p<2>(d, which, alpha, &v); break;
        case 3: st = ref_operator_p<3>(d, which, alpha, &v); break;
        case 4: st = ref_operator_p<4>(d, which, alpha, &v); break;
    }
    if (st != SLD_OK) return st;
    *count = (int64_t)v.size();
    if (!host_out) return SLD_OK;
    SLD_REQUIRE(cap >= (int64_t)v.size(), SLD_E_INVALID, "sld_ref_operator: cap too small");
    std::memcpy(host_out, v.data(), sizeof(double) * v.size());
    return SLD_OK;
}

sld_status sld_disc_info(sld_disc d, int32_t* p, int32_t* nphi, int32_t* npsi) {
    SLD_REQUIRE(d, SLD_E_INVALID, "sld_disc_info: NULL disc");
    if (p) *p = d->p;
    if (nphi) *nphi = d->nphi;
    if (npsi) *npsi = d->npsi;
    return SLD_OK;
}

sld_status sld_main_nodes(sld_disc d, double* xy_out) {
    SLD_REQUIRE(d && xy_out, SLD_E_INVALID, "sld_main_nodes: NULL argument");
    const sld_mesh_s* m = d->mesh;
    const int p = d->p;
    for (int64_t i = 0; i < m->ne; ++i) {
        const double* P = &m->P[6 * i];
        int k = 0;
        for (int b = 0; b <= p; ++b)
            for (int a = 0; a <= p - b; ++a, ++k) {
                double s = double(a) / p, t = double(b) / p;
                for (int c = 0; c < 2; ++c)
                    xy_out[(i * d->nphi + k) * 2 + c] =
                        P[c] + s * (P[2 + c] - P[c]) + t * (P[4 + c] - P[c]);
            }
    }
    return SLD_OK;
}

sld_status sld_dual_nodes(sld_disc d, double* xy_out) {
    SLD_REQUIRE(d && xy_out, SLD_E_INVALID, "sld_dual_nodes: NULL argument");
    const sld_mesh_s* m = d->mesh;
    const int p = d->p;
    for (int64_t j = 0; j < m->nd; ++j) {
        const int l = m->left[j], r = m->right[j], al = m->alpha_l[j];
        const double* Pl = &m->P[6 * l];
        double A[2], B[2], bl[2], br[2];
        for (int c = 0; c < 2; ++c) {
            A[c] = Pl[2 * al + c];
            B[c] = Pl[2 * ((al + 1) % 3) + c];
            bl[c] = (Pl[c] + Pl[2 + c] + Pl[4 + c]) / 3.0;
            br[c] = 0;
            if (r >= 0) {
                const double* Pr = &m->P[6 * r];
                br[c] = (Pr[c] + Pr[2 + c] + Pr[4 + c]) / 3.0 - m->shift[2 * j + c];
            }
        }
        for (int b = 0; b <= p; ++b)
            for (int a = 0; a <= p; ++a) {
                const int k = b * (p + 1) + a;
                const double s = double(a) / p, t = double(b) / p;
                for (int c = 0; c < 2; ++c) {
                    double v;
                    if (a + b <= p) v = bl[c] + s * (A[c] - bl[c]) + t * (B[c] - bl[c]);
                    else if (r >= 0) v = br[c] + (1 - t) * (A[c] - br[c]) + (1 - s) * (B[c] - br[c]);
                    else v = NAN;
                    xy_out[(j * d->npsi + k) * 2 + c] = v;
                }
            }
    }
    return SLD_OK;
}

sld_status sld_main_weights(sld_disc d, double* w_out) {
    SLD_REQUIRE(d && w_out, SLD_E_INVALID, "sld_main_weights: NULL argument");
    const sld_mesh_s* m = d->mesh;
    const double* w = ops_w(d);
    for (int64_t i = 0; i < m->ne; ++i) {
        const double* P = &m->P[6 * i];
        const double A = (P[2] - P[0]) * (P[5] - P[1]) - (P[3] - P[1]) * (P[4] - P[0]);
        for (int k = 0; k < d->nphi; ++k) w_out[i * d->nphi + k] = A * w[k];
    }
    return SLD_OK;
}

void sld_disc_destroy(sld_disc d) {
    if (!d) return;
    sld_mesh_s* m = d->mesh;
    if (m->device < 0) {
        free_disc(d);
    } else {
        DeviceGuard dg(m->device);
        std::lock_guard<std::mutex> lk(device_setup_mutex());
        free_disc(d);
    }
    release_mesh(m);
}

#define SLD_REQUIRE_DEVICE(d, fn) \
    SLD_REQUIRE((d)->mesh->device >= 0, SLD_E_INVALID, fn ": handle was created host-only (device -1)")

sld_status sld_schur_apply(sld_disc d, const double* p, double* Kp, void* stream) {
    SLD_REQUIRE(d && p && Kp, SLD_E_INVALID, "sld_schur_apply: NULL argument");
    SLD_REQUIRE(p != Kp, SLD_E_INVALID, "sld_schur_apply: p and Kp must not alias");
    SLD_REQUIRE_DEVICE(d, "sld_schur_apply");
    DeviceGuard dg(d->mesh->device);
    SLD_HIP_CHECK(launch_schur_apply(d, p, Kp, 1.0, (hipStream_t)stream));
    return SLD_OK;
}

sld_status sld_schur_apply_mx(sld_disc d, const void* p, void* Kp, int32_t engine, void* stream) {
    SLD_REQUIRE(d && p && Kp, SLD_E_INVALID, "sld_schur_apply_mx: NULL argument");
    SLD_REQUIRE(p != Kp, SLD_E_INVALID, "sld_schur_apply_mx: p and Kp must not alias");
    SLD_REQUIRE(engine == SLD_MX_F64 || engine == SLD_MX_BF16X3, SLD_E_INVALID,
                "sld_schur_apply_mx: engine must be SLD_MX_F64 or SLD_MX_BF16X3");
    SLD_REQUIRE_DEVICE(d, "sld_schur_apply_mx");
    SLD_REQUIRE(d->mx_dev && d->mesh->periodic, SLD_E_INVALID,
                "sld_schur_apply_mx: the MFMA operator runs on meshes without wall edges");
    SLD_REQUIRE(d->cg.mx_ok, SLD_E_INVALID,
                "sld_schur_apply_mx: the MFMA operator is off for this disc (its tile does not fit "
                "the device, or SLD_MX=0)");
    DeviceGuard dg(d->mesh->device);
    SLD_HIP_CHECK(launch_apply_mx(d, p, Kp, engine == SLD_MX_BF16X3, (hipStream_t)stream));
    return SLD_OK;
}

sld_status sld_gradient(sld_disc d, const double* p, double* g, void* stream) {
    SLD_REQUIRE(d && p && g, SLD_E_INVALID, "sld_gradient: NULL argument");
    SLD_REQUIRE_DEVICE(d, "sld_gradient");
    DeviceGuard dg(d->mesh->device);
    SLD_HIP_CHECK(launch_gradient(d, p, nullptr, 1.0, g, (hipStream_t)stream));
    return SLD_OK;
}

sld_status sld_divergence(sld_disc d, const double* v, double* out, void* stream) {
    SLD_REQUIRE(d && v && out, SLD_E_INVALID, "sld_divergence: NULL argument");
    SLD_REQUIRE_DEVICE(d, "sld_divergence");
    DeviceGuard dg(d->mesh->device);
    SLD_HIP_CHECK(launch_divergence(d, v, 1.0, out, (hipStream_t)stream));
    return SLD_OK;
}

sld_status sld_pressure_rhs(sld_disc d, const double* v_star, double scale, double* b, void* stream) {
    SLD_REQUIRE(d && v_star && b, SLD_E_INVALID, "sld_pressure_rhs: NULL argument");
    SLD_REQUIRE(std::isfinite(scale), SLD_E_INVALID, "sld_pressure_rhs: scale must be finite");
    SLD_REQUIRE_DEVICE(d, "sld_pressure_rhs");
    DeviceGuard dg(d->mesh->device);
    SLD_HIP_CHECK(launch_divergence(d, v_star, scale, b, (hipStream_t)stream));
    return SLD_OK;
}

sld_status sld_velocity_correct(sld_disc d, const double* v_star, const double* p, double coef,
                                double* v, void* stream) {
    SLD_REQUIRE(d && v_star && p && v, SLD_E_INVALID, "sld_velocity_correct: NULL argument");
    SLD_REQUIRE(std::isfinite(coef), SLD_E_INVALID, "sld_velocity_correct: coef must be finite");
    SLD_REQUIRE_DEVICE(d, "sld_velocity_correct");
    DeviceGuard dg(d->mesh->device);
    SLD_HIP_CHECK(launch_gradient(d, p, v_star, -coef, v, (hipStream_t)stream));
    return SLD_OK;
}

sld_status sld_sl_advect(sld_disc d, const double* vbar, const double* q, int32_t nc, double dt,
                         double* q_out, void* stream) {
    SLD_REQUIRE(d && vbar && q && q_out, SLD_E_INVALID, "sld_sl_advect: NULL argument");
    SLD_REQUIRE(nc >= 1 && nc <= 8, SLD_E_INVALID, "sld_sl_advect: nc must be in 1..8");
    SLD_REQUIRE(std::isfinite(dt), SLD_E_INVALID, "sld_sl_advect: dt must be finite");
    SLD_REQUIRE(q_out != q && q_out != vbar, SLD_E_INVALID,
                "sld_sl_advect: q_out must not alias q or vbar");
    SLD_REQUIRE_DEVICE(d, "sld_sl_advect");
    DeviceGuard dg(d->mesh->device);
    SLD_HIP_CHECK(launch_sl_advect(d, vbar, q, nc, dt, q_out, (hipStream_t)stream));
    return SLD_OK;
}

}  // extern "C"

namespace {

// Capture one block of gb CG iterations (FP64, FP64 mass-shifted, or the FP32 inner solve)
// into a graph.  The FP32 block ends with the peek at its process's recursive rr, so that the
// host reads the stop flag and that rr from one copy of the scalars.
hipError_t capture_block(sld_disc_s* d, bool fp32, bool shift, int gb, hipGraphExec_t* out) {
    CgWork& w = d->cg;
    if (*out) {
        hipError_t e = hipGraphExecDestroy(*out);
        *out = nullptr;
        if (e != hipSuccess) return e;
    }
    hipGraph_t g = nullptr;
    std::lock_guard<std::mutex> lk(device_setup_mutex());
    hipError_t e = hipStreamBeginCapture(w.capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t ce = hipSuccess;
    for (int k = 0; k < gb && ce == hipSuccess; ++k)
        ce = fp32 ? launch_cg_step32(d, k & 1, w.capture)
                  : launch_cg_step(d, k & 1, shift, w.capture);
    if (fp32 && ce == hipSuccess) ce = launch_rel_peek(d, 0, w.capture);
    e = hipStreamEndCapture(w.capture, &g);
    if (ce != hipSuccess) return ce;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

// Relative gap between the refreshed and the recursive FP32 residual beyond which a reliable
// update restarts the FP32 Krylov process instead of keeping its search direction.
#ifndef SLD_REL_GAP_MAX
#define SLD_REL_GAP_MAX 0.3
#endif
// FP32 iterations after which a reliable update is made even if the FP32 residual has not
// dropped by the refresh factor (checked after each captured block of iterations).  The
// residual norm of CG on this system is far from monotone (on the 512x512x2, p = 3 solve it
// first grows twelvefold and stays above its start for about 4000 iterations), and over such a
// stretch the FP32 recursion drifts: without this bound the first update found a 95% gap and
// restarted the process, and the mixed solve took 23483 FP32 iterations instead of 19491 at a
// bound of 512 (FP64 CG: 17767).  Frequent updates also keep the FP32 recursion close to the
// FP64 residual later on.  FP32 iterations and ms per mixed solve, p = 3, by bound:
//   512x512x2: 64: 17760 / 1318, 128: 17660 / 1285, 512: 19073 / 1370
//   256x256x2: 64:  8822 /  238, 128:  8824 /  233, 512:  9681 /  253
//   128x128x2: 64:  4906 /   55, 128:  4890 /   53, 512:  4912 /   52
// and the p = 2 cavity step 140 ms at 64 and 128, 146 ms at 512.  An update costs one FP64
// residual evaluation and a few flat kernels.
#ifndef SLD_REL_MAX_SPAN
#define SLD_REL_MAX_SPAN 128
#endif

// SLD_CG_TRACE=1 in the environment: each FP64 residual replacement and each reliable update of
// the mixed form is printed to stderr
bool cg_trace() {
    static const bool on = [] {
        const char* v = std::getenv("SLD_CG_TRACE");
        return v != nullptr && v[0] == '1';
    }();
    return on;
}

struct IterStats {
    int iters = 0, done = 0, timed = 0;
    double t_step = 0;
};

// Run CG iterations until the device flags DONE in `scal`.  `hs` is pinned host memory of
// 3 NSCAL doubles: the final scalars land in hs[0, NSCAL), and two copy slots follow.
//
// Each graph block of gb launches is followed by a copy of the scalars into its slot, which the
// host reads to decide whether to go on.  While the previous solve of the same kind on this disc
// says at least two more blocks are needed, the host queues the next block before reading the
// current one, so the device does not idle during the read (the fewest blocks of the last three
// solves of that kind: the viscous and temperature solves of a step share the kind).  A block queued after convergence
// only runs launches that exit at entry, and results do not depend on the queueing.
sld_status run_iterations(sld_disc_s* d, bool fp32, bool shift, int gb, bool prof, hipStream_t s,
                          double* scal, double* hs, IterStats* st) {
    typedef CgScalars S;
    CgWork& w = d->cg;
    hipGraphExec_t& graph = fp32 ? w.graph32 : (shift ? w.graph_shift : w.graph);
    int& graph_block = fp32 ? w.graph32_block : (shift ? w.graph_shift_block : w.graph_block);
    // events: profile start / end of each slot's block, then each slot's copy
    if (w.events.size() < 6) {
        for (hipEvent_t e : w.events) (void)hipEventDestroy(e);
        w.events.assign(6, nullptr);
        for (auto& e : w.events) SLD_HIP_CHECK(hipEventCreate(&e));
    }
    bool& gmx = w.graph_mx[fp32 ? 2 : (shift ? 1 : 0)];
    const bool pcg_key = !fp32 && !shift && w.graph_pcg != w.use_pcg;
    if (graph == nullptr || graph_block != gb || gmx != w.use_mx || pcg_key) {
        SLD_HIP_CHECK(capture_block(d, fp32, shift, gb, &graph));
        graph_block = gb;
        gmx = w.use_mx;
        if (!fp32 && !shift) w.graph_pcg = w.use_pcg;
    }
    const int kind = shift ? 1 : 0;
    int expect = 0;  // fewest blocks among the recorded solves (0: none recorded)
    if (!fp32 && w.last_gb[kind] == gb)
        for (int h = 0; h < 3; ++h)
            if (w.last_blocks[kind][h] > 0 && (expect == 0 || w.last_blocks[kind][h] < expect))
                expect = w.last_blocks[kind][h];
    double* slot[2] = {hs + S::NSCAL, hs + 2 * S::NSCAL};
    auto enqueue = [&](int b) -> hipError_t {
        const int k = b & 1;
        hipError_t e = hipSuccess;
        if (prof) e = hipEventRecord(w.events[2 * k], s);
        if (e == hipSuccess) e = hipGraphLaunch(graph, s);
        if (prof && e == hipSuccess) e = hipEventRecord(w.events[2 * k + 1], s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(slot[k], scal, S::NSCAL * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipEventRecord(w.events[4 + k], s);
        return e;
    };
    int launched = 0, queued = 0, read = 0;
    SLD_HIP_CHECK(enqueue(queued++));
    while (true) {
        // run one block ahead while the previous solve needed at least two more blocks
        if (queued == read + 1 && queued + 1 < expect) SLD_HIP_CHECK(enqueue(queued++));
        const int k = read & 1;
        // wait for this block's copy (polled, as a stream synchronisation spins)
        hipError_t q;
        while ((q = hipEventQuery(w.events[4 + k])) == hipErrorNotReady) std::this_thread::yield();
        SLD_HIP_CHECK(q);
        const double* h = slot[k];
        ++read;
        st->done = (int)h[S::DONE];
        const int before = launched;
        // launches that did work: the counter of the slot written last
        launched = (int)std::max(h[S::ITER0], h[S::ITER1]);
        st->iters = st->done ? (int)h[S::ITER] : launched - 1;
        if (prof && launched - before == gb) {
            // profile: HIP events on the solve stream around each captured block of gb
            // launches, for blocks whose launches all iterated (the last block exits early)
            float a = 0;
            SLD_HIP_CHECK(hipEventElapsedTime(&a, w.events[2 * k], w.events[2 * k + 1]));
            st->t_step += a;
            st->timed += gb;
        }
        if (st->done) {
            std::memcpy(hs, h, S::NSCAL * sizeof(double));
            if (!fp32) {
                if (w.last_gb[kind] != gb) {
                    for (int h = 0; h < 3; ++h) w.last_blocks[kind][h] = 0;
                    w.last_gb[kind] = gb;
                }
                w.last_blocks[kind][2] = w.last_blocks[kind][1];
                w.last_blocks[kind][1] = w.last_blocks[kind][0];
                w.last_blocks[kind][0] = read;
            }
            return SLD_OK;
        }
        if (queued == read) SLD_HIP_CHECK(enqueue(queued++));
    }
}

// One graph block of FP32 inner iterations; st->iters = launches that did work so far - 1.
sld_status run_block(sld_disc_s* d, int gb, hipStream_t s, IterStats* st) {
    typedef CgScalars S;
    CgWork& w = d->cg;
    if (w.graph32 == nullptr || w.graph32_block != gb || w.graph_mx[2] != w.use_mx) {
        SLD_HIP_CHECK(capture_block(d, true, false, gb, &w.graph32));
        w.graph32_block = gb;
        w.graph_mx[2] = w.use_mx;
    }
    SLD_HIP_CHECK(hipGraphLaunch(w.graph32, s));
    SLD_HIP_CHECK(hipMemcpyAsync(w.host_scal_in, w.scal_in, S::NSCAL * sizeof(double),
                                 hipMemcpyDeviceToHost, s));
    SLD_HIP_CHECK(hipStreamSynchronize(s));
    const int launched = (int)std::max(w.host_scal_in[S::ITER0], w.host_scal_in[S::ITER1]);
    st->done = (int)w.host_scal_in[S::DONE];
    st->iters = st->done ? (int)w.host_scal_in[S::ITER] : launched - 1;
    return SLD_OK;
}

// The FP64 iterations without graphs: blocks of gb plain launches, each followed by a copy of
// the scalars into slot 1 of the pinned mirror and a stream synchronisation (no graph
// instantiation and no event creation: nothing is allocated).
sld_status run_plain(const sld_disc_s* d, int gb, hipStream_t s, double* scal, double* hs,
                     IterStats* st) {
    typedef CgScalars S;
    double* slot = hs + S::NSCAL;
    while (true) {
        for (int k = 0; k < gb; ++k) SLD_HIP_CHECK(launch_cg_step(d, k & 1, false, s));
        SLD_HIP_CHECK(hipMemcpyAsync(slot, scal, S::NSCAL * sizeof(double), hipMemcpyDeviceToHost, s));
        SLD_HIP_CHECK(hipStreamSynchronize(s));
        st->done = (int)slot[S::DONE];
        const int launched = (int)std::max(slot[S::ITER0], slot[S::ITER1]);
        st->iters = st->done ? (int)slot[S::ITER] : launched - 1;
        if (st->done) {
            std::memcpy(hs, slot, S::NSCAL * sizeof(double));
            return SLD_OK;
        }
    }
}

// CG driver.  sigma = 0: the pressure system K p = b; sigma > 0: the viscous system
// (sigma Mbar - K) p = -b (FP64 only).  ws != nullptr: FP64 pressure solve with the CG
// workspace (vectors, partials, scalars) in ws instead of the disc's, run by plain launches.
sld_status cg_solve_impl(sld_disc d_in, const double* b, double* p, const sld_cg_params* prm,
                         sld_cg_report* rep, void* stream, double sigma, double* ws = nullptr);

size_t static_words(int64_t n) { return (size_t)((n + 31) & ~int64_t(31)); }

// Doubles of the static CG workspace for n DOFs and a grid of G blocks: x, e, b, r, q, d (two
// of each of the last three), partials, scalars; every array starts on a 256-byte boundary.
size_t static_ws_doubles(int64_t n, int G) {
    return 9 * static_words(n) + static_words(10 * (int64_t)G) + static_words(CgScalars::NSCAL);
}

}  // namespace

// CG driver (see the declaration above)
namespace {
sld_status cg_solve_impl(sld_disc d_in, const double* b, double* p, const sld_cg_params* prm,
                         sld_cg_report* rep, void* stream, double sigma, double* ws) {
    SLD_REQUIRE(d_in && b && p && prm, SLD_E_INVALID, "sld_cg_solve: NULL argument");
    SLD_REQUIRE(prm->rtol > 0 && std::isfinite(prm->rtol), SLD_E_INVALID,
                "sld_cg_solve: rtol must be positive");
    SLD_REQUIRE(prm->maxit >= 1, SLD_E_INVALID, "sld_cg_solve: maxit must be >= 1");
    SLD_REQUIRE(prm->graph_block >= 2 && prm->graph_block % 2 == 0 && prm->graph_block <= 4096,
                SLD_E_INVALID, "sld_cg_solve: graph_block must be even and in [2, 4096]");
    SLD_REQUIRE(prm->precision == 0 || prm->precision == 1, SLD_E_INVALID,
                "sld_cg_solve: precision must be 0 (FP64) or 1 (mixed)");
    const bool mixed = prm->precision == 1;
    const bool shift = sigma > 0.0;
    SLD_REQUIRE(!(mixed && shift), SLD_E_INVALID, "viscous solves run in FP64 only");
    if (mixed) {
        SLD_REQUIRE(prm->inner_rtol > 0 && prm->inner_rtol < 1, SLD_E_INVALID,
                    "sld_cg_solve: inner_rtol must be in (0, 1)");
        SLD_REQUIRE(prm->max_outer >= 1, SLD_E_INVALID, "sld_cg_solve: max_outer must be >= 1");
        SLD_REQUIRE(prm->profile == 0, SLD_E_INVALID, "sld_cg_solve: profile is FP64-only");
    }
    SLD_REQUIRE_DEVICE(d_in, "sld_cg_solve");
    DeviceGuard dg(d_in->mesh->device);
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    typedef CgScalars S;
    // the static-workspace solve runs on a shallow copy of the disc whose CG workspace points
    // into ws (the pinned scalar mirror stays the disc's)
    sld_disc_s shadow;
    sld_disc_s* d = d_in;
    if (ws != nullptr) {
        SLD_REQUIRE(!mixed && !shift && prm->profile == 0, SLD_E_INVALID,
                    "sld_cg_solve_static: FP64 pressure solves only, without profile");
        shadow.mesh = d_in->mesh;
        shadow.p = d_in->p;
        shadow.nphi = d_in->nphi;
        shadow.npsi = d_in->npsi;
        shadow.ops_dev = d_in->ops_dev;
        shadow.ops_bytes = d_in->ops_bytes;
        shadow.mx_dev = d_in->mx_dev;
        CgWork& sw = shadow.cg;
        const CgWork& dw = d_in->cg;
        const int64_t n = d_in->mesh->ne * d_in->nphi;
        const size_t nw = static_words(n);
        double* q = ws;
        sw.x = q; q += nw;
        sw.e = q; q += nw;
        sw.b = q; q += nw;
        for (int k = 0; k < 2; ++k) {
            sw.r[k] = q; q += nw;
            sw.q[k] = q; q += nw;
            sw.d[k] = q; q += nw;
        }
        sw.part = q;
        sw.part_s = q + 8 * (int64_t)dw.grid;
        q += static_words(10 * (int64_t)dw.grid);
        sw.scal = q;
        sw.host_scal = dw.host_scal;
        sw.grid = dw.grid;
        sw.grid32 = dw.grid32;
        sw.front = dw.front;
        sw.stream_x = dw.stream_x;
        sw.wall_i = dw.wall_i;
        sw.mx_ok = dw.mx_ok;
        d = &shadow;
    }
    CgWork& w = d->cg;
    SLD_REQUIRE(prm->engine >= 0 && prm->engine <= 2, SLD_E_INVALID,
                "sld_cg_solve: engine must be 0 (library's choice), 1 (vector units) or 2 "
                "(matrix cores)");
    w.use_mx = w.mx_ok && (prm->engine == 2 || (prm->engine == 0 && (mixed ? kAutoMx32 : kAutoMx64)));
    SLD_REQUIRE(prm->pipelined >= 0 && prm->pipelined <= 2, SLD_E_INVALID,
                "sld_cg_solve: pipelined must be 0 (library's choice), 1 (classic CG) or 2 "
                "(pipelined CG)");
    const bool pcg_ok = !mixed && !shift && ws == nullptr && !w.use_mx && pcg_possible(d);
    SLD_REQUIRE(prm->pipelined != 2 || pcg_ok, SLD_E_INVALID,
                "sld_cg_solve: pipelined CG serves FP64 pressure solves with the vector units on "
                "meshes whose CG grid holds one tile per block");
    w.use_pcg = pcg_ok && (prm->pipelined == 2 || (prm->pipelined == 0 && kAutoPcg));
    SLD_HIP_CHECK(launch_cg_setup(d, b, p, prm->warm_start != 0, prm->rtol, prm->maxit, sigma, s));
    if (w.use_pcg) SLD_HIP_CHECK(launch_pcg_init(d, s));
    IterStats st;
    // status: 1 converged, 2 no convergence (maxit, or the FP64 floor), 3 breakdown
    int outer = 0, status = 0;
    bool floor_stop = false;
    double rr = 0, bb = 0;
    if (!mixed) {
        // FP64 CG with residual replacement: the device stops when the recursive residual meets
        // its target, or when it has dropped by kReplaceFactor since the last replacement; then
        // x absorbs the accumulated correction, r = K x - b_int is recomputed in FP64 and the
        // iteration resumes from it with d and q kept (restarted if the gap between the two
        // residuals shows d is no longer conjugate to r).  The solve converges when the
        // recomputed residual meets rtol.  If it misses after the recursive one met its target,
        // the recursive target is lowered fourfold -- unless the gap itself is at least half of
        // rtol: the evaluation of K x - b_int in FP64 is then too coarse to confirm rtol (the
        // rounding floor, about eps | |K| |x| | / |b|), and the solve stops without convergence.
        constexpr int kMaxTighten = 6;
        int tighten = 0;
        int base = 0;  // iterations of the segments before the last restart
        // first iteration of the current segment: every captured block starts at parity 0, so
        // the launch that ran iteration k read the buffers of parity (k - seg0) & 1
        int seg0 = 0;
        while (true) {
            sld_status e = ws ? run_plain(d, prm->graph_block, s, w.scal, w.host_scal, &st)
                              : run_iterations(d, false, shift, prm->graph_block,
                                               prm->profile != 0, s, w.scal, w.host_scal, &st);
            if (e != SLD_OK) return e;
            rr = w.host_scal[S::RR];
            bb = w.host_scal[S::BB];
            status = st.done;
            const int seg_iters = (int)w.host_scal[S::ITER];
            st.iters = base + st.iters;
            if (status != S::kConverged && status != S::kRefresh) break;
            if (w.host_scal[S::ZERO] != 0.0) {
                status = S::kConverged;
                break;
            }
            const int src = (seg_iters + 1 - seg0) & 1;
            const double rr_rec = rr;
            SLD_HIP_CHECK(w.use_pcg ? launch_pcg_replace(d, s) : launch_cg_replace(d, src, sigma, s));
            SLD_HIP_CHECK(hipMemcpyAsync(w.host_scal, w.scal, S::NSCAL * sizeof(double),
                                         hipMemcpyDeviceToHost, s));
            SLD_HIP_CHECK(hipStreamSynchronize(s));
            ++outer;
            const bool restarted = w.host_scal[S::ITER0] == 0.0;
            const int total_iters = base + seg_iters;
            if (restarted) {
                base += seg_iters;
                seg0 = 0;
            } else {
                seg0 = seg_iters + 1;
            }
            const double rr_true = w.host_scal[S::RR];
            rr = rr_true;
            if (cg_trace())
                std::fprintf(stderr,
                             "sld cg: replacement %d (%s) after iteration %d, src %d: recursive "
                             "%.3e recomputed %.3e gap %.3e (relative to b)%s\n",
                             outer, status == S::kConverged ? "rtol" : "refresh", total_iters, src,
                             bb > 0 ? std::sqrt(rr_rec / bb) : 0.0,
                             bb > 0 ? std::sqrt(rr_true / bb) : 0.0,
                             bb > 0 ? std::sqrt(w.host_scal[S::GAP] / bb) : 0.0,
                             restarted ? ", restart" : "");
            if (!std::isfinite(rr_true)) {
                status = S::kBreakdown;
                break;
            }
            if (rr_true <= w.host_scal[S::TOLU]) {
                status = S::kConverged;
                break;
            }
            if (status == S::kConverged) {
                if (w.host_scal[S::GAP] >= 0.25 * w.host_scal[S::TOLU] || ++tighten > kMaxTighten) {
                    status = S::kMaxit;
                    floor_stop = true;
                    break;
                }
            }
            if (st.iters >= prm->maxit) {
                status = S::kMaxit;
                break;
            }
        }
        // the solution is x + e
        SLD_HIP_CHECK(launch_cg_fold(d, s));
    } else {
        // FP32 CG with FP64 reliable updates.  The setup left r64 = K x - b_int (partials in
        // part_s); one Krylov process runs in FP32 and is refreshed in FP64 whenever its
        // residual has dropped by `refresh` since the last refresh, and when it stops on its own
        // criterion (the FP64 residual then decides).  A refresh keeps the search direction
        // while the recursive FP32 residual still tracks the true one (relative gap <= kGapMax);
        // beyond that the kept direction is no longer conjugate to the new residual and the
        // FP32 process restarts from it.
        constexpr double kGapMax = SLD_REL_GAP_MAX;
        constexpr int kMaxSpan = SLD_REL_MAX_SPAN;
        // the host checks the bound after each captured block: blocks no longer than it
        const int gb32 = std::max(2, std::min(prm->graph_block, kMaxSpan) & ~1);
        int last_update = 0;
        const double refresh = prm->inner_rtol;
        int total = 0, base = 0;
        SLD_HIP_CHECK(launch_rel_init(d, prm->rtol, prm->maxit, s));
        double rr_ref = 1.0;   // scaled rr at the last refresh
        double prev64 = -1.0;  // FP64 rr when the FP32 process last stopped on its own
        while (true) {
            IterStats in;
            while (true) {
                sld_status e = run_block(d, gb32, s, &in);
                if (e != SLD_OK) return e;
                if (in.done || base + in.iters >= prm->maxit) break;
                // (the block's graph ended with the peek: RRNOW is current)
                if (w.host_scal_in[S::RRNOW] <= refresh * refresh * rr_ref) break;
                if (base + in.iters - last_update >= kMaxSpan) break;
            }
            total = base + in.iters;
            last_update = total;
            SLD_HIP_CHECK(launch_rel_update(d, s));
            SLD_HIP_CHECK(launch_rel_peek(d, 0, s));
            SLD_HIP_CHECK(hipMemcpyAsync(w.host_scal, w.scal, S::NSCAL * sizeof(double),
                                         hipMemcpyDeviceToHost, s));
            SLD_HIP_CHECK(hipMemcpyAsync(w.host_scal_in, w.scal_in, S::NSCAL * sizeof(double),
                                         hipMemcpyDeviceToHost, s));
            SLD_HIP_CHECK(hipStreamSynchronize(s));
            ++outer;
            rr = w.host_scal[S::RR];
            bb = w.host_scal[S::BB];
            rr_ref = w.host_scal_in[S::RRNOW];
            if (rr <= w.host_scal[S::TOL2]) {
                status = 1;
                break;
            }
            if (!std::isfinite(rr) || !std::isfinite(rr_ref)) {
                status = 3;
                break;
            }
            if (in.done == 2 || total >= prm->maxit || outer >= prm->max_outer) {
                status = 2;
                break;
            }
            bool restart = w.host_scal_in[S::GAP] > kGapMax * kGapMax * rr_ref;
            if (in.done) {
                // the FP32 process met rtol but the FP64 residual did not: go on from the
                // refreshed residual unless the FP64 residual has stopped improving (floor)
                if (prev64 >= 0 && rr > 0.25 * prev64) {
                    status = 2;
                    break;
                }
                prev64 = rr;
                restart = true;
            }
            if (cg_trace())
                std::fprintf(stderr,
                             "sld cg: reliable update %d after %d FP32 iterations: FP64 residual "
                             "%.3e, gap %.3e of the FP32 one%s%s\n",
                             outer, total, bb > 0 ? std::sqrt(rr / bb) : 0.0,
                             rr_ref > 0 ? std::sqrt(w.host_scal_in[S::GAP] / rr_ref) : 0.0,
                             in.done ? ", FP32 process at rtol" : "", restart ? ", restart" : "");
            if (restart) {
                base = total;
                SLD_HIP_CHECK(launch_rel_restart(d, s));
            }
        }
        st.iters = total;
    }
    SLD_HIP_CHECK(launch_cg_finish(d, p, sigma, s));
    SLD_HIP_CHECK(hipMemcpyAsync(w.host_scal, w.scal, S::NSCAL * sizeof(double),
                                 hipMemcpyDeviceToHost, s));
    SLD_HIP_CHECK(hipStreamSynchronize(s));
    const double rt = w.host_scal[S::RTRUE];
    if (rep) {
        rep->iters = st.iters;
        rep->converged = status == 1;
        rep->rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
        rep->rel_res_true = bb > 0 ? std::sqrt(rt / bb) : 0.0;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        rep->step_us = st.timed ? 1e3 * st.t_step / st.timed : 0.0;
        rep->timed_iters = st.timed;
        rep->outer_iters = outer;
    }
    if (status == 3) {
        sld_set_error("sld_cg_solve: breakdown (d.Ad <= 0 or non-finite)");
        return SLD_E_BREAKDOWN;
    }
    if (status == 2) {
        sld_set_error(mixed ? "sld_cg_solve: refinement stopped before rtol (maxit, max_outer or "
                              "the FP64 residual floor)"
                    : floor_stop ? "sld_cg_solve: the recomputed residual stagnated above rtol (the "
                                   "FP64 rounding floor of K x)"
                                 : "sld_cg_solve: maxit reached before rtol");
        return SLD_E_NOCONV;
    }
    return SLD_OK;
}

}  // namespace

extern "C" {

sld_status sld_cg_solve(sld_disc d, const double* b, double* p, const sld_cg_params* prm,
                        sld_cg_report* rep, void* stream) {
    return cg_solve_impl(d, b, p, prm, rep, stream, 0.0);
}

sld_status sld_cg_solve_static(sld_disc d, const double* b, double* p, const sld_cg_params* prm,
                               sld_cg_report* rep, void* stream) {
    SLD_REQUIRE(d && b && p && prm, SLD_E_INVALID, "sld_cg_solve_static: NULL argument");
    SLD_REQUIRE_DEVICE(d, "sld_cg_solve_static");
    DeviceGuard dg(d->mesh->device);
    double* ws = nullptr;
    SLD_HIP_CHECK(cg_static_scratch(d->mesh->device, &ws));
    const int64_t n = d->mesh->ne * d->nphi;
    const size_t need = static_ws_doubles(n, d->cg.grid);
    if (need > kStaticCgDoubles) {
        const int64_t fixed = (int64_t)static_ws_doubles(0, d->cg.grid);
        sld_set_error("sld_cg_solve_static: the CG workspace of this disc (" +
                      std::to_string(need) + " doubles for " + std::to_string(n) +
                      " DOFs) exceeds the static workspace of " +
                      std::to_string(kStaticCgDoubles) + " doubles (64 MiB); at most about " +
                      std::to_string(((int64_t)kStaticCgDoubles - fixed) / 9) +
                      " DOFs fit (ne * N_phi)");
        return SLD_E_BUDGET;
    }
    return cg_solve_impl(d, b, p, prm, rep, stream, 0.0, ws);
}

}  // extern "C"

// ---------------------------------------------------------------- IMEX step (Section 4)

namespace {

void free_state(sld_state_s* st) {
    if (!st) return;
    dfree(st->vbar);
    dfree(st->vfoot);
    dfree(st->vsbar);
    dfree(st->vs);
    dfree(st->b);
    dfree(st->wall_all);
    dfree(st->tfoot);
    dfree(st->gbt);
    dfree(st->tdual);
    delete st;
}

// (Mbar - c K_W) x = Mbar f + c G_b for one [ne][N] field (f read through strides); x [ne][N].
// K_W: the diffusion operator, with Dirichlet cells on the wall edges flagged in `mask` (device
// [nd], NULL none) and zero-flux cells on the other walls; gb: G_b of the data or NULL.
sld_status viscous_field(sld_disc d, const double* f, int64_t f_is, int64_t f_cs, int comp,
                         double c, const unsigned char* mask, const double* gb, double* x,
                         double* bbuf, const sld_cg_params* prm, sld_cg_report* rep,
                         hipStream_t s) {
    const double sigma = 1.0 / c;
    SLD_HIP_CHECK(launch_wall_mask(d, mask, s));
    // b = -sigma Mbar f - G_b (the CG runs -(K_W - sigma Mbar) x = -b); x = f is the initial
    // guess
    SLD_HIP_CHECK(launch_mass_rhs(d, f, f_is, f_cs, comp, -sigma, gb, -1.0, bbuf, x, s));
    sld_cg_params q = *prm;
    q.warm_start = 1;
    return cg_solve_impl(d, bbuf, x, &q, rep, s, sigma);
}

}  // namespace

extern "C" {

sld_status sld_dual_to_main(sld_disc d, const double* v, int32_t nc, double* out, void* stream) {
    SLD_REQUIRE(d && v && out, SLD_E_INVALID, "sld_dual_to_main: NULL argument");
    SLD_REQUIRE(nc >= 1 && nc <= 8, SLD_E_INVALID, "sld_dual_to_main: nc must be in 1..8");
    SLD_REQUIRE(v != out, SLD_E_INVALID, "sld_dual_to_main: out must not alias v");
    SLD_REQUIRE_DEVICE(d, "sld_dual_to_main");
    DeviceGuard dg(d->mesh->device);
    SLD_HIP_CHECK(launch_dual_to_main(d, v, nc, out, int64_t(nc) * d->nphi, d->nphi,
                                      (hipStream_t)stream));
    return SLD_OK;
}

sld_status sld_main_to_dual(sld_disc d, const double* v, int32_t nc, double* out, void* stream) {
    SLD_REQUIRE(d && v && out, SLD_E_INVALID, "sld_main_to_dual: NULL argument");
    SLD_REQUIRE(nc >= 1 && nc <= 8, SLD_E_INVALID, "sld_main_to_dual: nc must be in 1..8");
    SLD_REQUIRE(v != out, SLD_E_INVALID, "sld_main_to_dual: out must not alias v");
    SLD_REQUIRE_DEVICE(d, "sld_main_to_dual");
    DeviceGuard dg(d->mesh->device);
    SLD_HIP_CHECK(launch_main_to_dual(d, v, nc, int64_t(nc) * d->nphi, d->nphi, out,
                                      (hipStream_t)stream));
    return SLD_OK;
}

sld_status sld_viscous_solve(sld_disc d, const double* f, double c,
                             const uint8_t* wall_dirichlet, const double* wall_values, double* x,
                             const sld_cg_params* prm, sld_cg_report* rep, void* stream) {
    SLD_REQUIRE(d && f && x && prm, SLD_E_INVALID, "sld_viscous_solve: NULL argument");
    SLD_REQUIRE(std::isfinite(c) && c >= 0.0, SLD_E_INVALID,
                "sld_viscous_solve: c must be finite and >= 0");
    SLD_REQUIRE(prm->precision == 0, SLD_E_INVALID, "sld_viscous_solve: precision must be 0 (FP64)");
    SLD_REQUIRE_DEVICE(d, "sld_viscous_solve");
    DeviceGuard dg(d->mesh->device);
    hipStream_t s = (hipStream_t)stream;
    if (c == 0.0) {
        if (x != f)
            SLD_HIP_CHECK(hipMemcpyAsync(x, f, sizeof(double) * d->mesh->ne * d->nphi,
                                         hipMemcpyDeviceToDevice, s));
        if (rep) {
            *rep = sld_cg_report{};
            rep->converged = 1;
        }
        return SLD_OK;
    }
    // the caller-order right-hand side lives in the CG's second residual buffer and G_b in its
    // second q buffer: the setup touches neither before it has gathered b
    const double* gb = nullptr;
    if (wall_dirichlet && wall_values) {
        SLD_HIP_CHECK(launch_dirichlet_rhs(d, wall_dirichlet, wall_values, d->cg.q[1], s));
        gb = d->cg.q[1];
    }
    return viscous_field(d, f, d->nphi, 0, 0, c, wall_dirichlet, gb, x, d->cg.r[1], prm, rep, s);
}

sld_status sld_state_create(sld_disc d, sld_state* out) {
    SLD_REQUIRE(out, SLD_E_INVALID, "sld_state_create: out is NULL");
    *out = nullptr;
    SLD_REQUIRE(d, SLD_E_INVALID, "sld_state_create: NULL disc");
    SLD_REQUIRE_DEVICE(d, "sld_state_create");
    sld_state_s* st = new (std::nothrow) sld_state_s();
    SLD_REQUIRE(st, SLD_E_NOMEM, "sld_state_create: host allocation failed");
    st->disc = d;
    const size_t nm = size_t(d->mesh->ne) * d->nphi;
    const size_t ndv = size_t(d->mesh->nd) * 2 * d->npsi;
    DeviceGuard dg(d->mesh->device);
    std::lock_guard<std::mutex> lk(device_setup_mutex());
    hipError_t e = dalloc(&st->vbar, 2 * nm);
    if (e == hipSuccess) e = dalloc(&st->vfoot, 2 * nm);
    if (e == hipSuccess) e = dalloc(&st->vsbar, 2 * nm);
    if (e == hipSuccess) e = dalloc(&st->vs, ndv);
    if (e == hipSuccess) e = dalloc(&st->b, nm);
    const sld_mesh_s* m = d->mesh;
    std::vector<unsigned char> wall_h;
    for (int64_t j = 0; j < m->nd; ++j)
        if (m->right[j] < 0) {
            wall_h.assign(size_t(m->nd), 0);
            break;
        }
    if (!wall_h.empty()) {
        for (int64_t j = 0; j < m->nd; ++j) wall_h[j] = m->right[j] < 0 ? 1 : 0;
        if (e == hipSuccess) e = dalloc(&st->wall_all, size_t(m->nd));
        if (e == hipSuccess) e = dalloc(&st->tfoot, nm);
        if (e == hipSuccess) e = dalloc(&st->gbt, nm);
        if (e == hipSuccess) e = dalloc(&st->tdual, size_t(m->nd) * d->npsi);
        if (e == hipSuccess) {
            Uploader up;
            up.copy(st->wall_all, wall_h.data(), wall_h.size());
            e = up.finish();
        }
    }
    if (e != hipSuccess) {
        free_state(st);
        sld_set_error(std::string("sld_state_create: device allocation failed: ") + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? SLD_E_NOMEM : SLD_E_HIP;
    }
    *out = st;
    return SLD_OK;
}

void sld_state_destroy(sld_state st) {
    if (!st) return;
    DeviceGuard dg(st->disc->mesh->device);
    std::lock_guard<std::mutex> lk(device_setup_mutex());
    free_state(st);
}

sld_status sld_imex_step(sld_state st, const sld_imex_params* prm, double dt, double* v, double* p,
                         sld_imex_report* rep, void* stream) {
    SLD_REQUIRE(st && prm && v && p, SLD_E_INVALID, "sld_imex_step: NULL argument");
    SLD_REQUIRE(v != p, SLD_E_INVALID, "sld_imex_step: v and p must not alias");
    SLD_REQUIRE(std::isfinite(dt) && dt > 0.0, SLD_E_INVALID, "sld_imex_step: dt must be > 0");
    SLD_REQUIRE(std::isfinite(prm->nu) && prm->nu >= 0.0, SLD_E_INVALID,
                "sld_imex_step: nu must be finite and >= 0");
    SLD_REQUIRE(prm->R == 0, SLD_E_INVALID, "sld_imex_step: only R = 0 is built");
    SLD_REQUIRE(prm->viscous.precision == 0, SLD_E_INVALID,
                "sld_imex_step: the viscous solves run in FP64 (precision 0)");
    sld_disc d = st->disc;
    SLD_REQUIRE(d->mesh->periodic, SLD_E_INVALID,
                "sld_imex_step: periodic meshes only (no wall treatment of the velocity)");
    DeviceGuard dg(d->mesh->device);
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    sld_imex_report local{};
    sld_imex_report* r = rep ? rep : &local;
    *r = sld_imex_report{};
    const int64_t ne = d->mesh->ne;
    const int N = d->nphi;
    const double a_ss = 1.0;  // R = 0: implicit tableau a_11 = 1
    auto done = [&](sld_status e) {
        r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return e;
    };
    SLD_HIP_CHECK(launch_dual_to_main(d, v, 2, st->vbar, 2 * N, N, s));
    SLD_HIP_CHECK(launch_sl_advect(d, st->vbar, st->vbar, 2, dt, st->vfoot, s));
    const double c = a_ss * dt * prm->nu;
    if (c > 0.0) {
        for (int comp = 0; comp < 2; ++comp) {
            sld_status e = viscous_field(d, st->vfoot, 2 * N, N, comp, c, nullptr, nullptr,
                                         st->vsbar + comp * ne * N, st->b, &prm->viscous, &r->viscous[comp], s);
            if (e != SLD_OK) return done(e);
        }
        SLD_HIP_CHECK(launch_main_to_dual(d, st->vsbar, 2, N, ne * N, st->vs, s));
    } else {
        SLD_HIP_CHECK(launch_main_to_dual(d, st->vfoot, 2, 2 * N, N, st->vs, s));
    }
    SLD_HIP_CHECK(launch_divergence(d, st->vs, 1.0 / (a_ss * dt), st->b, s));
    sld_status e = cg_solve_impl(d, st->b, p, &prm->pressure, &r->pressure, s, 0.0);
    if (e != SLD_OK) return done(e);
    SLD_HIP_CHECK(launch_gradient(d, p, st->vs, -a_ss * dt, v, s));
    SLD_HIP_CHECK(hipStreamSynchronize(s));
    return done(SLD_OK);
}

}  // extern "C"

extern "C" {

sld_status sld_boussinesq_step(sld_state st, const sld_boussinesq_params* prm, double dt,
                               const uint8_t* temp_dirichlet, const double* temp_values,
                               double* v, double* T, double* p, sld_boussinesq_report* rep,
                               void* stream) {
    SLD_REQUIRE(st && prm && v && T && p, SLD_E_INVALID, "sld_boussinesq_step: NULL argument");
    SLD_REQUIRE(v != p && v != T && T != p, SLD_E_INVALID,
                "sld_boussinesq_step: v, T and p must not alias");
    SLD_REQUIRE(std::isfinite(dt) && dt > 0.0, SLD_E_INVALID, "sld_boussinesq_step: dt must be > 0");
    SLD_REQUIRE(std::isfinite(prm->nu) && prm->nu >= 0.0 && std::isfinite(prm->kappa) &&
                    prm->kappa >= 0.0 && std::isfinite(prm->gbeta),
                SLD_E_INVALID, "sld_boussinesq_step: nu, kappa must be finite and >= 0, gbeta finite");
    SLD_REQUIRE(prm->R == 0, SLD_E_INVALID, "sld_boussinesq_step: only R = 0 is built");
    SLD_REQUIRE(prm->viscous.precision == 0, SLD_E_INVALID,
                "sld_boussinesq_step: the diffusion solves run in FP64 (precision 0)");
    sld_disc d = st->disc;
    SLD_REQUIRE(st->wall_all != nullptr, SLD_E_INVALID,
                "sld_boussinesq_step: the mesh has no walls (a closed cavity is needed)");
    DeviceGuard dg(d->mesh->device);
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    sld_boussinesq_report local{};
    sld_boussinesq_report* r = rep ? rep : &local;
    *r = sld_boussinesq_report{};
    const int64_t ne = d->mesh->ne;
    const int N = d->nphi;
    auto done = [&](sld_status e) {
        r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return e;
    };
    // transport: velocity and temperature at the feet of the velocity on the main grid
    SLD_HIP_CHECK(launch_dual_to_main(d, v, 2, st->vbar, 2 * N, N, s));
    SLD_HIP_CHECK(launch_sl_advect(d, st->vbar, st->vbar, 2, dt, st->vfoot, s));
    SLD_HIP_CHECK(launch_sl_advect(d, st->vbar, T, 1, dt, st->tfoot, s));
    // temperature: implicit diffusion with Dirichlet data on the flagged walls
    const double ct = dt * prm->kappa;
    if (ct > 0.0) {
        const double* gb = nullptr;
        if (temp_dirichlet && temp_values) {
            SLD_HIP_CHECK(launch_dirichlet_rhs(d, temp_dirichlet, temp_values, st->gbt, s));
            gb = st->gbt;
        }
        sld_status e = viscous_field(d, st->tfoot, N, 0, 0, ct, temp_dirichlet, gb, T, st->b,
                                     &prm->viscous, &r->temperature, s);
        if (e != SLD_OK) return done(e);
    } else {
        SLD_HIP_CHECK(hipMemcpyAsync(T, st->tfoot, sizeof(double) * ne * N,
                                     hipMemcpyDeviceToDevice, s));
    }
    // velocity: implicit viscosity with no-slip walls
    const double cv = dt * prm->nu;
    if (cv > 0.0) {
        for (int comp = 0; comp < 2; ++comp) {
            sld_status e = viscous_field(d, st->vfoot, 2 * N, N, comp, cv, st->wall_all, nullptr,
                                         st->vsbar + comp * ne * N, st->b, &prm->viscous,
                                         &r->viscous[comp], s);
            if (e != SLD_OK) return done(e);
        }
        SLD_HIP_CHECK(launch_main_to_dual(d, st->vsbar, 2, N, ne * N, st->vs, s));
    } else {
        SLD_HIP_CHECK(launch_main_to_dual(d, st->vfoot, 2, 2 * N, N, st->vs, s));
    }
    // buoyancy with the new temperature, zero velocity on the wall cells
    SLD_HIP_CHECK(launch_main_to_dual(d, T, 1, N, 0, st->tdual, s));
    SLD_HIP_CHECK(launch_buoyancy(d, st->tdual, dt * prm->gbeta, st->vs, s));
    // pressure projection
    SLD_HIP_CHECK(launch_divergence(d, st->vs, 1.0 / dt, st->b, s));
    sld_status e = cg_solve_impl(d, st->b, p, &prm->pressure, &r->pressure, s, 0.0);
    if (e != SLD_OK) return done(e);
    SLD_HIP_CHECK(launch_gradient(d, p, st->vs, -dt, v, s));
    SLD_HIP_CHECK(hipStreamSynchronize(s));
    return done(SLD_OK);
}

}  // extern "C"
