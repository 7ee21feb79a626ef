// Field handle: geometry tables, link storage copies and the clover term.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "internal.h"
#include "block_tables.h"

namespace dfl {

static thread_local std::string g_last_error = "no error";

int set_error(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

// ---------------------------------------------------------------------------
// Workspace cache.  Scratch buffers are call-scoped (no call relies on what a
// previous call left in them), so a buffer that a handle gives up (outgrown,
// or the handle destroyed) is kept for the next handle on the same device
// instead of being freed: a run over many gauge fields allocates its
// workspace once (re-allocating some 200 GB per field costs about a second).
// A cached buffer is handed out only for requests of at least half its size;
// if an allocation fails, the device's cached buffers are freed and the
// allocation retried.  Calls on handles that share a device must not overlap
// in time on different streams (they share this workspace).
// ---------------------------------------------------------------------------
struct CachedBuf {
    int dev;
    void *p;
    size_t bytes;
};
static std::mutex g_ws_mu;
static std::vector<CachedBuf> g_ws_cache;

int ws_acquire(int dev, size_t bytes, void **p, size_t *got) {
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        int best = -1;
        for (size_t i = 0; i < g_ws_cache.size(); ++i) {
            const CachedBuf &c = g_ws_cache[i];
            if (c.dev == dev && c.bytes >= bytes && c.bytes / 2 <= bytes &&
                (best < 0 || c.bytes < g_ws_cache[best].bytes))
                best = (int)i;
        }
        if (best >= 0) {
            *p = g_ws_cache[best].p;
            *got = g_ws_cache[best].bytes;
            g_ws_cache.erase(g_ws_cache.begin() + best);
            return 0;
        }
    }
    if (!dev_alloc(dev, p, bytes))
        return set_error(QCD_ENOMEM, "scratch allocation of " + std::to_string(bytes) + " bytes failed");
    *got = bytes;
    return 0;
}

// hipMalloc on the current device (dev); when it fails, the device's cached
// workspace is freed and the allocation tried once more
bool dev_alloc(int dev, void **p, size_t bytes) {
    if (hipMalloc(p, bytes) == hipSuccess) return true;
    (void)hipGetLastError();
    std::vector<void *> drop;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        for (size_t i = 0; i < g_ws_cache.size();)
            if (g_ws_cache[i].dev == dev) {
                drop.push_back(g_ws_cache[i].p);
                g_ws_cache.erase(g_ws_cache.begin() + i);
            } else {
                ++i;
            }
    }
    if (drop.empty()) return false;
    if (hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    for (void *q : drop) (void)hipFree(q);
    if (hipMalloc(p, bytes) == hipSuccess) return true;
    (void)hipGetLastError();
    *p = nullptr;
    return false;
}

size_t ws_cached_bytes(int dev) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    size_t n = 0;
    for (const CachedBuf &c : g_ws_cache)
        if (c.dev == dev) n += c.bytes;
    return n;
}

void ws_release(int dev, void *p, size_t bytes) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    g_ws_cache.push_back({dev, p, bytes});
}

static thread_local bool g_nosync = false, g_capturing = false;
void set_nosync(bool on) { g_nosync = on; }
bool nosync() { return g_nosync; }
void set_capturing(bool on) { g_capturing = on; }
bool capturing() { return g_capturing; }

int field_buffer(qcd_field f, int slot, size_t bytes, void **p) {
    if (bytes > f->buf_bytes[slot]) {
        if (g_capturing) return set_error(QCD_EINVAL, "workspace growth during stream capture");
        ++f->graph_gen;
        if (f->buf[slot]) {
            DFL_HIP(hipDeviceSynchronize());   // the old buffer may still be in use by queued work
            ws_release(f->device, f->buf[slot], f->buf_bytes[slot]);
        }
        f->buf[slot] = nullptr;
        f->buf_bytes[slot] = 0;
        size_t got = 0;
        DFL_TRY(ws_acquire(f->device, bytes, &f->buf[slot], &got));
        f->buf_bytes[slot] = got;
    }
    *p = f->buf[slot];
    return 0;
}

// ---------------------------------------------------------------------------
// profiling with events
// ---------------------------------------------------------------------------
struct ProfRec {
    int cls;
    hipEvent_t e0, e1;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof_recs;
static std::vector<hipEvent_t> g_event_pool;
static double g_prof_ms[QCD_PROF_CLASSES];
static long long g_prof_n[QCD_PROF_CLASSES];
static double g_prof_work[QCD_PROF_CLASSES][3];   // flops, bytes, units

static hipEvent_t take_event() {
    hipEvent_t e = nullptr;
    if (!g_event_pool.empty()) {
        e = g_event_pool.back();
        g_event_pool.pop_back();
    } else {
        (void)hipEventCreate(&e);
    }
    return e;
}

ProfScope::ProfScope(int c, hipStream_t st, double flops, double bytes, double units) : cls(c), s(st) {
    if (g_nosync) return;   // captured work is timed as a whole by the caller
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    g_prof_work[c][0] += flops;
    g_prof_work[c][1] += bytes;
    g_prof_work[c][2] += units;
    e0 = take_event();
    e1 = take_event();
    (void)hipEventRecord(e0, s);
}

ProfScope::~ProfScope() {
    if (!e0) return;
    (void)hipEventRecord(e1, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_recs.push_back({cls, e0, e1});
    // keep the record list bounded: fold finished records periodically
    if (g_prof_recs.size() > 4096) {
        for (auto &r : g_prof_recs) {
            float ms = 0;
            (void)hipEventSynchronize(r.e1);
            (void)hipEventElapsedTime(&ms, r.e0, r.e1);
            g_prof_ms[r.cls] += ms;
            g_prof_n[r.cls] += 1;
            g_event_pool.push_back(r.e0);
            g_event_pool.push_back(r.e1);
        }
        g_prof_recs.clear();
    }
}

static void prof_fold() {
    for (auto &r : g_prof_recs) {
        float ms = 0;
        (void)hipEventSynchronize(r.e1);
        (void)hipEventElapsedTime(&ms, r.e0, r.e1);
        g_prof_ms[r.cls] += ms;
        g_prof_n[r.cls] += 1;
        g_event_pool.push_back(r.e0);
        g_event_pool.push_back(r.e1);
    }
    g_prof_recs.clear();
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
static int make_geom(const qcd_lattice *lat, Geom &g) {
    g.V = 1;
    g.Vb = 1;
    g.Nb = 1;
    for (int m = 0; m < 4; ++m) {
        int L = lat->dims[m], b = lat->block[m];
        if (L <= 0 || b <= 0)
            return set_error(QCD_EINVAL, "lattice and block extents must be positive");
        if (b % 2)
            return set_error(QCD_EGEOM, "block extent " + std::to_string(b) + " in direction " +
                                            std::to_string(m) + " is odd");
        if (L % b)
            return set_error(QCD_EGEOM, "block extent " + std::to_string(b) + " does not divide lattice extent " +
                                            std::to_string(L) + " in direction " + std::to_string(m));
        if ((L / b) % 2)
            return set_error(QCD_EGEOM, "odd number of blocks (" + std::to_string(L / b) + ") in direction " +
                                            std::to_string(m) + ": the block checkerboard would not close");
        g.L[m] = L;
        g.b[m] = b;
        g.nb[m] = L / b;
        g.V *= L;
        g.Vb *= b;
        g.Nb *= L / b;
    }
    if (g.V >= (1L << 31) / 12)
        return set_error(QCD_EINVAL, "lattice too large for 32-bit site tables");
    // Kernels address a table through a buffer descriptor with a 32-bit
    // chunk offset and a 32-bit element offset.  The largest sum is reached
    // by two FP64 (or four FP32) right-hand sides of one workgroup: 384 bytes
    // per site (the FP64 clover table needs 288).
    if ((unsigned long long)g.V * MAX_OFFSET_BYTES_PER_SITE >= (1ULL << 32))
        return set_error(QCD_EINVAL, "lattice too large: " + std::to_string(g.V) +
                                         " sites exceed the 32-bit buffer offsets (at most " +
                                         std::to_string(((1ULL << 32) - 1) / MAX_OFFSET_BYTES_PER_SITE) + ")");
    g.Vh = g.V / 2;
    g.Vbh = g.Vb / 2;
    return 0;
}

// Internal index of every lexicographic site.  Because the number of blocks
// in the fastest direction is even, consecutive blocks (2m, 2m+1) of the
// lexicographic block order have opposite colours, so the rank of block B
// among the blocks of its colour is B / 2.
__device__ inline long internal_index(const Geom &g, long i) {
    int c[4];
    long r = i;
    for (int m = 3; m >= 0; --m) {
        c[m] = (int)(r % g.L[m]);
        r /= g.L[m];
    }
    int Bl = 0, l = 0, bsum = 0;
    for (int m = 0; m < 4; ++m) {
        Bl = Bl * g.nb[m] + c[m] / g.b[m];
        l = l * g.b[m] + c[m] % g.b[m];
        bsum += c[m] / g.b[m];
    }
    const int p = (c[0] + c[1] + c[2] + c[3]) & 1;
    const long rank = (long)(bsum & 1) * (g.Nb / 2) + Bl / 2;
    return p * g.Vh + rank * g.Vbh + (l >> 1);
}

__global__ void k_site_tables(Geom g, int *__restrict__ int_of, int *__restrict__ lex_of) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.V) return;
    const long idx = internal_index(g, i);
    int_of[i] = (int)idx;
    lex_of[idx] = (int)i;
}

// nbr[2 mu + d][internal x] = internal neighbour, bit 31 set for a hop across
// the antiperiodic time boundary
__global__ void k_nbr_table(Geom g, int bc_t, const int *__restrict__ int_of, int *__restrict__ nbr) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.V) return;
    int c[4];
    long r = i;
    for (int m = 3; m >= 0; --m) {
        c[m] = (int)(r % g.L[m]);
        r /= g.L[m];
    }
    const int xi = int_of[i];
    for (int mu = 0; mu < 4; ++mu)
        for (int d = 0; d < 2; ++d) {
            int cc[4] = {c[0], c[1], c[2], c[3]};
            const bool wrap = (d == 0 && c[mu] == g.L[mu] - 1) || (d == 1 && c[mu] == 0);
            cc[mu] = (cc[mu] + (d == 0 ? 1 : -1) + g.L[mu]) % g.L[mu];
            const long j = cc[3] + (long)g.L[3] * (cc[2] + (long)g.L[2] * (cc[1] + (long)g.L[1] * cc[0]));
            int e = int_of[j];
            if (mu == 0 && wrap && bc_t == -1) e |= (int)0x80000000u;
            nbr[(2 * mu + d) * g.V + xi] = e;
        }
}

// ---------------------------------------------------------------------------
// link packing: canonical complex128 [V][4][3][3] -> storage copies
// ---------------------------------------------------------------------------
__device__ inline __half to_h(double x) { return __float2half((float)x); }
__device__ inline __hip_bfloat16 to_b(double x) { return __float2bfloat16((float)x); }

// F16R / BF16R link: rows 0 and 1 rounded to the half type, row 2 =
// conj(row0 x row1) of the rounded rows in FP64, stored in FP32
template <class H, class H8, class H4>
__device__ inline void pack_link_r(const double2 w[9], H (*rnd)(double), float4 *dst, long V, long idx) {
    H8 c0;
    H4 c1h;
    double2 a[6];
    for (int k = 0; k < 6; ++k) {
        const H re = rnd(w[k].x), im = rnd(w[k].y);
        a[k] = make_double2(to_f(re), to_f(im));
        if (k < 4) {
            c0.v[2 * k] = re;
            c0.v[2 * k + 1] = im;
        } else {
            c1h.v[2 * (k - 4)] = re;
            c1h.v[2 * (k - 4) + 1] = im;
        }
    }
    auto mul = [](double2 x, double2 y) { return make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x); };
    auto sub_conj = [](double2 x, double2 y) { return make_double2(x.x - y.x, -(x.y - y.y)); };
    const double2 w6 = sub_conj(mul(a[1], a[5]), mul(a[2], a[4]));
    const double2 w7 = sub_conj(mul(a[2], a[3]), mul(a[0], a[5]));
    const double2 w8 = sub_conj(mul(a[0], a[4]), mul(a[1], a[3]));
    float4 f0, f1;
    __builtin_memcpy(&f0, &c0, sizeof(float4));
    __builtin_memcpy(&f1, &c1h, sizeof(H4));
    f1.z = (float)w6.x;
    f1.w = (float)w6.y;
    dst[0 * V + idx] = f0;
    dst[1 * V + idx] = f1;
    dst[2 * V + idx] = make_float4((float)w7.x, (float)w7.y, (float)w8.x, (float)w8.y);
}

__global__ void k_pack_links(const double2 *__restrict__ canon, const int *__restrict__ lex_of, long V,
                             double2 *__restrict__ u64, float4 *__restrict__ u32, h4 *__restrict__ u16,
                             b4 *__restrict__ ubf, float4 *__restrict__ u16r, float4 *__restrict__ ubfr) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= V) return;
    long i = lex_of[idx];
    for (int mu = 0; mu < 4; ++mu) {
        const double2 *src = canon + (i * 4 + mu) * 9;
        double2 w[9];
        for (int k = 0; k < 9; ++k) w[k] = src[k];
        for (int k = 0; k < 9; ++k) u64[((long)mu * 9 + k) * V + idx] = w[k];
        pack_link_r<__half, h8, h4>(w, to_h, u16r + (long)mu * 3 * V, V, idx);
        pack_link_r<__hip_bfloat16, b8, b4>(w, to_b, ubfr + (long)mu * 3 * V, V, idx);
        for (int c = 0; c < 3; ++c) {
            double2 a = w[2 * c], b = w[2 * c + 1];
            u32[((long)mu * 3 + c) * V + idx] = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
            h4 h;
            h.v[0] = __float2half((float)(a.x));
            h.v[1] = __float2half((float)(a.y));
            h.v[2] = __float2half((float)(b.x));
            h.v[3] = __float2half((float)(b.y));
            u16[((long)mu * 3 + c) * V + idx] = h;
            b4 q;
            q.v[0] = __float2bfloat16((float)a.x);
            q.v[1] = __float2bfloat16((float)a.y);
            q.v[2] = __float2bfloat16((float)b.x);
            q.v[3] = __float2bfloat16((float)b.y);
            ubf[((long)mu * 3 + c) * V + idx] = q;
        }
    }
}

// ---------------------------------------------------------------------------
// clover term from the four plaquette leaves (FP64), and odd-site inverse
// ---------------------------------------------------------------------------
struct m3 {
    cx<double> e[9];
};
__device__ inline m3 mm(const m3 &a, const m3 &b) {
    m3 c;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cx<double> s = {0, 0};
            for (int k = 0; k < 3; ++k) s = s + a.e[i * 3 + k] * b.e[k * 3 + j];
            c.e[i * 3 + j] = s;
        }
    return c;
}
__device__ inline m3 dag(const m3 &a) {
    m3 c;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c.e[i * 3 + j] = conj(a.e[j * 3 + i]);
    return c;
}
__device__ inline m3 ld(const double2 *u, long V, int mu, long idx) {
    m3 m;
    for (int k = 0; k < 9; ++k) {
        double2 t = u[((long)mu * 9 + k) * V + idx];
        m.e[k] = {t.x, t.y};
    }
    return m;
}

// store one site's 72 reals into the three clover formats
__device__ inline void store_clover(const double a[72], long n, long at, double2 *c64, float4 *c32, h4 *c16) {
    for (int k = 0; k < 36; ++k) c64[k * n + at] = make_double2(a[2 * k], a[2 * k + 1]);
    for (int k = 0; k < 18; ++k)
        c32[k * n + at] = make_float4((float)a[4 * k], (float)a[4 * k + 1], (float)a[4 * k + 2], (float)a[4 * k + 3]);
    for (int k = 0; k < 18; ++k) {
        h4 h;
        for (int e = 0; e < 4; ++e) h.v[e] = __float2half((float)(a[4 * k + e]));
        c16[k * n + at] = h;
    }
}

// pack a full Hermitian 6x6 (row-major complex) into 36 reals
__device__ inline void pack_herm(const cx<double> *m, double *out) {
    for (int i = 0; i < 6; ++i) out[i] = m[i * 6 + i].re;
    int q = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j) {
            out[6 + 2 * q] = 0.5 * (m[i * 6 + j].re + m[j * 6 + i].re);
            out[7 + 2 * q] = 0.5 * (m[i * 6 + j].im - m[j * 6 + i].im);
            ++q;
        }
}

// in-place inverse of a 6x6 complex matrix (Gauss-Jordan, partial pivoting)
__device__ inline bool inv6(cx<double> *a) {
    cx<double> b[36];
    for (int i = 0; i < 36; ++i) b[i] = {0, 0};
    for (int i = 0; i < 6; ++i) b[i * 6 + i] = {1, 0};
    for (int c = 0; c < 6; ++c) {
        int p = c;
        double best = norm2(a[c * 6 + c]);
        for (int r = c + 1; r < 6; ++r)
            if (norm2(a[r * 6 + c]) > best) {
                best = norm2(a[r * 6 + c]);
                p = r;
            }
        if (!(best > 1e-24)) return false;
        if (p != c)
            for (int k = 0; k < 6; ++k) {
                cx<double> t = a[c * 6 + k];
                a[c * 6 + k] = a[p * 6 + k];
                a[p * 6 + k] = t;
                t = b[c * 6 + k];
                b[c * 6 + k] = b[p * 6 + k];
                b[p * 6 + k] = t;
            }
        cx<double> piv = a[c * 6 + c];
        double n2 = norm2(piv);
        cx<double> d = {piv.re / n2, -piv.im / n2};
        for (int k = 0; k < 6; ++k) {
            a[c * 6 + k] = a[c * 6 + k] * d;
            b[c * 6 + k] = b[c * 6 + k] * d;
        }
        for (int r = 0; r < 6; ++r) {
            if (r == c) continue;
            cx<double> f = a[r * 6 + c];
            for (int k = 0; k < 6; ++k) {
                a[r * 6 + k] = a[r * 6 + k] - f * a[c * 6 + k];
                b[r * 6 + k] = b[r * 6 + k] - f * b[c * 6 + k];
            }
        }
    }
    for (int i = 0; i < 36; ++i) a[i] = b[i];
    return true;
}

__global__ void k_clover(const double2 *__restrict__ u, const int *__restrict__ nbr, long V, long Vh,
                         double kappa, double csw, double2 *c64, float4 *c32, h4 *c16, double2 *i64,
                         float4 *i32, h4 *i16, int *flag) {
    long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= V) return;
    auto nb = [&](long s, int d) { return (long)(nbr[(long)d * V + s] & 0x7fffffff); };
    // Fhat for pairs (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
    const int PM[6] = {0, 0, 0, 1, 1, 2}, PN[6] = {1, 2, 3, 2, 3, 3};
    m3 F[6];
    for (int p = 0; p < 6; ++p) {
        int mu = PM[p], nu = PN[p];
        long xpm = nb(x, 2 * mu), xm = nb(x, 2 * mu + 1);
        long xpn = nb(x, 2 * nu), xn = nb(x, 2 * nu + 1);
        long xmn = nb(xm, 2 * nu + 1), xpm_mn = nb(xpm, 2 * nu + 1), xm_pn = nb(xm, 2 * nu);
        m3 Q;
        // leaves circulate mu -> nu (counter-clockwise in the mu-nu plane)
        m3 l1 = mm(mm(ld(u, V, mu, x), ld(u, V, nu, xpm)), mm(dag(ld(u, V, mu, xpn)), dag(ld(u, V, nu, x))));
        m3 l2 = mm(mm(ld(u, V, nu, x), dag(ld(u, V, mu, xm_pn))), mm(dag(ld(u, V, nu, xm)), ld(u, V, mu, xm)));
        m3 l3 = mm(mm(dag(ld(u, V, mu, xm)), dag(ld(u, V, nu, xmn))), mm(ld(u, V, mu, xmn), ld(u, V, nu, xn)));
        m3 l4 = mm(mm(dag(ld(u, V, nu, xn)), ld(u, V, mu, xn)), mm(ld(u, V, nu, xpm_mn), dag(ld(u, V, mu, x))));
        for (int k = 0; k < 9; ++k) Q.e[k] = l1.e[k] + l2.e[k] + l3.e[k] + l4.e[k];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) F[p].e[a * 3 + b] = 0.125 * (Q.e[a * 3 + b] - conj(Q.e[b * 3 + a]));
    }
    // chiral basis: sigma_{0k} = diag(s_k, -s_k), sigma_{jk} = -eps_{jkl} diag(s_l, s_l), so
    // half +: sum_k s_k (x) (B_k + E_k), half -: sum_k s_k (x) (B_k - E_k) with
    // E_k = Fhat_{0k}, B_1 = -Fhat_{23}, B_2 = Fhat_{13}, B_3 = -Fhat_{12}.
    double packed[72];
    cx<double> full[2][36];
    for (int h = 0; h < 2; ++h) {
        double sgn = h == 0 ? 1.0 : -1.0;
        m3 X[3];
        for (int k = 0; k < 9; ++k) {
            cx<double> B1 = -F[5].e[k], B2 = F[4].e[k], B3 = -F[3].e[k];
            cx<double> Y[3] = {B1 + sgn * F[0].e[k], B2 + sgn * F[1].e[k], B3 + sgn * F[2].e[k]};
            for (int q = 0; q < 3; ++q) X[q].e[k] = imul(kappa * csw * Y[q]);   // i kappa csw (B +- E)
        }
        cx<double> *m = full[h];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                cx<double> id = {a == b ? 1.0 : 0.0, 0.0};
                m[a * 6 + b] = id + X[2].e[a * 3 + b];                         // (0,0): X3
                m[a * 6 + 3 + b] = X[0].e[a * 3 + b] - imul(X[1].e[a * 3 + b]);    // (0,1): X1 - i X2
                m[(3 + a) * 6 + b] = X[0].e[a * 3 + b] + imul(X[1].e[a * 3 + b]);  // (1,0): X1 + i X2
                m[(3 + a) * 6 + 3 + b] = id - X[2].e[a * 3 + b];               // (1,1): -X3
            }
        pack_herm(m, packed + 36 * h);
    }
    store_clover(packed, V, x, c64, c32, c16);
    if (x >= Vh) {
        double pinv[72];
        for (int h = 0; h < 2; ++h) {
            if (!inv6(full[h])) atomicOr(flag, 1);
            pack_herm(full[h], pinv + 36 * h);
        }
        store_clover(pinv, Vh, x - Vh, i64, i32, i16);
    }
}

}  // namespace dfl

using namespace dfl;

extern "C" {

const char *qcd_last_error(void) { return g_last_error.c_str(); }

const char *qcd_strerror(int code) {
    switch (code) {
        case QCD_OK: return "ok";
        case QCD_NOCONV: return "solver did not converge";
        case QCD_EINVAL: return "invalid argument";
        case QCD_EGEOM: return "invalid lattice or block geometry";
        case QCD_ENOMEM: return "out of device memory";
        case QCD_EHIP: return "HIP runtime error";
        case QCD_ESINGULAR: return "singular matrix or rank-deficient fields";
        case QCD_ENAN: return "NaN or Inf encountered";
        case QCD_ENOTSET: return "required state not set up";
        default: return "unknown error";
    }
}

int qcd_field_tune(qcd_field f, int knob, int value) {
    if (!f) return set_error(QCD_EINVAL, "null field");
    switch (knob) {
        case QCD_TUNE_STENCIL_BLOCK: f->st_block = value ? 1 : 0; break;
        case QCD_TUNE_STENCIL_RG:
            if (value != 0 && value != 1 && value != 2 && value != 4)
                return set_error(QCD_EINVAL, "right-hand sides per site tile must be 0, 1, 2 or 4");
            f->st_rg = value;
            break;
        case QCD_TUNE_STENCIL_ORDER: f->st_order = value ? 1 : 0; break;
        case QCD_TUNE_STENCIL_LINKLDS: f->st_linklds = value ? 1 : 0; break;
        case QCD_TUNE_SAP_PAIR: f->st_sap_pair = value ? 1 : 0; break;
        case QCD_TUNE_STENCIL_NR:
            if (value != 0 && value != 1 && value != 2 && value != 4)
                return set_error(QCD_EINVAL, "right-hand sides per block workgroup must be 0, 1, 2 or 4");
            f->st_nr = value;
            break;
        default: return set_error(QCD_EINVAL, "unknown tuning knob");
    }
    ++f->graph_gen;   // captured graphs hold the previous launch choices
    return 0;
}

int qcd_workspace_cached(int device, size_t *bytes) {
    if (!bytes) return set_error(QCD_EINVAL, "null byte count");
    *bytes = ws_cached_bytes(device);
    return 0;
}

int qcd_field_trim(qcd_field f) {
    if (!f) return set_error(QCD_EINVAL, "null field");
    if (capturing()) return set_error(QCD_EINVAL, "workspace release during stream capture");
    DFL_HIP(hipDeviceSynchronize());
    graph_cache_free(f);
    ++f->graph_gen;
    for (int k = 0; k < (int)(sizeof(f->buf) / sizeof(f->buf[0])); ++k) {
        ws_release(f->device, f->buf[k], f->buf_bytes[k]);
        f->buf[k] = nullptr;
        f->buf_bytes[k] = 0;
    }
    return 0;
}

int qcd_workspace_trim(int device) {
    std::vector<CachedBuf> drop;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        for (size_t i = 0; i < g_ws_cache.size();)
            if (device < 0 || g_ws_cache[i].dev == device) {
                drop.push_back(g_ws_cache[i]);
                g_ws_cache.erase(g_ws_cache.begin() + i);
            } else {
                ++i;
            }
    }
    if (drop.empty()) return 0;
    int cur = 0;
    DFL_HIP(hipGetDevice(&cur));
    for (const CachedBuf &c : drop) {
        DFL_HIP(hipSetDevice(c.dev));
        DFL_HIP(hipDeviceSynchronize());
        DFL_HIP(hipFree(c.p));
    }
    DFL_HIP(hipSetDevice(cur));
    return 0;
}

int qcd_prof_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    // create the events up front (two per launch, up to the fold bound), so
    // that event creation does not land inside the measured launches
    if (g_prof_on)
        while (g_event_pool.size() < 2 * 4096 + 64) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGetLastError();
                break;
            }
            g_event_pool.push_back(e);
        }
    return 0;
}

int qcd_prof_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_fold();
    for (int c = 0; c < QCD_PROF_CLASSES; ++c) {
        g_prof_ms[c] = 0;
        g_prof_n[c] = 0;
        g_prof_work[c][0] = g_prof_work[c][1] = g_prof_work[c][2] = 0;
    }
    return 0;
}

int qcd_prof_get_work(int cls, double *flops, double *bytes, double *units) {
    if (cls < 0 || cls >= QCD_PROF_CLASSES || !flops || !bytes || !units)
        return set_error(QCD_EINVAL, "bad profiling class");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    *flops = g_prof_work[cls][0];
    *bytes = g_prof_work[cls][1];
    *units = g_prof_work[cls][2];
    return 0;
}

int qcd_prof_get(int cls, double *ms, long long *n) {
    if (cls < 0 || cls >= QCD_PROF_CLASSES || !ms || !n) return set_error(QCD_EINVAL, "bad profiling class");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_fold();
    *ms = g_prof_ms[cls];
    *n = g_prof_n[cls];
    return 0;
}

// Build a field handle from complex128 links already in device memory.
// Parameters and geometry, checked before any device call.
static int check_lattice(const qcd_lattice *lat, Geom &g) {
    if (lat->bc_t != 1 && lat->bc_t != -1) return set_error(QCD_EINVAL, "bc_t must be +1 or -1");
    if (!(lat->kappa > 0) || !std::isfinite(lat->kappa) || !std::isfinite(lat->csw))
        return set_error(QCD_EINVAL, "kappa must be positive and finite, csw finite");
    return make_geom(lat, g);
}

static int field_create_common(const qcd_lattice *lat, const double2 *canon, hipStream_t s, qcd_field *out) {
    Geom g;
    DFL_TRY(check_lattice(lat, g));
    qcd_field f = new qcd_field_s();
    f->lat = *lat;
    f->g = g;
    DFL_HIP(hipGetDevice(&f->device));
    {
        const int rc = static_scratch_init(f->device);
        if (rc < 0) {
            delete f;
            return rc;
        }
    }
    {
        int lds = 0;
        DFL_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, f->device));
        f->lds_max = lds > 0 ? (size_t)lds : 64 * 1024;
    }
    const long V = g.V, Vh = g.Vh;
    auto fail = [&](int rc) {
        qcd_field_destroy(f);
        return rc;
    };
#define ALLOC(ptr, bytes)                                                                        \
    if (!dev_alloc(f->device, (void **)&(ptr), (bytes))) {                                      \
        return fail(set_error(QCD_ENOMEM, "device allocation failed in qcd_field_create"));     \
    }
    ALLOC(f->nbr, sizeof(int) * 8 * V);
    ALLOC(f->lnbr, sizeof(short) * 16 * g.Vbh);
    ALLOC(f->int_of, sizeof(int) * V);
    ALLOC(f->lex_of, sizeof(int) * V);
    ALLOC(f->border, sizeof(int) * g.Nb);
    ALLOC(f->flag, sizeof(int));
    ALLOC(f->U[LNK_F64], sizeof(double2) * 36 * V);
    ALLOC(f->U[LNK_F32], sizeof(float4) * 12 * V);
    ALLOC(f->U[LNK_F16], sizeof(h4) * 12 * V);
    ALLOC(f->U[LNK_BF16], sizeof(b4) * 12 * V);
    ALLOC(f->U[LNK_F16R], sizeof(float4) * 12 * V);
    ALLOC(f->U[LNK_BF16R], sizeof(float4) * 12 * V);
    ALLOC(f->clo[CLO_F64], sizeof(double2) * 36 * V);
    ALLOC(f->clo[CLO_F32], sizeof(float4) * 18 * V);
    ALLOC(f->clo[CLO_F16], sizeof(h4) * 18 * V);
    ALLOC(f->cloinv[CLO_F64], sizeof(double2) * 36 * Vh);
    ALLOC(f->cloinv[CLO_F32], sizeof(float4) * 18 * Vh);
    ALLOC(f->cloinv[CLO_F16], sizeof(h4) * 18 * Vh);
#undef ALLOC
    if (hipHostMalloc((void **)&f->hp, sizeof(double) * 4096) != hipSuccess) {
        (void)hipGetLastError();
        return fail(set_error(QCD_ENOMEM, "pinned host allocation failed"));
    }
    // in-block neighbours, face lists and their sources, block order and the
    // face-exchange neighbours (block_tables.h)
    BlockTables bt;
    build_block_tables(g.b, g.nb, lat->bc_t, bt);
    if (g.Vbh > 32767) return fail(set_error(QCD_EINVAL, "Schwarz block too large"));
    f->face_cap = bt.face_cap;
    for (int mu = 0; mu < 4; ++mu) f->nface[mu] = bt.nface[mu];
    f->nface_tot = bt.nface_tot;
    if (!dev_alloc(f->device, (void **)&f->bface, sizeof(int) * bt.fl.size()) ||
        !dev_alloc(f->device, (void **)&f->bfsrc, sizeof(int) * bt.fsrc.size()) ||
        !dev_alloc(f->device, (void **)&f->bfnb, sizeof(int) * bt.fnb.size()))
        return fail(set_error(QCD_ENOMEM, "device allocation failed in qcd_field_create"));
    // stencil launch defaults, overridable from the environment
    if (const char *e = getenv("DFL_STENCIL_BLOCK")) f->st_block = atoi(e);
    if (const char *e = getenv("DFL_STENCIL_RG")) f->st_rg = atoi(e);
    if (const char *e = getenv("DFL_STENCIL_ORDER")) f->st_order = atoi(e);
    if (const char *e = getenv("DFL_STENCIL_LINKLDS")) f->st_linklds = atoi(e) ? 1 : 0;
    if (const char *e = getenv("DFL_SAP_PAIR")) f->st_sap_pair = atoi(e) ? 1 : 0;
    if (const char *e = getenv("DFL_STENCIL_NR")) {
        const int v = atoi(e);
        f->st_nr = v == 1 || v == 2 || v == 4 ? v : 0;
    }
    hipError_t e = hipMemcpyAsync(f->lnbr, bt.lnb.data(), sizeof(short) * bt.lnb.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(f->bface, bt.fl.data(), sizeof(int) * bt.fl.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(f->bfsrc, bt.fsrc.data(), sizeof(int) * bt.fsrc.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(f->bfnb, bt.fnb.data(), sizeof(int) * bt.fnb.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(f->border, bt.bord.data(), sizeof(int) * bt.bord.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(f->flag, 0, sizeof(int), s);
    if (e != hipSuccess) return fail(set_error(QCD_EHIP, std::string("field setup: ") + hipGetErrorString(e)));
    {
        ProfScope ps(PROF_OTHER, s);
        k_site_tables<<<nblocks(V, 256), 256, 0, s>>>(g, f->int_of, f->lex_of);
        k_nbr_table<<<nblocks(V, 256), 256, 0, s>>>(g, lat->bc_t, f->int_of, f->nbr);
        k_pack_links<<<nblocks(V, 256), 256, 0, s>>>(canon, f->lex_of, V, (double2 *)f->U[LNK_F64],
                                                    (float4 *)f->U[LNK_F32], (h4 *)f->U[LNK_F16],
                                                    (b4 *)f->U[LNK_BF16], (float4 *)f->U[LNK_F16R],
                                                    (float4 *)f->U[LNK_BF16R]);
        k_clover<<<nblocks(V, 128), 128, 0, s>>>((const double2 *)f->U[LNK_F64], f->nbr, V, Vh, lat->kappa,
                                                 lat->csw, (double2 *)f->clo[CLO_F64], (float4 *)f->clo[CLO_F32],
                                                 (h4 *)f->clo[CLO_F16], (double2 *)f->cloinv[CLO_F64],
                                                 (float4 *)f->cloinv[CLO_F32], (h4 *)f->cloinv[CLO_F16], f->flag);
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(f->hp, f->flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(set_error(QCD_EHIP, std::string("field setup: ") + hipGetErrorString(e)));
    if (*reinterpret_cast<int *>(f->hp)) return fail(set_error(QCD_ESINGULAR, "clover block singular on an odd site"));
    *out = f;
    return 0;
}

int qcd_field_create(const qcd_lattice *lat, const double *links_host, hipStream_t s, qcd_field *out) {
    if (!lat || !links_host || !out) return set_error(QCD_EINVAL, "null argument to qcd_field_create");
    *out = nullptr;
    Geom g;
    DFL_TRY(check_lattice(lat, g));
    const long V = g.V;
    double2 *canon = nullptr;
    int dev = 0;
    DFL_HIP(hipGetDevice(&dev));
    if (!dev_alloc(dev, (void **)&canon, sizeof(double2) * 36 * V))
        return set_error(QCD_ENOMEM, "device allocation failed in qcd_field_create");
    int rc = 0;
    hipError_t e = hipMemcpyAsync(canon, links_host, sizeof(double2) * 36 * V, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) rc = set_error(QCD_EHIP, std::string("upload: ") + hipGetErrorString(e));
    if (rc == 0) rc = field_create_common(lat, canon, s, out);
    (void)hipStreamSynchronize(s);
    (void)hipFree(canon);
    return rc;
}

int qcd_field_create_device(const qcd_lattice *lat, const double *links_dev, hipStream_t s, qcd_field *out) {
    if (!lat || !links_dev || !out) return set_error(QCD_EINVAL, "null argument to qcd_field_create_device");
    *out = nullptr;
    Geom g;
    DFL_TRY(check_lattice(lat, g));
    return field_create_common(lat, reinterpret_cast<const double2 *>(links_dev), s, out);
}

int qcd_field_destroy(qcd_field f) {
    if (!f) return 0;
    (void)hipFree(f->nbr);
    (void)hipFree(f->lnbr);
    (void)hipFree(f->bface);
    (void)hipFree(f->bfsrc);
    (void)hipFree(f->bfnb);
    (void)hipFree(f->border);
    (void)hipFree(f->int_of);
    (void)hipFree(f->lex_of);
    (void)hipFree(f->flag);
    for (auto p : f->U) (void)hipFree(p);
    for (auto p : f->clo) (void)hipFree(p);
    for (auto p : f->cloinv) (void)hipFree(p);
    (void)hipFree(f->Uape);
    // scratch goes back to the workspace cache once queued work is done
    (void)hipDeviceSynchronize();
    graph_cache_free(f);
    if (f->cap) (void)hipStreamDestroy(f->cap);
    for (int k = 0; k < (int)(sizeof(f->buf) / sizeof(f->buf[0])); ++k) ws_release(f->device, f->buf[k], f->buf_bytes[k]);
    if (f->hp) (void)hipHostFree(f->hp);
    delete f;
    return 0;
}

}  // extern "C"
