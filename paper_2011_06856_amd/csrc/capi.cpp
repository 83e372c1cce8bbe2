// capi.cpp -- the C ABI declared in include/rlbm.h.
#include <cmath>
#include <cstring>
#include <new>

#include "rlbm_internal.h"


namespace {

int fail(rlbm_ctx c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

int hip_fail(rlbm_ctx c, hipError_t e, const char* where)
{
    return fail(c, RLBM_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

size_t elem_size(int prec) { return store_size(prec); }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t f0, f1, fields, partials, flag, edges, pp0, pp1, cf0, cf1, total;
};

// Workspace: two population buffers, the field outputs, the per-block
// partial charges, the non-physical flag, the initial populations of the
// edge cells (FIXED boundaries) and the push kernel's two partial-sum
// buffers (present whichever kernel is chosen, so that neither rlbm_step nor
// rlbm_set_kernel allocates), and for deviation storage the two buffers of
// equilibrium coefficients paired with the population buffers.
Layout layout(int nvel, int nx, int ny, int prec, int cplanes)
{
    const long long S = (long long)nx * ny;
    Layout L;
    // nvel planes plus one spare plane written by the null table entries
    const size_t fb = align256((size_t)(nvel + 1) * S * elem_size(prec));
    const size_t pb = align256(push_partial_bytes(prec, nx, ny));
    L.f0 = 0;
    L.f1 = L.f0 + fb;
    L.fields = L.f1 + fb;
    L.partials = L.fields + align256((size_t)4 * S * sizeof(double));
    L.flag = L.partials + align256((size_t)fields_blocks(S) * 4 * sizeof(double));
    L.edges = L.flag + 256;
    L.pp0 = L.edges + align256((size_t)2 * (nx + ny) * nvel * elem_size(prec));
    L.pp1 = L.pp0 + pb;
    const size_t cb = is_dev(prec) ? align256((size_t)cplanes * S * arith_size(prec)) : 0;
    L.cf0 = L.pp1 + pb;
    L.cf1 = L.cf0 + cb;
    L.total = L.cf1 + cb;
    return L;
}

void free_tables(rlbm_ctx c)
{
    if (c->d_srec) (void)hipFree(c->d_srec);
    if (c->d_crec) (void)hipFree(c->d_crec);
    if (c->d_sgn) (void)hipFree(c->d_sgn);
    if (c->d_veld) (void)hipFree(c->d_veld);
    if (c->d_G) (void)hipFree(c->d_G);
    if (c->d_Pc) (void)hipFree(c->d_Pc);
    if (c->d_corr) (void)hipFree(c->d_corr);
    if (c->d_zeta) (void)hipFree(c->d_zeta);
    if (c->d_dz) (void)hipFree(c->d_dz);
    c->d_zeta = nullptr;
    c->d_dz = nullptr;
    c->d_srec = nullptr; c->d_crec = nullptr; c->d_sgn = nullptr; c->d_veld = nullptr; c->d_corr = nullptr; c->d_G = nullptr; c->d_Pc = nullptr;
}

template <typename T, int NM>
int upload_tables_t(rlbm_ctx c, const std::vector<VelRec<double>>& vd, long long S, int precision)
{
    const size_t nv = c->q.nvel, npad = nv + RLBM_VPAD;
    std::vector<SRec<T>> sr(npad);
    std::vector<CRec<T, NM>> cr(npad);
    std::vector<unsigned char> sg(npad, 0);
    for (size_t v = 0; v < npad; ++v) {
        const bool real = v < nv;
        SRec<T>& A = sr[v];
        CRec<T, NM>& B = cr[v];
        std::memset(&A, 0, sizeof(A));
        std::memset(&B, 0, sizeof(B));
        B.shell = real ? (int)(v / c->q.K) : c->q.Np - 1;
        if (!real) continue;
        const VelRec<double>& R = vd[v];
        A.w[0] = (T)R.w00; A.w[1] = (T)R.w10; A.w[2] = (T)R.w01; A.w[3] = (T)R.w11;
        for (int j = 0; j < (int)(sizeof(A.P) / sizeof(T)); ++j) A.P[j] = (T)R.P[j];
        for (int t = 0; t < 2 * NM + 1; ++t) B.H[t] = (T)R.H[t];
        B.cth = (T)R.cth; B.sth = (T)R.sth;
        // bit 2: the reversed velocity (theta + pi, same shell) is K/2
        // planes below; null entries read the last plane (angle K - 1), so
        // they carry it too (set below)
        sg[v] = (unsigned char)((R.sx > 0 ? 0 : 1) | (R.sy > 0 ? 0 : 2) | (v % c->q.K >= (size_t)c->q.K / 2 ? 4 : 0));
    }
    for (size_t v = nv; v < npad; ++v) sg[v] = 4;
    hipError_t e;
    if ((e = hipMalloc(&c->d_srec, npad * sizeof(SRec<T>))) != hipSuccess) return fail(c, RLBM_ENOMEM, "table alloc");
    if ((e = hipMalloc(&c->d_crec, npad * sizeof(CRec<T, NM>))) != hipSuccess) return fail(c, RLBM_ENOMEM, "table alloc");
    if ((e = hipMemcpy(c->d_srec, sr.data(), npad * sizeof(SRec<T>), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "table upload");
    if ((e = hipMemcpy(c->d_crec, cr.data(), npad * sizeof(CRec<T, NM>), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "table upload");
    if ((e = hipMalloc((void**)&c->d_sgn, npad)) != hipSuccess) return fail(c, RLBM_ENOMEM, "table alloc");
    if ((e = hipMemcpy(c->d_sgn, sg.data(), npad, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "table upload");
    return RLBM_OK;
}

template <typename T>
int upload_tables_p(rlbm_ctx c, const std::vector<VelRec<double>>& vd, long long S, int precision)
{
    switch (nmax_of(c->q.N)) {
        case 3: return upload_tables_t<T, 3>(c, vd, S, precision);
        case 5: return upload_tables_t<T, 5>(c, vd, S, precision);
        default: return upload_tables_t<T, 7>(c, vd, S, precision);
    }
}

int upload_kernel_tables(rlbm_ctx c, const std::vector<VelRec<double>>& vd, long long S, int precision)
{
    if (arith_size(precision) == 8) return upload_tables_p<double>(c, vd, S, precision);
    return upload_tables_p<float>(c, vd, S, precision);
}

bool finite_arr(const double* a, long long S)
{
    for (long long i = 0; i < S; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

}  // namespace

// Automatic choice: the push kernel where a tile's streamed values would not
// fit the register budget of the tile kernel (large velocity sets), unless a
// WALL or FIXED axis needs the tile kernel's boundary loads.
int resolve_kernel(rlbm_ctx c)
{
    if (is_dev(c->prec)) return RLBM_KERNEL_PUSH;   // deviation storage runs on the push kernel only
    if (c->kern != RLBM_KERNEL_AUTO) return c->kern;
    if (general_step(c->bcx, c->bcy, c->fstat)) return RLBM_KERNEL_TILE;
    return c->q.nvel >= RLBM_PUSH_MIN_NVEL ? RLBM_KERNEL_PUSH : RLBM_KERNEL_TILE;
}

SCParams make_params(rlbm_ctx c, int waves)
{
    SCParams p;
    p.fin = p.fout = nullptr;
    p.srec = c->d_srec;
    p.crec = c->d_crec;
    p.sgn = c->d_sgn;
    p.edges = c->d_edges;
    p.G = c->d_G;
    p.Pc = c->d_Pc;
    p.nx = c->nx; p.ny = c->ny; p.nvel = c->q.nvel; p.K = c->q.K; p.Np = c->q.Np; p.N = c->q.N;
    p.bcx = c->bcx; p.bcy = c->bcy; p.S = c->S; p.rate = c->rate; p.flag = c->d_flag;
    p.stat = c->fstat;
    p.ztab = c->d_zeta;
    const int chunk = (c->q.nvel + waves - 1) / waves;
    p.chunk = (chunk + RLBM_LB - 1) / RLBM_LB * RLBM_LB;
    p.band = RLBM_BAND_DEFAULT;
    return p;
}

extern "C" {

int rlbm_init_quadrature(rlbm_ctx* out, int n_radial, int n_angle, int order, int rotate)
{
    if (!out) return RLBM_EINVAL;
    *out = nullptr;
    rlbm_ctx c = new (std::nothrow) rlbm_ctx_s();
    if (!c) return RLBM_ENOMEM;
    std::string err;
    const int rc = build_host_quad(c->q, n_radial, n_angle, order, rotate, err);
    if (rc != RLBM_OK) {
        delete c;
        return rc;
    }
    build_zeta_table(c->zeta);
    *out = c;
    return RLBM_OK;
}

int rlbm_nvel(rlbm_ctx c) { return c ? c->q.nvel : RLBM_EINVAL; }

int rlbm_get_quadrature(rlbm_ctx c, double* p, double* theta, double* w)
{
    if (!c) return RLBM_EINVAL;
    for (int v = 0; v < c->q.nvel; ++v) {
        if (p) p[v] = c->q.p[v];
        if (theta) theta[v] = c->q.theta[v];
        if (w) w[v] = c->q.w[v];
    }
    return RLBM_OK;
}

int rlbm_workspace_bytes(rlbm_ctx c, int nx, int ny, int precision, size_t* bytes)
{
    if (!c || !bytes || nx < 1 || ny < 1) return fail(c, RLBM_EINVAL, "workspace_bytes: bad arguments");
    if (!valid_prec(precision)) return fail(c, RLBM_EINVAL, "unsupported precision");
    *bytes = layout(c->q.nvel, nx, ny, precision, dev_planes(c->q.Np, c->q.N)).total;
    return RLBM_OK;
}

int rlbm_init_fields(rlbm_ctx c, int nx, int ny, const double* n, const double* T, const double* ux,
                     const double* uy, double tau, double dt, int bc_x, int bc_y, int precision,
                     void* d_workspace, void* hip_stream)
{
    if (!c) return RLBM_EINVAL;
    if (nx < 1 || ny < 1 || (long long)nx * ny > (1LL << 31)) return fail(c, RLBM_EINVAL, "grid size out of range");
    if (!n || !T) return fail(c, RLBM_EINVAL, "n and T are required");
    if (!(tau > 0.0) || std::isnan(tau)) return fail(c, RLBM_EINVAL, "tau must be > 0 (inf allowed)");
    if (!(dt > 0.0 && dt <= 1.0)) return fail(c, RLBM_EINVAL, "dt must be in (0, 1]");
    if (bc_x < RLBM_BC_PERIODIC || bc_x > RLBM_BC_FIXED || bc_y < RLBM_BC_PERIODIC || bc_y > RLBM_BC_FIXED)
        return fail(c, RLBM_EINVAL, "bad boundary condition");
    if ((bc_x == RLBM_BC_WALL || bc_y == RLBM_BC_WALL) && (c->q.K % 2))
        return fail(c, RLBM_EINVAL, "a wall needs an even number of angles (reversed velocities)");
    if (!valid_prec(precision)) return fail(c, RLBM_EINVAL, "unsupported precision");
    if (is_dev(precision) && (special_bc(bc_x, bc_y) || c->stat != RLBM_STAT_MJ))
        return fail(c, RLBM_EINVAL, "deviation storage supports periodic and clamped axes and Maxwell-Juttner "
                                    "statistics");
    if (d_workspace && ((uintptr_t)d_workspace & 255)) return fail(c, RLBM_EINVAL, "workspace must be 256-byte aligned");
    const long long S = (long long)nx * ny;
    if (!finite_arr(n, S) || !finite_arr(T, S) || (ux && !finite_arr(ux, S)) || (uy && !finite_arr(uy, S)))
        return fail(c, RLBM_EINVAL, "fields must be finite");
    for (long long i = 0; i < S; ++i)
        if (!(n[i] > 0.0) || !(T[i] > 0.0)) return fail(c, RLBM_EINVAL, "n and T must be positive");
    if (c->stat == RLBM_STAT_BOSE)   // n = T^2 Li_2(z) <= T^2 zeta(2) for a Bose-Einstein equilibrium
        for (long long i = 0; i < S; ++i)
            if (!(n[i] / (T[i] * T[i]) < c->zeta[2 + RLBM_ZMIN]))
                return fail(c, RLBM_EINVAL, "no Bose-Einstein equilibrium: n / T^2 must stay below zeta(2)");

    // From here on the context holds no usable state until this call
    // succeeds: a failure below leaves rlbm_step and rlbm_moments returning
    // RLBM_ESTATE instead of running on freed or partial tables.
    if (c->have_fields) (void)hipStreamSynchronize(c->st);
    c->have_fields = 0;
    c->pvalid = 0;
    free_tables(c);
    push_free(c);

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(c, e, "hipGetDevice");
    if (scratch_setup(dev) != RLBM_OK) return fail(c, RLBM_EDEVICE, "device scratch address");
    c->dev = dev;
    const Layout L = layout(c->q.nvel, nx, ny, precision, dev_planes(c->q.Np, c->q.N));
    hipStream_t st = static_cast<hipStream_t>(hip_stream);

    if (d_workspace) {
        if (c->ws_owned && c->ws) (void)hipFree(c->ws);
        c->ws = static_cast<char*>(d_workspace);
        c->ws_owned = false;
        c->ws_bytes = L.total;
    } else if (!c->ws_owned || c->ws_bytes < L.total) {
        if (c->ws_owned && c->ws) (void)hipFree(c->ws);
        c->ws = nullptr;
        c->ws_owned = false;
        void* p = nullptr;
        e = hipMalloc(&p, L.total);
        if (e != hipSuccess) return fail(c, RLBM_ENOMEM, "hipMalloc of the workspace failed");
        c->ws = static_cast<char*>(p);
        c->ws_owned = true;
        c->ws_bytes = L.total;
    }
    c->nx = nx; c->ny = ny; c->S = S; c->prec = precision;
    c->fstat = c->stat;
    c->bcx = bc_x; c->bcy = bc_y; c->tau = tau; c->dt = dt;
    c->rate = std::isinf(tau) ? 0.0 : dt / tau;
    c->st = st;
    c->f[0] = c->ws + L.f0;
    c->f[1] = c->ws + L.f1;
    c->d_fields = reinterpret_cast<double*>(c->ws + L.fields);
    c->d_partials = reinterpret_cast<double*>(c->ws + L.partials);
    c->d_flag = reinterpret_cast<int*>(c->ws + L.flag);
    c->d_edges = c->ws + L.edges;
    c->pp[0] = c->ws + L.pp0;
    c->pp[1] = c->ws + L.pp1;
    c->cf[0] = is_dev(precision) ? c->ws + L.cf0 : nullptr;
    c->cf[1] = is_dev(precision) ? c->ws + L.cf1 : nullptr;
    c->cur = 0;
    c->pcur = 0;
    c->steps = 0;

    // device tables
    std::vector<VelRec<double>> vd;
    build_vel_table(c->q, dt, vd);
    const size_t nv = c->q.nvel;
    if ((e = hipMalloc(&c->d_veld, nv * sizeof(VelRec<double>))) != hipSuccess) return fail(c, RLBM_ENOMEM, "table alloc");
    if ((e = hipMalloc(&c->d_G, c->q.G.size() * sizeof(double))) != hipSuccess) return fail(c, RLBM_ENOMEM, "table alloc");
    if ((e = hipMalloc(&c->d_Pc, c->q.Pc.size() * sizeof(double))) != hipSuccess) return fail(c, RLBM_ENOMEM, "table alloc");
    if ((e = hipMemcpy(c->d_veld, vd.data(), nv * sizeof(VelRec<double>), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "table upload");
    if ((e = hipMemcpy(c->d_G, c->q.G.data(), c->q.G.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "table upload");
    if ((e = hipMemcpy(c->d_Pc, c->q.Pc.data(), c->q.Pc.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "table upload");
    if ((e = hipMalloc(&c->d_zeta, sizeof(c->zeta))) != hipSuccess) return fail(c, RLBM_ENOMEM, "table alloc");
    if ((e = hipMemcpy(c->d_zeta, c->zeta, sizeof(c->zeta), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "table upload");
    // kernel tables, padded with null entries (zero weights, spare plane),
    // for both step kernels
    {
        const int rc = upload_kernel_tables(c, vd, S, precision);
        if (rc != RLBM_OK) return rc;
        std::string err;
        const int prc = push_setup(c, err);
        if (prc != RLBM_OK) {
            push_free(c);
            return fail(c, prc, "push kernel tables: " + err);
        }
        if (is_dev(precision)) {
            const int drc = dev_setup(c, err);
            if (drc != RLBM_OK) return fail(c, drc, "deviation tables: " + err);
        }
    }

    // upload the fields and build f = f_eq
    std::vector<double> h(4 * (size_t)S, 0.0);
    std::memcpy(h.data(), n, S * sizeof(double));
    std::memcpy(h.data() + S, T, S * sizeof(double));
    if (ux) std::memcpy(h.data() + 2 * S, ux, S * sizeof(double));
    if (uy) std::memcpy(h.data() + 3 * S, uy, S * sizeof(double));
    if ((e = hipMemcpyAsync(c->d_fields, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, st)) != hipSuccess)
        return hip_fail(c, e, "field upload");
    if ((e = hipMemsetAsync(c->d_flag, 0, sizeof(int), st)) != hipSuccess) return hip_fail(c, e, "flag clear");
    if (is_dev(precision)) {
        // f = F exactly: the equilibrium's coefficients, zero deviations
        if ((e = launch_dev_init(c, st)) != hipSuccess) return hip_fail(c, e, "deviation init kernel");
    } else {
        for (int b = 0; b < 2; ++b) {   // spare planes written by the null table entries
            char* spare = static_cast<char*>(c->f[b]) + (size_t)c->q.nvel * S * elem_size(precision);
            if ((e = hipMemsetAsync(spare, 0, (size_t)S * elem_size(precision), st)) != hipSuccess)
                return hip_fail(c, e, "spare clear");
        }
        e = launch_init(precision, nmax_of(c->q.N), c->d_fields, c->f[0], c->d_veld, c->d_G, c->d_Pc, nx, ny,
                        c->q.nvel, c->q.K, c->q.Np, c->fstat, c->d_zeta, st);
        if (e != hipSuccess) return hip_fail(c, e, "init kernel");
        e = launch_edges(precision, c->f[0], c->d_edges, nx, ny, c->q.nvel, st);
        if (e != hipSuccess) return hip_fail(c, e, "edge copy kernel");
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(c, e, "init sync");
    if (!c->ev0) {
        if ((e = hipEventCreate(&c->ev0)) != hipSuccess) return hip_fail(c, e, "event");
        if ((e = hipEventCreate(&c->ev1)) != hipSuccess) return hip_fail(c, e, "event");
    }
    c->have_fields = 1;
    return RLBM_OK;
}

int rlbm_set_waves(rlbm_ctx c, int waves)
{
    if (!c) return RLBM_EINVAL;
    if (waves < 0 || waves > 16) return fail(c, RLBM_EINVAL, "waves must be in [0, 16]");
    c->waves = waves;
    return RLBM_OK;
}

int rlbm_get_waves(rlbm_ctx c, int* waves)
{
    if (!c || !waves) return RLBM_EINVAL;
    *waves = c->waves ? c->waves : default_waves(c->prec, nmax_of(c->q.N), c->q.nvel);
    return RLBM_OK;
}

int rlbm_step(rlbm_ctx c, int nsteps)
{
    if (!c) return RLBM_EINVAL;
    if (!c->have_fields) return fail(c, RLBM_ESTATE, "rlbm_step before rlbm_init_fields");
    if (nsteps < 0) return fail(c, RLBM_EINVAL, "nsteps < 0");
    if (resolve_kernel(c) == RLBM_KERNEL_PUSH) {
        if (general_step(c->bcx, c->bcy, c->fstat))
            return fail(c, RLBM_EINVAL, "walls, fixed edges and quantum statistics need the tile kernel");
        if (!c->d_prec) return fail(c, RLBM_ESTATE, "push kernel tables missing");
        hipError_t e;
        if (!c->pvalid && nsteps > 0) {
            if ((e = launch_push(c, true)) != hipSuccess) return hip_fail(c, e, "push partial sums launch");
            c->pvalid = 1;
        }
        for (int s = 0; s < nsteps; ++s) {
            if ((e = launch_push(c, false)) != hipSuccess) return hip_fail(c, e, "push step launch");
            c->cur ^= 1;
            c->pcur ^= 1;
            ++c->steps;
        }
        return RLBM_OK;
    }
    c->pvalid = 0;
    const int waves = c->waves ? c->waves : default_waves(c->prec, nmax_of(c->q.N), c->q.nvel);
    SCParams p = make_params(c, waves);
    for (int s = 0; s < nsteps; ++s) {
        p.fin = c->f[c->cur];
        p.fout = c->f[c->cur ^ 1];
        const hipError_t e = launch_stream_collide(c->prec, nmax_of(c->q.N), waves, p, c->st);
        if (e != hipSuccess) return hip_fail(c, e, "stream_collide launch");
        c->cur ^= 1;
        ++c->steps;
    }
    return RLBM_OK;
}

int rlbm_step_timed(rlbm_ctx c, int nsteps, double* ms)
{
    if (!c || !ms) return RLBM_EINVAL;
    if (!c->have_fields) return fail(c, RLBM_ESTATE, "rlbm_step_timed before rlbm_init_fields");
    hipError_t e = hipEventRecord(c->ev0, c->st);
    if (e != hipSuccess) return hip_fail(c, e, "event record");
    const int rc = rlbm_step(c, nsteps);
    if (rc != RLBM_OK) return rc;
    if ((e = hipEventRecord(c->ev1, c->st)) != hipSuccess) return hip_fail(c, e, "event record");
    if ((e = hipEventSynchronize(c->ev1)) != hipSuccess) return hip_fail(c, e, "event sync");
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, c->ev0, c->ev1)) != hipSuccess) return hip_fail(c, e, "elapsed");
    *ms = t;
    return RLBM_OK;
}

int rlbm_moments(rlbm_ctx c, double* n, double* eps, double* ux, double* uy, double* charges)
{
    if (!c) return RLBM_EINVAL;
    if (!c->have_fields) return fail(c, RLBM_ESTATE, "rlbm_moments before rlbm_init_fields");
    hipError_t e = is_dev(c->prec) ? launch_dev_fields(c, c->d_fields, c->d_partials, c->st)
                                   : launch_fields(c->prec, c->f[c->cur], c->d_veld, c->d_fields, c->d_partials,
                                                   c->d_flag, c->nx, c->ny, c->q.nvel, c->st);
    if (e != hipSuccess) return hip_fail(c, e, "fields launch");
    return fields_out(c, n, eps, ux, uy, charges);
}

// The fields and charges of rlbm_moments into caller-owned device memory,
// asynchronously, with the partial charges in the fixed device scratch.
int rlbm_moments_device(rlbm_ctx c, double* d_fields, double* d_charges)
{
    if (!c) return RLBM_EINVAL;
    if (!c->have_fields) return fail(c, RLBM_ESTATE, "rlbm_moments_device before rlbm_init_fields");
    if (c->S > scratch_max_sites())
        return fail(c, RLBM_EINVAL, "rlbm_moments_device: grid larger than the device scratch allows (" +
                                        std::to_string(scratch_max_sites()) + " sites)");
    double* partials = static_cast<double*>(scratch_ptr(c->dev));
    if (!partials) return fail(c, RLBM_ESTATE, "device scratch not set up");
    hipError_t e;
    if (is_dev(c->prec)) {
        e = launch_dev_fields(c, d_fields ? d_fields : c->d_fields, partials, c->st);
        if (e == hipSuccess && d_charges) e = launch_charges_sum(partials, fields_blocks(c->S), d_charges, c->st);
    } else {
        e = launch_fields_charges(c->prec, c->f[c->cur], c->d_veld, d_fields ? d_fields : c->d_fields, partials,
                                  d_charges, c->d_flag, c->nx, c->ny, c->q.nvel, c->st);
    }
    return e == hipSuccess ? RLBM_OK : hip_fail(c, e, "moments_device launch");
}

}  // extern "C"

// Copy the fields computed into d_fields (and the charges) to the host,
// synchronise, and report a non-physical state met since the last call.
int fields_out(rlbm_ctx c, double* n, double* eps, double* ux, double* uy, double* charges)
{
    hipError_t e;
    const long long S = c->S;
    double* outs[4] = {n, eps, ux, uy};
    for (int k = 0; k < 4; ++k)
        if (outs[k]) {
            e = hipMemcpyAsync(outs[k], c->d_fields + k * S, S * sizeof(double), hipMemcpyDeviceToHost, c->st);
            if (e != hipSuccess) return hip_fail(c, e, "fields copy");
        }
    const int nb = fields_blocks(S);
    std::vector<double> part(4 * (size_t)nb);
    e = hipMemcpyAsync(part.data(), c->d_partials, part.size() * sizeof(double), hipMemcpyDeviceToHost, c->st);
    if (e != hipSuccess) return hip_fail(c, e, "charges copy");
    int flag = 0;
    if ((e = hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->st)) != hipSuccess)
        return hip_fail(c, e, "flag copy");
    if ((e = hipStreamSynchronize(c->st)) != hipSuccess) return hip_fail(c, e, "moments sync");
    if (charges) {
        long double acc[4] = {0, 0, 0, 0};
        for (int b = 0; b < nb; ++b)
            for (int k = 0; k < 4; ++k) acc[k] += part[4 * (size_t)b + k];
        for (int k = 0; k < 4; ++k) charges[k] = (double)acc[k];
    }
    if (flag) {
        if ((e = hipMemsetAsync(c->d_flag, 0, sizeof(int), c->st)) != hipSuccess) return hip_fail(c, e, "flag clear");
        (void)hipStreamSynchronize(c->st);
        return fail(c, RLBM_ENONPHYS, "non-physical state met (no timelike Landau frame, n <= 0 or eps <= 0)");
    }
    return RLBM_OK;
}

extern "C" {

int rlbm_populations_bytes(rlbm_ctx c, size_t* bytes)
{
    if (!c || !bytes) return RLBM_EINVAL;
    if (!c->have_fields) return fail(c, RLBM_ESTATE, "no populations yet");
    *bytes = (size_t)c->q.nvel * c->S * elem_size(c->prec);
    if (is_dev(c->prec)) *bytes += (size_t)dev_planes(c->q.Np, c->q.N) * c->S * arith_size(c->prec);
    return RLBM_OK;
}

int rlbm_get_populations(rlbm_ctx c, void* host, size_t bytes)
{
    size_t need = 0;
    int rc = rlbm_populations_bytes(c, &need);
    if (rc != RLBM_OK) return rc;
    if (!host || bytes != need) return fail(c, RLBM_EINVAL, "population buffer size mismatch");
    hipError_t e = hipStreamSynchronize(c->st);
    const size_t gb = (size_t)c->q.nvel * c->S * elem_size(c->prec);
    if (e == hipSuccess) e = hipMemcpy(host, c->f[c->cur], gb, hipMemcpyDeviceToHost);
    if (e == hipSuccess && is_dev(c->prec))
        e = hipMemcpy(static_cast<char*>(host) + gb, c->cf[c->cur], need - gb, hipMemcpyDeviceToHost);
    return e == hipSuccess ? RLBM_OK : hip_fail(c, e, "get_populations");
}

int rlbm_set_populations(rlbm_ctx c, const void* host, size_t bytes)
{
    size_t need = 0;
    int rc = rlbm_populations_bytes(c, &need);
    if (rc != RLBM_OK) return rc;
    if (!host || bytes != need) return fail(c, RLBM_EINVAL, "population buffer size mismatch");
    hipError_t e = hipStreamSynchronize(c->st);
    const size_t gb = (size_t)c->q.nvel * c->S * elem_size(c->prec);
    if (e == hipSuccess) e = hipMemcpy(c->f[c->cur], host, gb, hipMemcpyHostToDevice);
    if (e == hipSuccess && is_dev(c->prec))
        e = hipMemcpy(c->cf[c->cur], static_cast<const char*>(host) + gb, need - gb, hipMemcpyHostToDevice);
    c->pvalid = 0;
    return e == hipSuccess ? RLBM_OK : hip_fail(c, e, "set_populations");
}

int rlbm_set_kernel(rlbm_ctx c, int kind)
{
    if (!c) return RLBM_EINVAL;
    if (kind != RLBM_KERNEL_AUTO && kind != RLBM_KERNEL_TILE && kind != RLBM_KERNEL_PUSH)
        return fail(c, RLBM_EINVAL, "unknown kernel kind");
    if (kind == RLBM_KERNEL_PUSH && c->have_fields && general_step(c->bcx, c->bcy, c->fstat))
        return fail(c, RLBM_EINVAL, "walls, fixed edges and quantum statistics need the tile kernel");
    if (kind == RLBM_KERNEL_TILE && c->have_fields && is_dev(c->prec))
        return fail(c, RLBM_EINVAL, "deviation storage runs on the push kernel");
    c->kern = kind;
    c->pvalid = 0;
    return RLBM_OK;
}

int rlbm_get_kernel(rlbm_ctx c, int* kind)
{
    if (!c || !kind) return RLBM_EINVAL;
    *kind = resolve_kernel(c);
    return RLBM_OK;
}

const char* rlbm_last_error(rlbm_ctx c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

int rlbm_destroy(rlbm_ctx c)
{
    if (!c) return RLBM_EINVAL;
    if (c->have_fields) (void)hipStreamSynchronize(c->st);
    free_tables(c);
    push_free(c);
    if (c->ws_owned && c->ws) (void)hipFree(c->ws);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
    return RLBM_OK;
}

// Host-side evaluations with the library's own tables (no device call): the
// discrete equilibrium of given fields and the Landau frame of nine moments.
int rlbm_host_feq(rlbm_ctx c, double n, double T, double ux, double uy, double* feq)
{
    if (!c || !feq) return RLBM_EINVAL;
    std::vector<VelRec<double>> vd;
    build_vel_table(c->q, 1.0, vd);
    const double U0 = std::sqrt(1.0 + ux * ux + uy * uy);
    const int GS = (RLBM_NMAX + 1) * (RLBM_NMAX + 1);
    double phi[RLBM_NMAX + 1];
    if (qs_phi_of_nT(n, T, c->stat, RLBM_NMAX, (const double*)c->zeta, phi)) return RLBM_ENONPHYS;
    for (int i = 0; i < c->q.Np; ++i) {
        double cf[RLBM_NT];
        shell_coeffs<RLBM_NMAX>(c->q.G.data() + (size_t)i * GS, c->q.Pc.data(), n, T, U0, ux, uy,
                                [&](int m, double cm, double sm) {
                                    if (m == 0) {
                                        cf[0] = cm;
                                    } else {
                                        cf[2 * m - 1] = cm;
                                        cf[2 * m] = sm;
                                    }
                                },
                                c->stat != RLBM_STAT_MJ ? phi : nullptr);
        for (int j = 0; j < c->q.K; ++j) {
            const int v = i * c->q.K + j;
            double fe = 0.0;
            for (int t = 0; t < RLBM_NT; ++t) fe += cf[t] * vd[v].H[t];
            feq[v] = fe;
        }
    }
    return RLBM_OK;
}

int rlbm_set_statistics(rlbm_ctx c, int statistics)
{
    if (!c) return RLBM_EINVAL;
    if (statistics != RLBM_STAT_MJ && statistics != RLBM_STAT_FERMI && statistics != RLBM_STAT_BOSE)
        return fail(c, RLBM_EINVAL, "unknown statistics");
    c->stat = statistics;
    return RLBM_OK;
}

int rlbm_host_landau(const double* mom9, double* out6)
{
    if (!mom9 || !out6) return RLBM_EINVAL;
    const Frame fr = landau_frame(mom9);
    out6[0] = fr.n; out6[1] = fr.eps; out6[2] = fr.Ux; out6[3] = fr.Uy; out6[4] = fr.T; out6[5] = fr.U0;
    return fr.ok ? RLBM_OK : RLBM_ENONPHYS;
}

// Device evaluation of the Landau frame of count moment sets (host arrays
// mom[count][9] -> out[count][7] = n, eps, U^x, U^y, T, U^0, ok), through the
// same device function as the kernels.  Synchronous; allocates scratch.
int rlbm_device_landau(int count, const double* mom, double* out)
{
    if (count < 0 || (count > 0 && (!mom || !out))) return RLBM_EINVAL;
    if (count == 0) return RLBM_OK;
    double *dm = nullptr, *dout = nullptr;
    hipError_t e = hipMalloc(&dm, sizeof(double) * 9 * (size_t)count);
    if (e == hipSuccess) e = hipMalloc(&dout, sizeof(double) * 7 * (size_t)count);
    if (e == hipSuccess) e = hipMemcpy(dm, mom, sizeof(double) * 9 * (size_t)count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_landau_probe(dm, dout, count, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, dout, sizeof(double) * 7 * (size_t)count, hipMemcpyDeviceToHost);
    if (dm) (void)hipFree(dm);
    if (dout) (void)hipFree(dout);
    return e == hipSuccess ? RLBM_OK : RLBM_EDEVICE;
}

}  // extern "C"
