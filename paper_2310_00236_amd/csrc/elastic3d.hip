// 3D elastic (velocity-stress) leapfrog step and energy kernels for gfx950.
//
// A step advances the velocities from the divergence of the old stresses,
// then the six stresses from the new velocities (the 3D form of Eq. A1,
// App. A, 2nd-order staggered differences).  The fields ping-pong between
// two sets: a step reads set n and writes set n+1.  Two kernel shapes are
// compiled (the autotuner picks per problem):
//   two-pass: a velocity kernel, then a stress kernel, one thread per cell
//             of one z plane;
//   fused:    one kernel; a workgroup walks a column of cells along z and
//             computes, at each plane, the new velocities of the plane
//             above and then the new stresses of the plane itself, so every
//             word of the state is read once and written once per step.
// Every arithmetic operation follows the same op-by-op definition as the
// CPU reference, so results are bit-identical to it and independent of the
// kernel shape and of the batch a shot runs in.
#include "hw_device.h"
#include "hw_internal.h"

#pragma clang fp contract(off)

namespace hw {

__device__ __forceinline__ int32_t xcd_tile3(int32_t b, int32_t n)
{
    return xcd_band<kNumXcd>(b, n);
}

__device__ __forceinline__ int find_shot3(const El3dBatch &a, int32_t t)
{
    int lo = 0, hi = a.nshots - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.tile_start[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int wrapu(int i, int n)
{
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Periodic wrap of a 32-bit index (any offset).
__device__ __forceinline__ int wrap3(int i, int n)
{
    const int r = i % n;
    return r < 0 ? r + n : r;
}

// ------------------------------------------------------------ two-pass --

struct Cell {
    int i, j, k;
    bool valid;
};

template <int TX, int TY>
__device__ __forceinline__ Cell locate(const El3dBatch &a, const El3dDesc *&dp,
                                       int &par)
{
    int32_t tile = xcd_tile3(blockIdx.x, a.total_tiles);
    const int shot = find_shot3(a, tile);
    dp = a.desc[shot];
    par = a.parity[shot];
    const El3dDesc &d = *dp;
    tile -= a.tile_start[shot];
    const int ntx = a.tiles_x[shot];
    const int per_slice = ntx * a.tiles_y[shot];
    const int r = tile % per_slice;
    Cell c;
    c.k = tile / per_slice;
    c.i = (r % ntx) * TX + (int)threadIdx.x % TX;
    c.j = (r / ntx) * TY + (int)threadIdx.x / TX;
    c.valid = c.i < (int)d.nx && c.j < (int)d.ny;
    return c;
}

// Velocities of one cell: old stresses and velocities from set par, new
// velocities to set par^1.  The cell's own words are read and written once
// per pass, non-temporally (6-8% faster at 512^3); the neighbours' stresses
// go through the caches.
template <class S, int COMP, int TX, int TY>
__global__ __launch_bounds__(kThreads) void el3d_velocity_kernel(const El3dBatch a)
{
    using WD = Word<S, COMP>;
    using W = typename WD::type;
    const El3dDesc *dp;
    int par;
    const Cell cl = locate<TX, TY>(a, dp, par);
    if (!cl.valid)
        return;
    const El3dDesc &d = *dp;
    const int nx = (int)d.nx, ny = (int)d.ny, nz = (int)d.nz;
    const int pitch = (int)d.pitch, slab = (int)d.slab;
    const int i = cl.i, j = cl.j, k = cl.k;
    const int ip = wrapu(i + 1, nx), im = wrapu(i - 1, nx);
    const int jp = wrapu(j + 1, ny), jm = wrapu(j - 1, ny);
    const int kp = wrapu(k + 1, nz), km = wrapu(k - 1, nz);
    const int row = k * slab + j * pitch;
    const int q = row + i;
    const float w = d.w;
    using GW = const W HW_GLOBAL *;
    const float HW_GLOBAL *__restrict__ B = gmem(d.b);
    GW sxx = gmem((const W *)d.f[par][3]), syy = gmem((const W *)d.f[par][4]);
    GW szz = gmem((const W *)d.f[par][5]), sxy = gmem((const W *)d.f[par][6]);
    GW sxz = gmem((const W *)d.f[par][7]), syz = gmem((const W *)d.f[par][8]);
    auto L = [](GW p, int idx) { return S::load(WD::v(p[idx])); };
    const float sxy_q = L(sxy, q), sxz_q = L(sxz, q), syz_q = L(syz, q);
    const float bq = B[q];
    float inc[3];
    {   // vx at (i+1/2, j, k)
        const float d1 = L(sxx, row + ip) - L(sxx, q);
        const float d2 = sxy_q - L(sxy, k * slab + jm * pitch + i);
        const float d3 = sxz_q - L(sxz, km * slab + j * pitch + i);
        const float g = w * ((d1 + d2) + d3);
        const float bb = 0.5f * (bq + B[row + ip]);
        inc[0] = bb * g;
    }
    {   // vy at (i, j+1/2, k)
        const float d1 = sxy_q - L(sxy, row + im);
        const float d2 = L(syy, k * slab + jp * pitch + i) - L(syy, q);
        const float d3 = syz_q - L(syz, km * slab + j * pitch + i);
        const float g = w * ((d1 + d2) + d3);
        const float bb = 0.5f * (bq + B[k * slab + jp * pitch + i]);
        inc[1] = bb * g;
    }
    {   // vz at (i, j, k+1/2)
        const float d1 = sxz_q - L(sxz, row + im);
        const float d2 = syz_q - L(syz, k * slab + jm * pitch + i);
        const float d3 = L(szz, kp * slab + j * pitch + i) - L(szz, q);
        const float g = w * ((d1 + d2) + d3);
        const float bb = 0.5f * (bq + B[kp * slab + j * pitch + i]);
        inc[2] = bb * g;
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const W old = __builtin_nontemporal_load(gmem((const W *)d.f[par][f]) + q);
        auto v = WD::v(old), c = WD::c(old);
        update_store<S, COMP>(v, c, inc[f]);
        __builtin_nontemporal_store(WD::make(v, c), gmem((W *)d.f[par ^ 1][f]) + q);
    }
}

// Stresses of one cell: new velocities from set par^1, old stresses from
// set par, new stresses to set par^1.
template <class S, int COMP, int TX, int TY>
__global__ __launch_bounds__(kThreads) void el3d_stress_kernel(const El3dBatch a)
{
    using WD = Word<S, COMP>;
    using W = typename WD::type;
    const El3dDesc *dp;
    int par;
    const Cell cl = locate<TX, TY>(a, dp, par);
    if (!cl.valid)
        return;
    const El3dDesc &d = *dp;
    const int nx = (int)d.nx, ny = (int)d.ny, nz = (int)d.nz;
    const int pitch = (int)d.pitch, slab = (int)d.slab;
    const int i = cl.i, j = cl.j, k = cl.k;
    const int ip = wrapu(i + 1, nx), im = wrapu(i - 1, nx);
    const int jp = wrapu(j + 1, ny), jm = wrapu(j - 1, ny);
    const int kp = wrapu(k + 1, nz), km = wrapu(k - 1, nz);
    const int row = k * slab + j * pitch;
    const int q = row + i;
    const float w = d.w;
    using GW = const W HW_GLOBAL *;
    GW vx = gmem((const W *)d.f[par ^ 1][0]), vy = gmem((const W *)d.f[par ^ 1][1]);
    GW vz = gmem((const W *)d.f[par ^ 1][2]);
    auto L = [](GW p, int idx) { return S::load(WD::v(p[idx])); };
    const float HW_GLOBAL *__restrict__ M = gmem(d.mu);
    const float HW_GLOBAL *__restrict__ LM = gmem(d.lam);
    const float vx_q = L(vx, q), vy_q = L(vy, q), vz_q = L(vz, q);
    const float ex = w * (vx_q - L(vx, row + im));
    const float ey = w * (vy_q - L(vy, k * slab + jm * pitch + i));
    const float ez = w * (vz_q - L(vz, km * slab + j * pitch + i));
    const float lam = __builtin_nontemporal_load(LM + q);
    const float mq = M[q];
    const float l2m = lam + 2.0f * mq;
    float inc[6];
    inc[0] = l2m * ex + lam * (ey + ez);
    inc[1] = l2m * ey + lam * (ex + ez);
    inc[2] = l2m * ez + lam * (ex + ey);
    const int q_ip = row + ip;
    const int q_jp = k * slab + jp * pitch + i;
    const int q_kp = kp * slab + j * pitch + i;
    {   // sxy at (i+1/2, j+1/2, k)
        const float a1 = L(vy, q_ip) - vy_q;
        const float a2 = L(vx, q_jp) - vx_q;
        const float g = w * (a1 + a2);
        const float m = 0.25f * ((mq + M[q_ip]) +
                                 (M[q_jp] + M[k * slab + jp * pitch + ip]));
        inc[3] = m * g;
    }
    {   // sxz at (i+1/2, j, k+1/2)
        const float a1 = L(vz, q_ip) - vz_q;
        const float a2 = L(vx, q_kp) - vx_q;
        const float g = w * (a1 + a2);
        const float m = 0.25f * ((mq + M[q_ip]) +
                                 (M[q_kp] + M[kp * slab + j * pitch + ip]));
        inc[4] = m * g;
    }
    {   // syz at (i, j+1/2, k+1/2)
        const float a1 = L(vz, q_jp) - vz_q;
        const float a2 = L(vy, q_kp) - vy_q;
        const float g = w * (a1 + a2);
        const float m = 0.25f * ((mq + M[q_jp]) +
                                 (M[q_kp] + M[kp * slab + jp * pitch + i]));
        inc[5] = m * g;
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const W old = __builtin_nontemporal_load(gmem((const W *)d.f[par][3 + f]) + q);
        auto v = WD::v(old), c = WD::c(old);
        update_store<S, COMP>(v, c, inc[f]);
        __builtin_nontemporal_store(WD::make(v, c), gmem((W *)d.f[par ^ 1][3 + f]) + q);
    }
}

// --------------------------------------------------------------- fused --

template <class S, int COMP>
__device__ __forceinline__ void update_word(typename Word<S, COMP>::type &w, float inc)
{
    using WD = Word<S, COMP>;
    auto v = WD::v(w), c = WD::c(w);
    update_store<S, COMP>(v, c, inc);
    w = WD::make(v, c);
}

// One fused step over a column of cells: tile columns [x0, x0+64), rows
// [y0, y0+TY), planes [k0, k1).
//
// Plane m = k+1 of the new velocities needs the old stresses of planes k,
// k+1 and k+2; plane k of the new stresses needs the new velocities of
// planes k-1, k and k+1.  So iteration k computes the velocities of plane
// k+1 (from old values only: the inputs come from set par, the outputs go
// to set par^1) and then the stresses of plane k.  Along z everything a
// cell needs from the planes before stays in that thread's registers; in
// the plane, neighbours are exchanged through LDS.  The stress stencil
// reads velocities one cell outside the tile (column -1, row -1, column 64,
// row TY); those are recomputed here from old values, so the workgroup
// never waits for its neighbours.  Two warm-up iterations (k0-2, k0-1)
// build the velocities of planes k0-1 and k0; the workgroup writes the
// velocities of planes k0+1 .. k1 and the stresses of planes k0 .. k1-1, so
// the columns of a grid partition both.
//
// Threads handle "positions" of the extended tile [-1, 64] x [-1, TY]:
// wavefront w, lane l takes column l of extended rows w-1, w+3, ...; the
// two halo columns (-1 and 64) of all extended rows are spread over the
// first lanes of the four wavefronts.  Each position loads only the words
// its own computations and its neighbours' stencils read.
template <class S, int COMP, int TY>
__device__ __forceinline__ void el3d_fused(const El3dDesc &d, int par, int x0,
                                           int y0, int k0, int k1, float *lds)
{
    using WD = Word<S, COMP>;
    using W = typename WD::type;
    constexpr int TX = 64;
    constexpr int ER = TY + 2;            // extended rows -1 .. TY
    constexpr int M = ER / 4;             // extended rows per wavefront
    constexpr int NP = M + 1;             // + one halo-column position
    constexpr int LS = TX + 2;            // LDS row stride, column c at c+1
    constexpr int NG = ER * LS;           // one LDS grid
    static_assert(ER % 4 == 0 && ER / 2 <= 64, "extended tile layout");
    enum { XX = 0, YY, XY, XZ, YZ };      // stresses staged in LDS
    float *gs = lds;                      // 5 grids: old stresses, plane k+1
    float *gb = lds + 5 * NG;             // 1/rho, plane k+1
    float *gm = lds + 6 * NG;             // mu, 2 planes (plane parity)
    float *gv = lds + 8 * NG;             // new velocities, 2 planes x 3
    enum : unsigned {
        F_ACT = 1u, F_SXX = 4u, F_SYY = 8u, F_SZZ = 16u,
        F_SXZ = 32u, F_SYZ = 64u, F_VX = 128u, F_VY = 256u, F_VZ = 512u,
        F_MU = 1024u
    };
    // the wavefront index in a scalar register: the flags of the row
    // positions (q < M) are then wavefront-uniform and their tests scalar
    // branches; only ownership (the grid's ragged edge) is decided per lane
    const int tid = threadIdx.x, ln = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    __builtin_assume(wv >= 0 && wv < 4);     // (the range the copy hides)
    const int nx = (int)d.nx, ny = (int)d.ny, nz = (int)d.nz;
    const int pitch = (int)d.pitch, slab = (int)d.slab;
    const float w = d.w;
    using GW = const W HW_GLOBAL *;
    using OW = W HW_GLOBAL *;
    GW vin[3] = {gmem((const W *)d.f[par][0]), gmem((const W *)d.f[par][1]),
                 gmem((const W *)d.f[par][2])};
    GW sin[5] = {gmem((const W *)d.f[par][3]), gmem((const W *)d.f[par][4]),
                 gmem((const W *)d.f[par][6]), gmem((const W *)d.f[par][7]),
                 gmem((const W *)d.f[par][8])};
    GW zin = gmem((const W *)d.f[par][5]);
    OW vout[3] = {gmem((W *)d.f[par ^ 1][0]), gmem((W *)d.f[par ^ 1][1]),
                  gmem((W *)d.f[par ^ 1][2])};
    OW sout[5] = {gmem((W *)d.f[par ^ 1][3]), gmem((W *)d.f[par ^ 1][4]),
                  gmem((W *)d.f[par ^ 1][6]), gmem((W *)d.f[par ^ 1][7]),
                  gmem((W *)d.f[par ^ 1][8])};
    OW zout = gmem((W *)d.f[par ^ 1][5]);
    const float HW_GLOBAL *__restrict__ B = gmem(d.b);
    const float HW_GLOBAL *__restrict__ MU = gmem(d.mu);
    const float HW_GLOBAL *__restrict__ LAM = gmem(d.lam);

    // ---- positions and what each needs
    int off[NP], li[NP];
    unsigned fl[NP];
    bool own[NP];          // the position is a cell of this column (F_OWN)
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        int lx, ly;
        bool act;
        if (q < M) {
            lx = ln;
            ly = wv + 4 * q - 1;
            act = true;
        } else {
            const int h = ln * 4 + wv;
            const int hr = h < ER ? h : h - ER;
            lx = h < ER ? -1 : TX;
            ly = hr - 1;
            act = ln < ER / 2;
        }
        const bool rowm = ly < 0, colm = lx < 0, colp = lx == TX;
        const bool inx = lx >= 0 && lx < TX, iny = ly >= 0 && ly < TY;
        unsigned f = act ? F_ACT : 0u;
        own[q] = act && inx && iny && x0 + lx < nx && y0 + ly < ny;
        if (act) {
            if (!rowm)
                f |= F_SXX | F_SXZ;
            if (!colm)
                f |= F_SYY | F_SYZ;
            if (!colm && !rowm)
                f |= F_SZZ | F_MU;
            if ((lx < TX && iny) || (inx && ly == TY))
                f |= F_VX;
            if ((inx && ly < TY) || (colp && iny))
                f |= F_VY;
            if ((inx && ly >= 0) || (colp && iny))
                f |= F_VZ;
        }
        fl[q] = f;
        off[q] = wrap3(y0 + ly, ny) * pitch + wrap3(x0 + lx, nx);
        li[q] = (ly + 1) * LS + (lx + 1);
    }

    // ---- per-iteration inputs (loaded one iteration ahead)
    struct In {
        W s[5];     // old stresses xx yy xy xz yz, plane k+1
        W zz;       // old szz, plane k+2
        W v[3];     // old velocities, plane k+1
        float b;    // 1/rho, plane k+2
        float mu;   // plane k+1
        float lam;  // plane k
    };
    auto load = [&](int k, In (&in)[NP], bool lite) {
        const int o0 = wrap3(k, nz) * slab, o1 = wrap3(k + 1, nz) * slab;
        const int o2 = wrap3(k + 2, nz) * slab;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const unsigned f = fl[q];
            if (!(f & F_ACT))
                continue;
            const int a1 = o1 + off[q], a2 = o2 + off[q];
            if (f & F_SXZ)
                in[q].s[XZ] = sin[XZ][a1];
            if (f & F_SYZ)
                in[q].s[YZ] = sin[YZ][a1];
            if (f & F_SZZ)
                in[q].zz = zin[a2];
            in[q].b = B[a2];
            if (lite)
                continue;
            if (f & F_SXX)
                in[q].s[XX] = sin[XX][a1];
            if (f & F_SYY)
                in[q].s[YY] = sin[YY][a1];
            in[q].s[XY] = sin[XY][a1];
            if (f & F_VX)
                in[q].v[0] = vin[0][a1];
            if (f & F_VY)
                in[q].v[1] = vin[1][a1];
            if (f & F_VZ)
                in[q].v[2] = vin[2][a1];
            if (f & F_MU)
                in[q].mu = MU[a1];
            if (own[q])
                in[q].lam = LAM[o0 + off[q]];
        }
    };
    auto val = [](W x) { return S::load(WD::v(x)); };

    In cur[NP] = {}, nxt[NP] = {};
    // carried along z, per position
    float sxz_k[NP], syz_k[NP], b_m[NP], vz_k[NP], vz_km1[NP];
    W zz_m[NP], zz_k[NP], sk[NP][5];
    load(k0 - 3, cur, true);
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        sxz_k[q] = val(cur[q].s[XZ]);
        syz_k[q] = val(cur[q].s[YZ]);
        zz_m[q] = cur[q].zz;
        zz_k[q] = cur[q].zz;
        b_m[q] = cur[q].b;
        vz_k[q] = vz_km1[q] = 0.0f;
#pragma unroll
        for (int n = 0; n < 5; ++n)
            sk[q][n] = cur[q].s[n];
    }
    load(k0 - 2, cur, false);

    for (int k = k0 - 2; k < k1; ++k) {
        const int pm = (k + 1) & 1, pk = k & 1;
        const int om = wrap3(k + 1, nz) * slab, ok = wrap3(k, nz) * slab;
        // ---- stage plane k+1: old stresses, 1/rho, mu
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            if (!(fl[q] & F_ACT))
                continue;
            const int l = li[q];
#pragma unroll
            for (int n = 0; n < 5; ++n)
                gs[n * NG + l] = val(cur[q].s[n]);
            gb[l] = b_m[q];
            gm[pm * NG + l] = cur[q].mu;
        }
        if (k + 1 < k1)
            load(k + 1, nxt, false);
        __syncthreads();

        // ---- new velocities of plane k+1
        const bool wr = k >= k0;
        float *vxm = gv + (3 * pm + 0) * NG, *vym = gv + (3 * pm + 1) * NG;
        float *vzm = gv + (3 * pm + 2) * NG;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const unsigned f = fl[q];
            const int l = li[q];
            if (f & F_VX) {   // vx at (i+1/2, j, k+1)
                const float d1 = gs[XX * NG + l + 1] - gs[XX * NG + l];
                const float d2 = gs[XY * NG + l] - gs[XY * NG + l - LS];
                const float d3 = val(cur[q].s[XZ]) - sxz_k[q];
                const float g = w * ((d1 + d2) + d3);
                const float bb = 0.5f * (gb[l] + gb[l + 1]);
                update_word<S, COMP>(cur[q].v[0], bb * g);
                vxm[l] = val(cur[q].v[0]);
                if (wr && own[q])
                    __builtin_nontemporal_store(cur[q].v[0], vout[0] + om + off[q]);
            }
            if (f & F_VY) {   // vy at (i, j+1/2, k+1)
                const float d1 = gs[XY * NG + l] - gs[XY * NG + l - 1];
                const float d2 = gs[YY * NG + l + LS] - gs[YY * NG + l];
                const float d3 = val(cur[q].s[YZ]) - syz_k[q];
                const float g = w * ((d1 + d2) + d3);
                const float bb = 0.5f * (gb[l] + gb[l + LS]);
                update_word<S, COMP>(cur[q].v[1], bb * g);
                vym[l] = val(cur[q].v[1]);
                if (wr && own[q])
                    __builtin_nontemporal_store(cur[q].v[1], vout[1] + om + off[q]);
            }
            if (f & F_VZ) {   // vz at (i, j, k+3/2)
                const float d1 = gs[XZ * NG + l] - gs[XZ * NG + l - 1];
                const float d2 = gs[YZ * NG + l] - gs[YZ * NG + l - LS];
                const float d3 = val(cur[q].zz) - val(zz_m[q]);
                const float g = w * ((d1 + d2) + d3);
                const float bb = 0.5f * (b_m[q] + cur[q].b);
                update_word<S, COMP>(cur[q].v[2], bb * g);
                vzm[l] = val(cur[q].v[2]);
                if (wr && own[q])
                    __builtin_nontemporal_store(cur[q].v[2], vout[2] + om + off[q]);
            }
        }

        // ---- new stresses of plane k (own cells; halo positions own none)
        if (wr) {
            const float *vxk = gv + (3 * pk + 0) * NG, *vyk = gv + (3 * pk + 1) * NG;
            const float *vzk = gv + (3 * pk + 2) * NG;
            const float *mk = gm + pk * NG, *mm = gm + pm * NG;
#pragma unroll
            for (int q = 0; q < M; ++q) {
                if (!own[q])
                    continue;
                const int l = li[q];
                const float ex = w * (vxk[l] - vxk[l - 1]);
                const float ey = w * (vyk[l] - vyk[l - LS]);
                const float ez = w * (vz_k[q] - vz_km1[q]);
                const float lam = cur[q].lam;
                const float mq = mk[l];
                const float l2m = lam + 2.0f * mq;
                float inc[6];
                inc[0] = l2m * ex + lam * (ey + ez);
                inc[1] = l2m * ey + lam * (ex + ez);
                inc[2] = l2m * ez + lam * (ex + ey);
                {   // sxy at (i+1/2, j+1/2, k)
                    const float a1 = vyk[l + 1] - vyk[l];
                    const float a2 = vxk[l + LS] - vxk[l];
                    const float g = w * (a1 + a2);
                    const float m = 0.25f * ((mq + mk[l + 1]) + (mk[l + LS] + mk[l + LS + 1]));
                    inc[3] = m * g;
                }
                {   // sxz at (i+1/2, j, k+1/2)
                    const float a1 = vzk[l + 1] - vzk[l];
                    const float a2 = val(cur[q].v[0]) - vxk[l];
                    const float g = w * (a1 + a2);
                    const float m = 0.25f * ((mq + mk[l + 1]) + (mm[l] + mm[l + 1]));
                    inc[4] = m * g;
                }
                {   // syz at (i, j+1/2, k+1/2)
                    const float a1 = vzk[l + LS] - vzk[l];
                    const float a2 = val(cur[q].v[1]) - vyk[l];
                    const float g = w * (a1 + a2);
                    const float m = 0.25f * ((mq + mk[l + LS]) + (mm[l] + mm[l + LS]));
                    inc[5] = m * g;
                }
                const int a = ok + off[q];
                update_word<S, COMP>(sk[q][XX], inc[0]);
                __builtin_nontemporal_store(sk[q][XX], sout[XX] + a);
                update_word<S, COMP>(sk[q][YY], inc[1]);
                __builtin_nontemporal_store(sk[q][YY], sout[YY] + a);
                update_word<S, COMP>(zz_k[q], inc[2]);
                __builtin_nontemporal_store(zz_k[q], zout + a);
                update_word<S, COMP>(sk[q][XY], inc[3]);
                __builtin_nontemporal_store(sk[q][XY], sout[XY] + a);
                update_word<S, COMP>(sk[q][XZ], inc[4]);
                __builtin_nontemporal_store(sk[q][XZ], sout[XZ] + a);
                update_word<S, COMP>(sk[q][YZ], inc[5]);
                __builtin_nontemporal_store(sk[q][YZ], sout[YZ] + a);
            }
        }
        __syncthreads();

        // ---- move up one plane
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            sxz_k[q] = val(cur[q].s[XZ]);
            syz_k[q] = val(cur[q].s[YZ]);
            zz_k[q] = zz_m[q];
            zz_m[q] = cur[q].zz;
            b_m[q] = cur[q].b;
            vz_km1[q] = vz_k[q];
            vz_k[q] = val(cur[q].v[2]);
#pragma unroll
            for (int n = 0; n < 5; ++n)
                sk[q][n] = cur[q].s[n];
            cur[q] = nxt[q];
        }
    }
}

template <int TY>
constexpr int fused_lds_floats()
{
    return 14 * (TY + 2) * 66;
}

template <class S, int COMP, int TY>
__device__ __forceinline__ void el3d_fused_entry(const El3dDesc &d, int par,
                                                 int tile, int ntx, int nty,
                                                 int tz, float *lds)
{
    const int per = ntx * nty;
    const int seg = tile / per, r = tile % per;
    const int x0 = (r % ntx) * 64, y0 = (r / ntx) * TY;
    const int k0 = seg * tz;
    const int k1 = k0 + tz < (int)d.nz ? k0 + tz : (int)d.nz;
    el3d_fused<S, COMP, TY>(d, par, x0, y0, k0, k1, lds);
}

template <class S, int COMP, int TY>
__global__ __launch_bounds__(kThreads) void el3d_fused_kernel(const El3dBatch a, int tz)
{
    __shared__ float lds[fused_lds_floats<TY>()];
    int32_t tile = xcd_tile3(blockIdx.x, a.total_tiles);
    const int shot = find_shot3(a, tile);
    tile -= a.tile_start[shot];
    el3d_fused_entry<S, COMP, TY>(*a.desc[shot], a.parity[shot], tile,
                                  a.tiles_x[shot], a.tiles_y[shot], tz, lds);
}

template <class S, int COMP, int TY>
__global__ __launch_bounds__(kThreads) void el3d_fused1_kernel(const El3dOne a, int tz)
{
    __shared__ float lds[fused_lds_floats<TY>()];
    const int32_t tile = xcd_tile3(blockIdx.x, a.total_tiles);
    el3d_fused_entry<S, COMP, TY>(a.d, a.parity, tile, a.tiles_x, a.tiles_y, tz, lds);
}

// -------------------------------------------------------------- energy --

__device__ __forceinline__ double block_sum3(double v, double *red)
{
    return block_sum_f64<kThreads>(v, red);
}

// Energy of the elastic state, one workgroup per (j, k) row, fp64.
template <class S>
__global__ __launch_bounds__(kThreads) void el3d_energy_kernel(
    const El3dDesc *__restrict__ dd, int par, int st, double *__restrict__ partial)
{
    using T = typename S::store_t;
    __shared__ double red[kThreads];
    const El3dDesc &d = *dd;
    const int64_t nx = d.nx, ny = d.ny, nz = d.nz, pitch = d.pitch, slab = d.slab;
    const int64_t r = xcd_band<kNumXcd>(blockIdx.x, gridDim.x);
    const int64_t k = r / ny, j = r % ny;
    const int64_t jp = wrap1(j + 1, ny), jm = wrap1(j - 1, ny);
    const int64_t kp = wrap1(k + 1, nz), km = wrap1(k - 1, nz);
    const double w = d.w;
    const T *f[9];
    for (int n = 0; n < 9; ++n)
        f[n] = (const T *)d.f[par][n];
    auto L = [&](int n, int64_t idx) { return (double)S::load(f[n][idx * st]); };
    const float *B = d.b, *LM = d.lam, *M = d.mu;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < nx; i += kThreads) {
        const int64_t ip = wrap1(i + 1, nx), im = wrap1(i - 1, nx);
        const int64_t row = k * slab + j * pitch;
        const int64_t q = row + i;
        const int64_t q_ip = row + ip, q_im = row + im;
        const int64_t q_jp = k * slab + jp * pitch + i;
        const int64_t q_jm = k * slab + jm * pitch + i;
        const int64_t q_kp = kp * slab + j * pitch + i;
        const int64_t q_km = km * slab + j * pitch + i;
        const double sxx = L(3, q), syy = L(4, q), szz = L(5, q);
        const double sxy = L(6, q), sxz = L(7, q), syz = L(8, q);
        const double gx = w * ((L(3, q_ip) - sxx) + (sxy - L(6, q_jm)) +
                               (sxz - L(7, q_km)));
        const double gy = w * ((sxy - L(6, q_im)) + (L(4, q_jp) - syy) +
                               (syz - L(8, q_km)));
        const double gz = w * ((sxz - L(7, q_im)) + (syz - L(8, q_jm)) +
                               (L(5, q_kp) - szz));
        const double bq = B[q];
        const double bx = 0.5 * (bq + (double)B[q_ip]);
        const double by = 0.5 * (bq + (double)B[q_jp]);
        const double bz = 0.5 * (bq + (double)B[q_kp]);
        const double vx = L(0, q), vy = L(1, q), vz = L(2, q);
        const double vxp = vx + bx * gx;
        const double vyp = vy + by * gy;
        const double vzp = vz + bz * gz;
        double ev = (vx * vxp) / bx + (vy * vyp) / by;
        ev = ev + (vz * vzp) / bz;
        const double lam = LM[q], mu = M[q];
        const double tr = (sxx + syy) + szz;
        const double sq = (sxx * sxx + syy * syy) + szz * szz;
        const double en = (sq - (lam / (3.0 * lam + 2.0 * mu)) * (tr * tr)) /
                          (2.0 * mu);
        const double mxy = 0.25 * (((double)M[q] + (double)M[q_ip]) +
                                   ((double)M[q_jp] + (double)M[k * slab + jp * pitch + ip]));
        const double mxz = 0.25 * (((double)M[q] + (double)M[q_ip]) +
                                   ((double)M[q_kp] + (double)M[kp * slab + j * pitch + ip]));
        const double myz = 0.25 * (((double)M[q] + (double)M[q_jp]) +
                                   ((double)M[q_kp] + (double)M[kp * slab + jp * pitch + i]));
        double es = (sxy * sxy) / mxy + (sxz * sxz) / mxz;
        es = es + (syz * syz) / myz;
        acc += (ev + en) + es;
    }
    const double s = block_sum3(acc, red);
    if (threadIdx.x == 0)
        partial[r] = s;
}

// ------------------------------------------------------------- dispatch --

template <class S, int COMP>
static hipError_t el3d_tile(const El3dBatch &a, const El3dDesc *one, int tile,
                            hipStream_t s)
{
    const dim3 grid(a.total_tiles), block(kThreads);
    El3dOne o;
    if (one) {
        o.d = *one;
        o.parity = a.parity[0];
        o.tiles_x = a.tiles_x[0];
        o.tiles_y = a.tiles_y[0];
        o.total_tiles = a.total_tiles;
    }
    switch (tile) {
#define HW_TILE(n)                                                              \
    case n:                                                                     \
        if constexpr (kTiles3D[n].kind == 0) {                                  \
            hipLaunchKernelGGL((el3d_velocity_kernel<S, COMP, kTiles3D[n].tx,   \
                                                     kTiles3D[n].ty>),          \
                               grid, block, 0, s, a);                           \
            hipLaunchKernelGGL((el3d_stress_kernel<S, COMP, kTiles3D[n].tx,     \
                                                   kTiles3D[n].ty>),            \
                               grid, block, 0, s, a);                           \
        } else {                                                                \
            static_assert(kTiles3D[n].tx == 64, "fused tiles are 64 wide");     \
            if (one)                                                            \
                hipLaunchKernelGGL((el3d_fused1_kernel<S, COMP, kTiles3D[n].ty>), \
                                   grid, block, 0, s, o, kTiles3D[n].tz);       \
            else                                                                \
                hipLaunchKernelGGL((el3d_fused_kernel<S, COMP, kTiles3D[n].ty>), \
                                   grid, block, 0, s, a, kTiles3D[n].tz);       \
        }                                                                       \
        break;
        HW_TILE(0) HW_TILE(1) HW_TILE(2) HW_TILE(3) HW_TILE(4) HW_TILE(5) HW_TILE(6)
#undef HW_TILE
    default:
        return hipErrorInvalidValue;
    }
    static_assert(kNumTiles3D == 7, "update the tile dispatch");
    return hipGetLastError();
}

template <class S>
static hipError_t el3d_comp(const El3dBatch &a, const El3dDesc *one, int comp,
                            int tile, hipStream_t s)
{
    switch (comp) {
    case COMP_NONE: return el3d_tile<S, COMP_NONE>(a, one, tile, s);
    case COMP_FAST2SUM: return el3d_tile<S, COMP_FAST2SUM>(a, one, tile, s);
    case COMP_TWOSUM: return el3d_tile<S, COMP_TWOSUM>(a, one, tile, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_el3d_step(const El3dBatch &a, const El3dDesc *one, int storage,
                            int comp, int tile, hipStream_t s)
{
    if (a.total_tiles <= 0)
        return hipSuccess;
    switch (storage) {
    case HW_F32: return el3d_comp<F32>(a, one, comp, tile, s);
    case HW_F16: return el3d_comp<F16>(a, one, comp, tile, s);
    case HW_BF16: return el3d_comp<BF16>(a, one, comp, tile, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_el3d_energy(const El3dDesc *d_desc, int parity, int64_t rows,
                              int storage, int stride, double *partial,
                              hipStream_t s)
{
    switch (storage) {
    case HW_F32:
        hipLaunchKernelGGL(el3d_energy_kernel<F32>, dim3(rows), dim3(kThreads),
                           0, s, d_desc, parity, stride, partial);
        break;
    case HW_F16:
        hipLaunchKernelGGL(el3d_energy_kernel<F16>, dim3(rows), dim3(kThreads),
                           0, s, d_desc, parity, stride, partial);
        break;
    case HW_BF16:
        hipLaunchKernelGGL(el3d_energy_kernel<BF16>, dim3(rows), dim3(kThreads),
                           0, s, d_desc, parity, stride, partial);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hw
