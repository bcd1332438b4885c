// Step kernels of the 2D acoustic system (templates), shared by the
// translation units that instantiate them: acoustic2d.hip (the default
// kernels, energy and dispatch) and acoustic2d_var.hip (the variants with a
// point source, receivers or another stencil precision).
#pragma once

#include "hw_device.h"
#include "hw_internal.h"

#pragma clang fp contract(off)

namespace hw {


// Workgroups are dealt to the 8 XCDs round-robin; give each XCD a
// contiguous range of tiles so that tiles sharing halos share an L2.
__device__ __forceinline__ int32_t xcd_tile(int32_t b, int32_t n)
{
    return xcd_band<kNumXcd>(b, n);
}

template <class A>
__device__ __forceinline__ int find_shot(const A &a, int32_t t)
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

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// Periodic wrap of a 32-bit index (any offset).
__device__ __forceinline__ int wrapi(int i, int n)
{
    const int r = i % n;
    return r < 0 ? r + n : r;
}

// ---- vectors of V adjacent cells' words (one global access per lane)

template <int BYTES> struct RawOf;
template <> struct RawOf<2> { using type = uint16_t; };
template <> struct RawOf<4> { using type = uint32_t; };
template <> struct RawOf<8> { typedef uint32_t type __attribute__((ext_vector_type(2))); };
template <> struct RawOf<16> { typedef uint32_t type __attribute__((ext_vector_type(4))); };

template <class W, int V>
struct Cells {
    W w[V];
};

// Accesses of up to 16 bytes per lane are single instructions; wider ones
// are split into 16-byte pieces.
template <class W, int V>
__device__ __forceinline__ Cells<W, V> load_cells(const W HW_GLOBAL *p)
{
    constexpr int BYTES = V * (int)sizeof(W);
    constexpr int PIECE = BYTES < 16 ? BYTES : 16;
    using R = typename RawOf<PIECE>::type;
    R r[BYTES / PIECE];
#pragma unroll
    for (int i = 0; i < BYTES / PIECE; ++i)
        r[i] = ((const R HW_GLOBAL *)p)[i];
    Cells<W, V> c;
    __builtin_memcpy(&c, r, BYTES);
    return c;
}

// The same with non-temporal loads, for words that only one workgroup reads
// (they need not stay in L2 for a neighbouring tile's halo).
template <class W, int V>
__device__ __forceinline__ Cells<W, V> load_cells_nt(const W HW_GLOBAL *p)
{
    constexpr int BYTES = V * (int)sizeof(W);
    constexpr int PIECE = BYTES < 16 ? BYTES : 16;
    using R = typename RawOf<PIECE>::type;
    R r[BYTES / PIECE];
#pragma unroll
    for (int i = 0; i < BYTES / PIECE; ++i)
        r[i] = __builtin_nontemporal_load(((const R HW_GLOBAL *)p) + i);
    Cells<W, V> c;
    __builtin_memcpy(&c, r, BYTES);
    return c;
}

template <class W, int V>
__device__ __forceinline__ void store_cells_nt(W HW_GLOBAL *p, const Cells<W, V> &c)
{
    constexpr int BYTES = V * (int)sizeof(W);
    constexpr int PIECE = BYTES < 16 ? BYTES : 16;
    using R = typename RawOf<PIECE>::type;
    R r[BYTES / PIECE];
    __builtin_memcpy(r, &c, BYTES);
#pragma unroll
    for (int i = 0; i < BYTES / PIECE; ++i) {
        // Non-temporal stores for lane accesses of 4 bytes and more (with
        // plain stores the 32-bit word kernels lose 10%); plain stores for
        // 2-byte ones (5% faster for plain fp16, measured at 4096^2).
        if constexpr (PIECE >= 4)
            __builtin_nontemporal_store(r[i], ((R HW_GLOBAL *)p) + i);
        else
            ((R HW_GLOBAL *)p)[i] = r[i];
    }
}

// Solution updates of two independent cells (the words w0 and w1, the fp32
// increments inc0 and inc1).  For fp16 they run on packed half-precision
// instructions: two cells per instruction, each lane correctly rounded, so
// the bits equal two scalar updates (update_store); the two narrowings of
// the increments are one packed conversion, rounding to nearest even like
// the scalar one.  Other formats go one cell after the other.
template <class S, int COMP>
__device__ __forceinline__ void update_pair(typename Word<S, COMP>::type &w0,
                                            typename Word<S, COMP>::type &w1,
                                            float inc0, float inc1)
{
    using WD = Word<S, COMP>;
    if constexpr (S::id == F16::id) {
        typedef _Float16 h2 __attribute__((ext_vector_type(2)));
        typedef float f2 __attribute__((ext_vector_type(2)));
        const h2 v = {WD::v(w0), WD::v(w1)};
        f2 a = {inc0, inc1};
        if constexpr (COMP != COMP_NONE)
            a = f2{inc0 + (float)WD::c(w0), inc1 + (float)WD::c(w1)};
        __asm__("" : "+v"(a));        // no fusing into the narrowing (see opaque)
        const h2 y = __builtin_convertvector(a, h2);
        const h2 s = v + y;
        if constexpr (COMP == COMP_NONE) {
            w0 = WD::make(s[0], _Float16(0));
            w1 = WD::make(s[1], _Float16(0));
        } else {
            h2 t;
            if constexpr (COMP == COMP_FAST2SUM) {
                const h2 z = s - v;
                t = y - z;
            } else {
                const h2 pa = s - y;
                const h2 pb = s - pa;
                const h2 da = v - pa;
                const h2 db = y - pb;
                t = da + db;
            }
            w0 = WD::make(s[0], t[0]);
            w1 = WD::make(s[1], t[1]);
        }
    } else {
        auto v0 = WD::v(w0), c0 = WD::c(w0), v1 = WD::v(w1), c1 = WD::c(w1);
        update_store<S, COMP>(v0, c0, inc0);
        update_store<S, COMP>(v1, c1, inc1);
        w0 = WD::make(v0, c0);
        w1 = WD::make(v1, c1);
    }
}

// Solution update of V adjacent cells: pairs of cells through update_pair
// (packed for fp16), a last odd cell alone.
template <class S, int COMP, int V>
__device__ __forceinline__ void update_cells(Cells<typename Word<S, COMP>::type, V> &c,
                                             const float (&inc)[V])
{
    using WD = Word<S, COMP>;
#pragma unroll
    for (int i = 0; i + 1 < V; i += 2)
        update_pair<S, COMP>(c.w[i], c.w[i + 1], inc[i], inc[i + 1]);
    if constexpr (V % 2 == 1) {
        auto v = WD::v(c.w[V - 1]), cc = WD::c(c.w[V - 1]);
        update_store<S, COMP>(v, cc, inc[V - 1]);
        c.w[V - 1] = WD::make(v, cc);
    }
}

template <class S, int COMP>
__device__ __forceinline__ void update_one(typename Word<S, COMP>::type &w, float inc)
{
    using WD = Word<S, COMP>;
    auto v = WD::v(w), c = WD::c(w);
    update_store<S, COMP>(v, c, inc);
    w = WD::make(v, c);
}

// Updates of V cells whose compensation terms are 8-bit words q (held next
// to the values, see update_store8); fp16 cells in pairs on packed
// instructions (update_pair8_f16), a last odd cell alone.
template <class S, int V>
__device__ __forceinline__ void update_cells8(Cells<typename S::store_t, V> &c,
                                              int8_t (&q)[V], const float (&inc)[V])
{
    constexpr int NP = S::id == F16::id ? V / 2 : 0;
    if constexpr (NP > 0) {
#pragma unroll
        for (int i = 0; i < NP; ++i)
            update_pair8_f16(c.w[2 * i], q[2 * i], c.w[2 * i + 1], q[2 * i + 1], inc[2 * i],
                             inc[2 * i + 1]);
    }
#pragma unroll
    for (int i = 2 * NP; i < V; ++i)
        update_store8<S>(c.w[i], q[i], inc[i]);
}

template <class S, int V>
__device__ __forceinline__ void update_cells8(Cells<typename S::store_t, V> &c,
                                              int8_t (&q)[V], const double (&inc)[V])
{
#pragma unroll
    for (int i = 0; i < V; ++i)
        update_store8_d<S>(c.w[i], q[i], inc[i]);
}

// Arithmetic of the stencil (the spatial differences, the staggered
// material and the scaling; the solution update is always in the storage
// format).  SP 0: fp32, the library's default.  SP 1: every operation in
// the storage format, with weights and material rounded to it first -- the
// all-fp16 step of Alg. 1 read literally.  SP 2: fp64 from the stored values
// and the fp32 weights and material -- the promoted stencil of App. B.
template <class S, int SP> struct Sten;
template <class S> struct Sten<S, 0> {
    using T = float;
    __device__ __forceinline__ static T m(float x) { return x; }   // coefficient
    __device__ __forceinline__ static T r(T x) { return x; }       // op result
};
template <class S> struct Sten<S, 1> {
    using T = float;
    __device__ __forceinline__ static T m(float x) { return S::rn(x); }
    __device__ __forceinline__ static T r(T x) { return S::rn(x); }
};
template <class S> struct Sten<S, 2> {
    using T = double;
    __device__ __forceinline__ static T m(float x) { return (double)x; }
    __device__ __forceinline__ static T r(T x) { return x; }
};

// Updates of V cells with an fp64 increment (stencil in fp64).
template <class S, int COMP, int V>
__device__ __forceinline__ void update_cells(Cells<typename Word<S, COMP>::type, V> &c,
                                             const double (&inc)[V])
{
    using WD = Word<S, COMP>;
#pragma unroll
    for (int i = 0; i < V; ++i) {
        auto v = WD::v(c.w[i]), cc = WD::c(c.w[i]);
        update_store_d<S, COMP>(v, cc, inc[i]);
        c.w[i] = WD::make(v, cc);
    }
}

template <class S, int COMP>
__device__ __forceinline__ void update_one(typename Word<S, COMP>::type &w, double inc)
{
    using WD = Word<S, COMP>;
    auto v = WD::v(w), c = WD::c(w);
    update_store_d<S, COMP>(v, c, inc);
    w = WD::make(v, c);
}

// Point source and receivers of one plan in the current step, or `ahead`
// steps after it (Sec. 3: the s_p term of Eq. 1, and the receivers' time
// histories).  The plan's device step counter tells which sample and which
// trace row the step uses; it is read only when the plan has a source or
// receivers.
struct Forcing {
    bool src;        // the source is active in this step
    float s;         // its sample (fp32)
    int sx, sy;      // source cell
    int rn;          // receivers recorded in this step (0: none)
    int64_t row;     // their trace row
};

__device__ __forceinline__ Forcing forcing(const Ac2dDesc &d, int ahead = 0)
{
    Forcing f{false, 0.0f, d.src_x, d.src_y, 0, 0};
    if (d.src_n > 0 || d.rec_n > 0) {
        const int64_t n = *gmem(d.step) + ahead;
        if (n < d.src_n) {
            f.src = true;
            f.s = gmem(d.src)[n];
        }
        if (d.rec_n > 0 && n < d.rec_rows) {
            f.rn = d.rec_n;
            f.row = n;
        }
    }
    return f;
}

// Record component c (0 p, 1 vx, 2 vy) of cell (x, y) if it is a receiver;
// values are unscaled and widened to fp64 exactly.
__device__ __forceinline__ void record(const Ac2dDesc &d, const Forcing &f, int c,
                                       int x, int y, float v)
{
    const int32_t HW_GLOBAL *xy = gmem(d.rec_xy);
    for (int r = 0; r < f.rn; ++r)
        if (xy[2 * r] == x && xy[2 * r + 1] == y)
            gmem(d.rec)[(f.row * f.rn + r) * 3 + c] = (double)v * d.rec_scale;
}

// A workgroup of NW wavefronts (4 or 8) owns a tile of TX = 64*V by TY
// cells.  Each wavefront handles whole tile rows (row r goes to wavefront
// r mod NW) and
// each lane V adjacent cells of a row, so every field of a lane's cells is
// one global access; the few halo columns of a row are handled by the first
// lanes.  Rows are enumerated from a multiple of 4 below the halo so that a
// row keeps the same wavefront and register slot in every region (a cell's
// old pressure word, loaded with the pressure tile, is still in registers
// when its update runs).
template <class S, int COMP, int ORDER, int V, int TY, bool WX, bool FRC, int SP, int NW>
__device__ __forceinline__ void ac2d_tile(const Ac2dDesc &d, int par, int x0,
                                          int y0, bool yin, float *ps, float *bs,
                                          float *vxs, float *vys)
{
    // With 8-bit compensation words the value arrays hold values only (the
    // words of a plain state) and the compensation bytes sit comp_off bytes
    // after each value array.
    constexpr bool C8 = COMP == COMP_TWOSUM8;
    using WD = Word<S, C8 ? COMP_NONE : COMP>;
    using W = typename WD::type;
    using CV = Cells<W, V>;
    constexpr int TX = 64 * V;
    constexpr int R = ORDER / 2;              // velocity halo
    constexpr int H = 2 * R - 1;              // pressure halo
    constexpr int PW = TX + 2 * H;
    constexpr int BW = TX + 2 * R;
    constexpr int VXW = TX + 2 * R - 1;       // vx columns [-R, TX+R-1)
    constexpr int OP = NW * cdiv(H, NW);        // first pressure row is -OP
    constexpr int OB = NW * cdiv(R, NW);        // first buoyancy / vy row is -OB
    constexpr int KP = cdiv(TY + H + OP, NW);  // pressure rows [-H, TY+H)
    constexpr int KB = cdiv(TY + R + OB, NW);  // buoyancy rows [-R, TY+R)
    constexpr int KY = cdiv(TY + R - 1 + OB, NW);   // vy rows [-R, TY+R-1)
    constexpr int KC = TY / NW;                // the tile's own rows
    static_assert(TY % NW == 0, "tile height must be a multiple of the wavefront count");
    // the wavefront index in a scalar register: row tests become scalar
    // branches and row offsets scalar arithmetic
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __builtin_assume(wv >= 0 && wv < NW);    // (the range the copy hides)
    const int ln = threadIdx.x & 63;
    const int nx = (int)d.nx, ny = (int)d.ny, pitch = (int)d.pitch;
    using A = Sten<S, SP>;
    using AT = typename A::T;
    const AT w1 = A::m(d.w1), w2 = A::m(d.w2);
    const float HW_GLOBAL *__restrict__ b = gmem(d.b);
    const float HW_GLOBAL *__restrict__ kap = gmem(d.k);
    const W HW_GLOBAL *__restrict__ p_in = gmem((const W *)d.p[par]);
    const W HW_GLOBAL *__restrict__ vx_in = gmem((const W *)d.vx[par]);
    const W HW_GLOBAL *__restrict__ vy_in = gmem((const W *)d.vy[par]);
    W HW_GLOBAL *__restrict__ p_out = gmem((W *)d.p[par ^ 1]);
    W HW_GLOBAL *__restrict__ vx_out = gmem((W *)d.vx[par ^ 1]);
    W HW_GLOBAL *__restrict__ vy_out = gmem((W *)d.vy[par ^ 1]);
    using QP = const uint8_t HW_GLOBAL *;
    using QO = uint8_t HW_GLOBAL *;
    QP qp_in = gmem((const uint8_t *)d.p[par] + d.comp_off);
    QP qx_in = gmem((const uint8_t *)d.vx[par] + d.comp_off);
    QP qy_in = gmem((const uint8_t *)d.vy[par] + d.comp_off);
    QO qp_out = gmem((uint8_t *)d.p[par ^ 1] + d.comp_off);
    QO qx_out = gmem((uint8_t *)d.vx[par ^ 1] + d.comp_off);
    QO qy_out = gmem((uint8_t *)d.vy[par ^ 1] + d.comp_off);
    const int xl = V * ln;                    // first tile column of the lane
    // point source and receivers: compiled in only for plans that have them
    const Forcing fc = FRC ? forcing(d) : Forcing{false, 0.0f, 0, 0, 0, 0};
    auto grow = [&](int ly) { const int g = y0 + ly; return yin ? g : wrapi(g, ny); };
    auto gcol = [&](int lx) { const int g = x0 + lx; return WX ? wrapi(g, nx) : g; };
    // V adjacent words of one row starting at tile column xl
    auto ldw = [&](const W HW_GLOBAL *base, int row) {
        if constexpr (!WX) {
            return load_cells<W, V>(base + row + x0 + xl);
        } else {
            CV c;
#pragma unroll
            for (int i = 0; i < V; ++i)
                c.w[i] = base[row + gcol(xl + i)];
            return c;
        }
    };
    // words only this workgroup reads: non-temporal loads
    auto ldw_nt = [&](const W HW_GLOBAL *base, int row) {
        if constexpr (!WX) {
            return load_cells_nt<W, V>(base + row + x0 + xl);
        } else {
            return ldw(base, row);
        }
    };
    // 8-bit compensation words of the lane's V cells of one row
    auto ldq = [&](QP base, int row, int8_t (&out)[V]) {
#pragma unroll
        for (int c = 0; c < V; ++c)
            out[c] = (int8_t)base[row + (WX ? gcol(xl + c) : x0 + xl + c)];
    };
    auto stq = [&](QO base, int row, const int8_t (&q)[V]) {
#pragma unroll
        for (int c = 0; c < V; ++c)
            if (!WX || x0 + xl + c < nx)
                __builtin_nontemporal_store((uint8_t)q[c], base + row + x0 + xl + c);
    };
    auto upd = [&](CV &cells, int8_t (&q)[V], const auto &inc) {
        if constexpr (C8)
            update_cells8<S, V>(cells, q, inc);
        else
            update_cells<S, COMP, V>(cells, inc);
    };
    // Halo columns: the cells of a region left and right of the tile, all
    // rows together, enumerated e = 0 .. NH-1 and handled one per thread,
    // so a whole region's halo costs one instruction per wavefront.  Element
    // e is row e / (nl+nr), column nl+nr cells wide: tile column c - nl for
    // c < nl, else TX + c - nl (c = e mod (nl+nr)).
    struct Halo {
        int ly, lx;
    };
    auto halo = [&](int e, int first_row, int nl, int nr) {
        const int w = nl + nr;
        const int c = e % w;
        return Halo{first_row + e / w, c < nl ? c - nl : TX + c - nl};
    };
    constexpr int NHP = 2 * H * (TY + 2 * H);      // pressure halo cells
    constexpr int NHB = 2 * R * (TY + 2 * R);      // buoyancy halo cells
    constexpr int NHX = (2 * R - 1) * TY;          // velocity (vx) halo cells
    static_assert(NHP <= kThreads && NHB <= kThreads && NHX <= kThreads,
                  "halo lists must fit one pass of the workgroup");
    const int tid = threadIdx.x;
    const Halo hp = halo(tid, -H, H, H);
    const Halo hb = halo(tid, -R, R, R);
    const Halo hx = halo(tid, 0, R, R - 1);

    // ---- 1. issue every global load of the tile
    CV pw[KP];
    float ph = 0.0f, bh = 0.0f;
    float bm[KB][V];
    CV vxw[KC];
    W vxh;
    CV vyw[KY];
    float km[KC][V];
    int8_t qx[KC][V], qy[KY][V], qpp[KC][V], qxh = 0;   // 8-bit words
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int ly = -OP + wv + NW * k;
        if (ly >= -H && ly < TY + H)
            pw[k] = ldw(p_in, grow(ly) * pitch);
    }
    if (tid < NHP)
        ph = S::load(WD::v(p_in[grow(hp.ly) * pitch + gcol(hp.lx)]));
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int ly = -OB + wv + NW * k;
        if (ly >= -R && ly < TY + R) {
            const int row = grow(ly) * pitch;
            if constexpr (!WX) {
                const float HW_GLOBAL *q = b + row + x0 + xl;
#pragma unroll
                for (int i = 0; i < V; ++i)
                    bm[k][i] = q[i];
            } else {
#pragma unroll
                for (int i = 0; i < V; ++i)
                    bm[k][i] = b[row + gcol(xl + i)];
            }
        }
    }
    if (tid < NHB)
        bh = b[grow(hb.ly) * pitch + gcol(hb.lx)];
    if (tid < NHX && y0 + hx.ly < ny) {
        vxh = vx_in[(y0 + hx.ly) * pitch + gcol(hx.lx)];
        if constexpr (C8)
            qxh = (int8_t)qx_in[(y0 + hx.ly) * pitch + gcol(hx.lx)];
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int ly = wv + NW * k;
        if (y0 + ly < ny) {
            const int row = (y0 + ly) * pitch;
            vxw[k] = ldw_nt(vx_in, row);
            if constexpr (C8) {
                ldq(qx_in, row, qx[k]);
                ldq(qp_in, row, qpp[k]);
            }
            if constexpr (!WX) {
                const float HW_GLOBAL *q = kap + row + x0 + xl;
#pragma unroll
                for (int i = 0; i < V; ++i)
                    km[k][i] = __builtin_nontemporal_load(q + i);
            } else {
#pragma unroll
                for (int i = 0; i < V; ++i)
                    km[k][i] = kap[row + gcol(xl + i)];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KY; ++k) {
        const int ly = -OB + wv + NW * k;
        if (ly >= -R && ly < TY + R - 1) {
            vyw[k] = ldw(vy_in, grow(ly) * pitch);
            if constexpr (C8)
                ldq(qy_in, grow(ly) * pitch, qy[k]);
        }
    }

    // ---- 2. old pressure and buoyancy to LDS
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int ly = -OP + wv + NW * k;
        if (ly >= -H && ly < TY + H) {
            float *r = ps + (ly + H) * PW + H;
#pragma unroll
            for (int i = 0; i < V; ++i)
                r[xl + i] = S::load(WD::v(pw[k].w[i]));
        }
    }
    if (tid < NHP)
        ps[(hp.ly + H) * PW + H + hp.lx] = ph;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int ly = -OB + wv + NW * k;
        if (ly >= -R && ly < TY + R) {
            float *r = bs + (ly + R) * BW + R;
#pragma unroll
            for (int i = 0; i < V; ++i)
                r[xl + i] = bm[k][i];
        }
    }
    if (tid < NHB)
        bs[(hb.ly + R) * BW + R + hb.lx] = bh;
    __syncthreads();

    // vx at tile column lx of tile row ly: d p/dx, scaled by the staggered
    // buoyancy
    auto vx_inc = [&](int ly, int lx) {
        const float *pp = ps + (ly + H) * PW + (lx + H);
        const AT a0 = A::r(AT(pp[1]) - AT(pp[0]));
        AT g;
        if constexpr (ORDER == 4) {
            const AT a1 = A::r(AT(pp[2]) - AT(pp[-1]));
            g = A::r(A::r(w1 * a0) + A::r(w2 * a1));
        } else {
            g = A::r(w1 * a0);
        }
        const float *bb = bs + (ly + R) * BW + (lx + R);
        const AT bx = A::r(AT(0.5f) * A::r(A::m(bb[0]) + A::m(bb[1])));
        return A::r(bx * g);
    };

    // ---- 3a. new vx: the lane's V cells of each own row, plus the halo
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int ly = wv + NW * k;
        if (y0 + ly < ny) {
            AT inc[V];
#pragma unroll
            for (int i = 0; i < V; ++i)
                inc[i] = vx_inc(ly, xl + i);
            upd(vxw[k], qx[k], inc);
            float *r = vxs + ly * VXW + R;
#pragma unroll
            for (int i = 0; i < V; ++i)
                r[xl + i] = S::load(WD::v(vxw[k].w[i]));
            if (fc.rn > 0) {
#pragma unroll
                for (int i = 0; i < V; ++i)
                    if (x0 + xl + i < nx)
                        record(d, fc, 1, x0 + xl + i, y0 + ly, S::load(WD::v(vxw[k].w[i])));
            }
            W HW_GLOBAL *o = vx_out + (y0 + ly) * pitch + x0 + xl;
            if (!WX || x0 + TX <= nx) {
                store_cells_nt<W, V>(o, vxw[k]);
            } else {
#pragma unroll
                for (int i = 0; i < V; ++i)
                    if (x0 + xl + i < nx)
                        __builtin_nontemporal_store(vxw[k].w[i], o + i);
            }
            if constexpr (C8)
                stq(qx_out, (y0 + ly) * pitch, qx[k]);
        }
    }
    if (tid < NHX && y0 + hx.ly < ny) {
        if constexpr (C8 && SP == 2)
            update_store8_d<S>(vxh, qxh, vx_inc(hx.ly, hx.lx));
        else if constexpr (C8)
            update_store8<S>(vxh, qxh, vx_inc(hx.ly, hx.lx));
        else
            update_one<S, COMP>(vxh, vx_inc(hx.ly, hx.lx));
        vxs[hx.ly * VXW + R + hx.lx] = S::load(WD::v(vxh));
    }

    // ---- 3b. new vy: the lane's V cells of rows [-R, TY+R-1)
#pragma unroll
    for (int k = 0; k < KY; ++k) {
        const int ly = -OB + wv + NW * k;
        if (ly >= -R && ly < TY + R - 1) {
            AT inc[V];
#pragma unroll
            for (int i = 0; i < V; ++i) {
                const float *pc = ps + (ly + H) * PW + (xl + i + H);
                const AT a0 = A::r(AT(pc[PW]) - AT(pc[0]));
                AT g;
                if constexpr (ORDER == 4) {
                    const AT a1 = A::r(AT(pc[2 * PW]) - AT(pc[-PW]));
                    g = A::r(A::r(w1 * a0) + A::r(w2 * a1));
                } else {
                    g = A::r(w1 * a0);
                }
                const float *bb = bs + (ly + R) * BW + (xl + i + R);
                const AT by = A::r(AT(0.5f) * A::r(A::m(bb[0]) + A::m(bb[BW])));
                inc[i] = A::r(by * g);
            }
            upd(vyw[k], qy[k], inc);
            float *r = vys + (ly + R) * TX;
#pragma unroll
            for (int i = 0; i < V; ++i)
                r[xl + i] = S::load(WD::v(vyw[k].w[i]));
            if (ly >= 0 && ly < TY && y0 + ly < ny) {
                if (fc.rn > 0) {
#pragma unroll
                    for (int i = 0; i < V; ++i)
                        if (x0 + xl + i < nx)
                            record(d, fc, 2, x0 + xl + i, y0 + ly, S::load(WD::v(vyw[k].w[i])));
                }
                W HW_GLOBAL *o = vy_out + (y0 + ly) * pitch + x0 + xl;
                if (!WX || x0 + TX <= nx) {
                    store_cells_nt<W, V>(o, vyw[k]);
                } else {
#pragma unroll
                    for (int i = 0; i < V; ++i)
                        if (x0 + xl + i < nx)
                            __builtin_nontemporal_store(vyw[k].w[i], o + i);
                }
                if constexpr (C8)
                    stq(qy_out, (y0 + ly) * pitch, qy[k]);
            }
        }
    }
    __syncthreads();

    // ---- 4. new pressure on the lane's cells of each own row
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int ly = wv + NW * k;
        if (y0 + ly < ny) {
            AT inc[V];
#pragma unroll
            for (int i = 0; i < V; ++i) {
                const float *vr = vxs + ly * VXW + (xl + i + R);
                const float *vc = vys + (ly + R) * TX + (xl + i);
                const AT ax0 = A::r(AT(vr[0]) - AT(vr[-1]));
                const AT ay0 = A::r(AT(vc[0]) - AT(vc[-TX]));
                AT gxv, gyv;
                if constexpr (ORDER == 4) {
                    const AT ax1 = A::r(AT(vr[1]) - AT(vr[-2]));
                    const AT ay1 = A::r(AT(vc[TX]) - AT(vc[-2 * TX]));
                    gxv = A::r(A::r(w1 * ax0) + A::r(w2 * ax1));
                    gyv = A::r(A::r(w1 * ay0) + A::r(w2 * ay1));
                } else {
                    gxv = A::r(w1 * ax0);
                    gyv = A::r(w1 * ay0);
                }
                AT dv = A::r(gxv + gyv);
                // point source: the sample joins the right-hand side
                // before the scaling by kappa
                if (fc.src && y0 + ly == fc.sy && x0 + xl + i == fc.sx)
                    dv = A::r(dv + A::m(fc.s));
                inc[i] = A::r(A::m(km[k][i]) * dv);
            }
            CV &pc = pw[k + OP / NW];          // row ly's pressure words
            upd(pc, qpp[k], inc);
            if (fc.rn > 0) {
#pragma unroll
                for (int i = 0; i < V; ++i)
                    if (x0 + xl + i < nx)
                        record(d, fc, 0, x0 + xl + i, y0 + ly, S::load(WD::v(pc.w[i])));
            }
            W HW_GLOBAL *o = p_out + (y0 + ly) * pitch + x0 + xl;
            if (!WX || x0 + TX <= nx) {
                store_cells_nt<W, V>(o, pc);
            } else {
#pragma unroll
                for (int i = 0; i < V; ++i)
                    if (x0 + xl + i < nx)
                        __builtin_nontemporal_store(pc.w[i], o + i);
            }
            if constexpr (C8)
                stq(qp_out, (y0 + ly) * pitch, qpp[k]);
        }
    }
}

// Marching variant.  A workgroup owns a strip TX = 64*V cells wide and NR
// rows tall and walks down it four rows per iteration (row y+w goes to
// wavefront w).  Old pressure and buoyancy rows enter 8-row LDS rings once
// each, new vy rows an 8-row ring, so no row is loaded twice by the strip;
// only the first two iterations reload the rows above the strip.  While an
// iteration computes, the global loads of the next one are already in
// flight (register double buffering).
//   iteration j (y = 4j):  load    p row y+2R-1+w, b row y+R+w, vy row
//                                   y+R-1+w, and for the own row y+w: vx,
//                                   kappa, old p word
//                          compute vy row y+R-1+w (from iteration -1),
//                                   vx row y+w and p row y+w (from 0)
template <class S, int COMP, int ORDER, int V, int NR, bool WX>
__device__ __forceinline__ void ac2d_march(const Ac2dDesc &d, int par, int x0,
                                           int y0, bool yin, float *lds)
{
    using WD = Word<S, COMP>;
    using W = typename WD::type;
    using CV = Cells<W, V>;
    constexpr int TX = 64 * V;
    constexpr int R = ORDER / 2, H = 2 * R - 1;
    constexpr int PS = TX + 8;                // LDS row stride, column x at 4+x
    constexpr int NIT = NR / 4;
    static_assert(NR % 4 == 0 && R <= 2, "march layout");
    float *pring = lds;                       // 8 rows of old p
    float *bring = lds + 8 * PS;              // 8 rows of 1/rho
    float *vxrow = lds + 16 * PS;             // 4 rows of new vx
    float *vyring = lds + 20 * PS;            // 8 rows of new vy, TX wide
    const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
    const int xl = V * ln;
    const int nx = (int)d.nx, ny = (int)d.ny, pitch = (int)d.pitch;
    const float w1 = d.w1, w2 = d.w2;
    const float HW_GLOBAL *__restrict__ b = gmem(d.b);
    const float HW_GLOBAL *__restrict__ kap = gmem(d.k);
    const W HW_GLOBAL *__restrict__ p_in = gmem((const W *)d.p[par]);
    const W HW_GLOBAL *__restrict__ vx_in = gmem((const W *)d.vx[par]);
    const W HW_GLOBAL *__restrict__ vy_in = gmem((const W *)d.vy[par]);
    W HW_GLOBAL *__restrict__ p_out = gmem((W *)d.p[par ^ 1]);
    W HW_GLOBAL *__restrict__ vx_out = gmem((W *)d.vx[par ^ 1]);
    W HW_GLOBAL *__restrict__ vy_out = gmem((W *)d.vy[par ^ 1]);
    auto grow = [&](int r) { const int g = y0 + r; return yin ? g : wrapi(g, ny); };
    auto gcol = [&](int lx) { const int g = x0 + lx; return WX ? wrapi(g, nx) : g; };
    auto ldw = [&](const W HW_GLOBAL *base, int row) {
        if constexpr (!WX) {
            return load_cells<W, V>(base + row + x0 + xl);
        } else {
            CV c;
#pragma unroll
            for (int i = 0; i < V; ++i)
                c.w[i] = base[row + gcol(xl + i)];
            return c;
        }
    };
    auto ldf = [&](const float HW_GLOBAL *base, int row, float (&out)[V]) {
#pragma unroll
        for (int i = 0; i < V; ++i)
            out[i] = base[row + (WX ? gcol(xl + i) : x0 + xl + i)];
    };
    auto store = [&](W HW_GLOBAL *base, int row, const CV &c) {
        W HW_GLOBAL *o = base + row + x0 + xl;
        if (!WX || x0 + TX <= nx) {
            store_cells_nt<W, V>(o, c);
        } else {
#pragma unroll
            for (int i = 0; i < V; ++i)
                if (x0 + xl + i < nx)
                    __builtin_nontemporal_store(c.w[i], o + i);
        }
    };
    // Halo columns of the four rows of an iteration, one cell per lane of a
    // single wavefront: pressure (H each side) on wavefront 1, buoyancy (R
    // each side) on wavefront 2, vx (R left, R-1 right) on wavefront 0.
    const bool hp_on = wv == 1 && ln < 8 * H;
    const int hp_r = ln / (2 * H), hp_c = ln % (2 * H);
    const int hp_x = hp_c < H ? hp_c - H : TX + hp_c - H;
    const bool hb_on = wv == 2 && ln < 8 * R;
    const int hb_r = ln / (2 * R), hb_c = ln % (2 * R);
    const int hb_x = hb_c < R ? hb_c - R : TX + hb_c - R;
    const bool hx_on = wv == 0 && ln < 4 * (2 * R - 1);
    const int hx_r = ln / (2 * R - 1), hx_c = ln % (2 * R - 1);
    const int hx_x = hx_c < R ? hx_c - R : TX + hx_c - R;

    struct In {
        CV p, vx, vy, pc;
        W vxh;
        float ph, bh, bm[V], km[V];
    };
    auto load = [&](int j, In &in) {
        const int y = 4 * j;
        in.p = ldw(p_in, grow(y + 2 * R - 1 + wv) * pitch);
        if (hp_on)
            in.ph = S::load(WD::v(p_in[grow(y + 2 * R - 1 + hp_r) * pitch + gcol(hp_x)]));
        ldf(b, grow(y + R + wv) * pitch, in.bm);
        if (hb_on)
            in.bh = b[grow(y + R + hb_r) * pitch + gcol(hb_x)];
        if (j >= -1)
            in.vy = ldw(vy_in, grow(y + R - 1 + wv) * pitch);
        if (j >= 0) {
            const int row = grow(y + wv) * pitch;
            in.vx = ldw(vx_in, row);
            in.pc = ldw(p_in, row);
            ldf(kap, row, in.km);
            if (hx_on)
                in.vxh = vx_in[grow(y + hx_r) * pitch + gcol(hx_x)];
        }
    };
    auto slot = [](int r) { return r & 7; };
    auto vx_inc = [&](int k, int lx) {
        const float *pp = pring + slot(k) * PS + 4 + lx;
        const float a0 = pp[1] - pp[0];
        float g;
        if constexpr (ORDER == 4) {
            const float a1 = pp[2] - pp[-1];
            g = w1 * a0 + w2 * a1;
        } else {
            g = w1 * a0;
        }
        const float *bb = bring + slot(k) * PS + 4 + lx;
        const float bx = 0.5f * (bb[0] + bb[1]);
        return bx * g;
    };

    In cur, nxt;
    load(-2, cur);
    for (int j = -2; j < NIT; ++j) {
        const int y = 4 * j;
        // ---- stage this iteration's old pressure and buoyancy rows
        {
            float *pr = pring + slot(y + 2 * R - 1 + wv) * PS + 4;
            float *br = bring + slot(y + R + wv) * PS + 4;
#pragma unroll
            for (int i = 0; i < V; ++i) {
                pr[xl + i] = S::load(WD::v(cur.p.w[i]));
                br[xl + i] = cur.bm[i];
            }
            if (hp_on)
                pring[slot(y + 2 * R - 1 + hp_r) * PS + 4 + hp_x] = cur.ph;
            if (hb_on)
                bring[slot(y + R + hb_r) * PS + 4 + hb_x] = cur.bh;
        }
        if (j + 1 < NIT)
            load(j + 1, nxt);
        __syncthreads();

        // ---- new vy row m = y+R-1+w and new vx row y+w
        if (j >= -1) {
            const int m = y + R - 1 + wv;
            float inc[V];
#pragma unroll
            for (int i = 0; i < V; ++i) {
                const int c = 4 + xl + i;
                const float pm = pring[slot(m) * PS + c];
                const float pn = pring[slot(m + 1) * PS + c];
                const float a0 = pn - pm;
                float g;
                if constexpr (ORDER == 4) {
                    const float a1 = pring[slot(m + 2) * PS + c] - pring[slot(m - 1) * PS + c];
                    g = w1 * a0 + w2 * a1;
                } else {
                    g = w1 * a0;
                }
                const float by = 0.5f * (bring[slot(m) * PS + c] + bring[slot(m + 1) * PS + c]);
                inc[i] = by * g;
            }
            update_cells<S, COMP, V>(cur.vy, inc);
            float *vr = vyring + slot(m) * TX;
#pragma unroll
            for (int i = 0; i < V; ++i)
                vr[xl + i] = S::load(WD::v(cur.vy.w[i]));
            if (m >= 0 && m < NR && y0 + m < ny)
                store(vy_out, (y0 + m) * pitch, cur.vy);
        }
        if (j >= 0) {
            const int k = y + wv;
            float inc[V];
#pragma unroll
            for (int i = 0; i < V; ++i)
                inc[i] = vx_inc(k, xl + i);
            update_cells<S, COMP, V>(cur.vx, inc);
            float *xr = vxrow + wv * PS + 4;
#pragma unroll
            for (int i = 0; i < V; ++i)
                xr[xl + i] = S::load(WD::v(cur.vx.w[i]));
            if (y0 + k < ny)
                store(vx_out, (y0 + k) * pitch, cur.vx);
            if (hx_on) {
                update_one<S, COMP>(cur.vxh, vx_inc(y + hx_r, hx_x));
                vxrow[hx_r * PS + 4 + hx_x] = S::load(WD::v(cur.vxh));
            }
        }
        __syncthreads();

        // ---- new pressure row y+w
        if (j >= 0) {
            const int k = y + wv;
            float inc[V];
#pragma unroll
            for (int i = 0; i < V; ++i) {
                const float *vr = vxrow + wv * PS + 4 + xl + i;
                const int c = xl + i;
                const float ax0 = vr[0] - vr[-1];
                const float ay0 = vyring[slot(k) * TX + c] - vyring[slot(k - 1) * TX + c];
                float gxv, gyv;
                if constexpr (ORDER == 4) {
                    const float ax1 = vr[1] - vr[-2];
                    const float ay1 = vyring[slot(k + 1) * TX + c] - vyring[slot(k - 2) * TX + c];
                    gxv = w1 * ax0 + w2 * ax1;
                    gyv = w1 * ay0 + w2 * ay1;
                } else {
                    gxv = w1 * ax0;
                    gyv = w1 * ay0;
                }
                const float dv = gxv + gyv;
                inc[i] = cur.km[i] * dv;
            }
            update_cells<S, COMP, V>(cur.pc, inc);
            if (y0 + k < ny)
                store(p_out, (y0 + k) * pitch, cur.pc);
        }
        cur = nxt;
    }
}

template <class S, int COMP, int ORDER, int V, int NR>
__device__ __forceinline__ void ac2d_march_entry(const Ac2dDesc &d, int par,
                                                 int tile, int ntx, float *lds)
{
    constexpr int TX = 64 * V;
    const int nx = (int)d.nx, ny = (int)d.ny;
    const int x0 = (tile % ntx) * TX;
    const int y0 = (tile / ntx) * NR;
    constexpr int H = ORDER - 1;
    // every row the strip touches lies in [y0-8, y0+NR+4)
    const bool xin = x0 >= H && x0 + TX + H <= nx;
    const bool yin = y0 >= 8 && y0 + NR + 4 <= ny;
    if (xin)
        ac2d_march<S, COMP, ORDER, V, NR, false>(d, par, x0, y0, yin, lds);
    else
        ac2d_march<S, COMP, ORDER, V, NR, true>(d, par, x0, y0, yin, lds);
}

template <class S, int COMP, int ORDER, int V, int NR>
__global__ __launch_bounds__(kThreads) void ac2d_march_kernel(const Ac2dBatch a)
{
    __shared__ float lds[20 * (64 * V + 8) + 8 * 64 * V];
    int32_t tile = xcd_tile(blockIdx.x, a.total_tiles);
    const int shot = find_shot(a, tile);
    ac2d_march_entry<S, COMP, ORDER, V, NR>(*a.desc[shot], a.parity[shot],
                                            tile - a.tile_start[shot],
                                            a.tiles_x[shot], lds);
}

// Single-plan launches carry the descriptor in the kernel arguments, so a
// workgroup's first loads do not wait on a chain of dependent scalar loads.
template <class S, int COMP, int ORDER, int V, int NR>
__global__ __launch_bounds__(kThreads) void ac2d_march1_kernel(const Ac2dOne o)
{
    __shared__ float lds[20 * (64 * V + 8) + 8 * 64 * V];
    ac2d_march_entry<S, COMP, ORDER, V, NR>(o.d, o.parity,
                                            xcd_tile(blockIdx.x, o.total_tiles),
                                            o.tiles_x, lds);
}

template <class S, int COMP, int ORDER, int V, int TY>
struct TileLds {
    static constexpr int TX = 64 * V, R = ORDER / 2, H = 2 * R - 1;
    float ps[(TY + 2 * H) * (TX + 2 * H)];   // old p
    float bs[(TY + 2 * R) * (TX + 2 * R)];   // 1/rho
    float vxs[TY * (TX + 2 * R - 1)];        // new vx
    float vys[(TY + 2 * R - 1) * TX];        // new vy
};

template <class S, int COMP, int ORDER, int V, int TY, bool FRC, int SP, int NW>
__device__ __forceinline__ void ac2d_tile_entry(const Ac2dDesc &d, int par,
                                                int tile, int ntx,
                                                TileLds<S, COMP, ORDER, V, TY> &L)
{
    constexpr int TX = 64 * V;
    constexpr int R = ORDER / 2, H = 2 * R - 1;
    const int nx = (int)d.nx, ny = (int)d.ny;
    const int x0 = (tile % ntx) * TX;
    const int y0 = (tile / ntx) * TY;
    // tiles whose halo stays inside the grid need no periodic wrapping
    const bool xin = x0 >= H && x0 + TX + H <= nx;
    const bool yin = y0 >= H && y0 + TY + H <= ny;
    if (xin)
        ac2d_tile<S, COMP, ORDER, V, TY, false, FRC, SP, NW>(d, par, x0, y0, yin, L.ps, L.bs, L.vxs, L.vys);
    else
        ac2d_tile<S, COMP, ORDER, V, TY, true, FRC, SP, NW>(d, par, x0, y0, yin, L.ps, L.bs, L.vxs, L.vys);
}

// Occupancy hint of the step kernels.  A workgroup of 8 wavefronts puts two
// on each SIMD, so occupancy steps between 6 and 8 waves per SIMD at 64
// VGPRs.  The plain fp16/bf16 updates fit in 64 VGPRs without scratch when
// asked to; the compensated and fp32 variants would spill, and keep the
// compiler's choice.
template <class S, int COMP, int NW>
constexpr int step_min_waves()
{
    return NW == 8 && COMP == COMP_NONE && S::id != F32::id ? 8 : 1;
}

template <class S, int COMP, int ORDER, int V, int TY, bool FRC = false, int SP = 0,
          int NW = 4>
__global__ __launch_bounds__(64 * NW)
__attribute__((amdgpu_waves_per_eu(step_min_waves<S, COMP, NW>())))
void ac2d_step_kernel(const Ac2dBatch a)
{
    __shared__ TileLds<S, COMP, ORDER, V, TY> L;
    int32_t tile = xcd_tile(blockIdx.x, a.total_tiles);
    const int shot = find_shot(a, tile);
    ac2d_tile_entry<S, COMP, ORDER, V, TY, FRC, SP, NW>(*a.desc[shot], a.parity[shot],
                                           tile - a.tile_start[shot],
                                           a.tiles_x[shot], L);
}

template <class S, int COMP, int ORDER, int V, int TY, bool FRC = false, int SP = 0,
          int NW = 4>
__global__ __launch_bounds__(64 * NW)
__attribute__((amdgpu_waves_per_eu(step_min_waves<S, COMP, NW>())))
void ac2d_step1_kernel(const Ac2dOne o)
{
    __shared__ TileLds<S, COMP, ORDER, V, TY> L;
    ac2d_tile_entry<S, COMP, ORDER, V, TY, FRC, SP, NW>(o.d, o.parity,
                                           xcd_tile(blockIdx.x, o.total_tiles),
                                           o.tiles_x, L);
}

}  // namespace hw
