// 2D acoustic leapfrog, two time steps per launch (temporal blocking).
//
// A workgroup owns a 64 x TY tile and advances it from the state at step n
// (v^{n-1/2}, p^n) to the state at step n+2 in one pass over HBM: every
// field word (value and compensation term) is read once and written once
// per two steps.  To do so it first advances, by one step, every cell the
// second step of its tile depends on -- the tile grown by 2R-1 cells for the
// pressure and by up to 3R-1 cells for the velocities (R = order / 2) --
// from old values read around the tile, exactly as a one-step launch would
// advance those cells.  The compensation terms of that intermediate state
// never leave the registers of the threads that own the cells, and every
// cell's operations are the op-by-op definition the one-step kernels and
// the CPU reference use, so two steps of this kernel are bit-identical to
// two one-step launches (Sec. 3 and Alg. 1/2 of Sec. 4; the update with the
// 3- or 6-operation sum of Code 1 / Code 2).
//
// Work layout: each wavefront takes whole rows of a region (row r goes to
// wavefront (r - RB) mod NW and register slot (r - RB) / NW, the same for
// every field and both steps, so a cell's word stays with one thread), each
// lane one column of the 64 tile columns; the cells of a region left and
// right of the tile columns are flattened into lists handled one per thread.
//
//   phase 1  global loads; old pressure and buoyancy values to LDS
//   phase 2  v^{n+1/2} on the grown regions              (values to LDS)
//   phase 3  p^{n+1}   on the tile grown by 2R-1          (values to LDS)
//   phase 4  v^{n+3/2} on the cells the tile's p^{n+2} needs; tile cells stored
//   phase 5  p^{n+2}   on the tile; stored
#pragma once

#include "acoustic2d_kernels.h"

#pragma clang fp contract(off)

namespace hw {

namespace tb {

// A region: rows [r0, r1) by the columns left of the tile [-cl, 0) and right
// of it [TX, TX + cr); element e of its flattened list.
struct Side {
    int r, c;
};
template <int TX, int R0, int CL, int CR>
__device__ __forceinline__ Side side(int e)
{
    constexpr int W = CL + CR;
    const int c = e % W;
    return Side{R0 + e / W, c < CL ? c - CL : TX + c - CL};
}

// An LDS address the compiler may not fold into the accesses made from it:
// a stencil's reads then share one base register with small immediate
// offsets (two paired reads from one add) instead of one add per pair.
typedef __attribute__((address_space(3))) const float lds_f;
__device__ __forceinline__ const lds_f *lds_base(const float *p)
{
    const lds_f *q = (const lds_f *)p;
    __asm__("" : "+v"(q));
    return q;
}

// A pointer that is the same in every lane, read into scalar registers
// (the row bases of the interior tiles' loads; the compiler cannot always
// see that they are uniform, for instance when the descriptor comes from a
// batch table indexed at run time).
template <class T>
__device__ __forceinline__ const T HW_GLOBAL *scalar(const T HW_GLOBAL *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const T HW_GLOBAL *)(((uint64_t)hi << 32) | lo);
}

// A compile-time slot bound passed to a generic lambda.
template <int N> struct IC {
    static constexpr int value = N;
};

}  // namespace tb

template <int ORDER, int TY>
struct Tb2Geom {
    static constexpr int TX = 64;
    static constexpr int R = ORDER / 2;          // reach of one derivative
    static constexpr int H = 2 * R - 1;          // reach of one step on p
    static constexpr int G = H + R;              // reach of one step on v
    // LDS arrays and the origin (row, column) of their element 0
    static constexpr int PW = TX + 4 * H, PR = TY + 4 * H;         // p values
    static constexpr int BW = TX + 2 * G, BR = TY + 2 * G;         // buoyancy
    static constexpr int XW = TX + H + G + R - 1, XR = TY + 2 * H; // vx values
    static constexpr int YW = TX + 2 * H, YR = TY + H + G + R - 1; // vy values
};

template <int ORDER, int TY>
struct Tb2Lds {
    using Gm = Tb2Geom<ORDER, TY>;
    float ps[Gm::PR * Gm::PW];
    float bs[Gm::BR * Gm::BW];
    float xs[Gm::XR * Gm::XW];
    float ys[Gm::YR * Gm::YW];
};

// EDGE: the tile lies within 2H cells of a grid edge (or the grid is
// narrower than the tile): rows and columns wrap around the periodic grid and
// stores skip cells past its end.  Interior tiles take neither step.
// FRC: the plan may have a point source or receivers (Sec. 3): the source
// sample of each step joins the pressure right-hand side at its cell --
// in the intermediate step wherever that cell lies in the grown region, so
// the recomputed cells match their owners' -- and the tile's own cells
// record the receivers' values of both steps.
template <class S, int COMP, int ORDER, int TY, int NW, bool EDGE, bool FRC>
__device__ __forceinline__ void ac2d_tile2(const Ac2dDesc &d, int par, int x0, int y0,
                                           Tb2Lds<ORDER, TY> &L)
{
    using Gm = Tb2Geom<ORDER, TY>;
    // With 8-bit compensation words the value arrays hold values only and
    // each cell's word is a byte comp_off bytes after its value array.
    constexpr bool C8 = COMP == COMP_TWOSUM8;
    using WD = Word<S, C8 ? COMP_NONE : COMP>;
    using W = typename WD::type;
    constexpr int TX = Gm::TX, R = Gm::R, H = Gm::H, G = Gm::G;
    constexpr int PW = Gm::PW, BW = Gm::BW, XW = Gm::XW, YW = Gm::YW;
    constexpr int NT = 64 * NW;
    static_assert(TY % NW == 0, "tile height must be a multiple of the wavefronts");
    // the wavefront index is the same in every lane: kept in a scalar
    // register, the row tests below are scalar branches and the row parts of
    // addresses scalar offsets
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // (its range, which the scalar copy hides from the compiler: the slots
    // whose rows lie inside a phase's region for every wavefront then need
    // no test at all)
    __builtin_assume(wv >= 0 && wv < NW);
    const int ln = threadIdx.x & 63, tid = threadIdx.x;
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
    using QP = const int8_t HW_GLOBAL *;
    using QO = int8_t HW_GLOBAL *;
    QP qp_in = gmem((const int8_t *)((const char *)d.p[par] + d.comp_off));
    QP qx_in = gmem((const int8_t *)((const char *)d.vx[par] + d.comp_off));
    QP qy_in = gmem((const int8_t *)((const char *)d.vy[par] + d.comp_off));
    QO qp_out = gmem((int8_t *)((char *)d.p[par ^ 1] + d.comp_off));
    QO qx_out = gmem((int8_t *)((char *)d.vx[par ^ 1] + d.comp_off));
    QO qy_out = gmem((int8_t *)((char *)d.vy[par ^ 1] + d.comp_off));
    auto grow = [&](int r) { const int g = y0 + r; return EDGE ? wrapi(g, ny) : g; };
    auto gcol = [&](int c) { const int g = x0 + c; return EDGE ? wrapi(g, nx) : g; };
    // LDS element of tile-relative (row, column) in each array
    auto P = [&](int r, int c) { return L.ps + (r + 2 * H) * PW + (c + 2 * H); };
    auto B = [&](int r, int c) { return L.bs + (r + G) * BW + (c + G); };
    auto X = [&](int r, int c) { return L.xs + (r + H) * XW + (c + G); };
    auto Y = [&](int r, int c) { return L.ys + (r + G) * YW + (c + H); };
    // this lane's grid column (unsigned: a row pointer in scalar registers
    // plus a 32-bit lane offset is one addressing mode)
    const unsigned col = (unsigned)gcol(ln);
    // the element of tile row r in this lane's column of array a: in interior
    // tiles the row and the tile's first column make a base in scalar
    // registers (read there explicitly: otherwise the compiler folds the lane
    // into a 64-bit vector base and adds each row to it) and the lane is the
    // load's offset, so no load needs vector address arithmetic
    auto row_at = [&](auto a, int r) {
        if constexpr (EDGE) {
            return (a + grow(r) * pitch)[col];
        } else {
            return tb::scalar(a + ((y0 + r) * pitch + x0))[(unsigned)ln];
        }
    };
    // point source and receivers of step n (first) and n+1 (second step)
    const Forcing f0 = FRC ? forcing(d, 0) : Forcing{false, 0.0f, 0, 0, 0, 0};
    const Forcing f1 = FRC ? forcing(d, 1) : Forcing{false, 0.0f, 0, 0, 0, 0};
    // whether grid cell (gx, gy) is the source cell of a step that has one
    auto src_at = [&](const Forcing &f, int gx, int gy) {
        return FRC && f.src && gx == f.sx && gy == f.sy;
    };
    // record a value of the tile's own cell (row r, this lane's column) if it
    // is a receiver (component c: 0 p, 1 vx, 2 vy)
    auto rec = [&](const Forcing &f, int c, int r, float v) {
        if constexpr (FRC)
            if (f.rn > 0 && r >= 0 && r < TY && y0 + r < ny && x0 + ln < nx)
                record(d, f, c, x0 + ln, y0 + r, v);
    };

    // Row r belongs to wavefront (r - RB) mod NW and register slot
    // (r - RB) / NW; a region of rows [lo, hi) uses slots [lo', hi') below.
    constexpr int RB = -NW * cdiv(2 * H, NW);
    auto row_of = [&](int k) { return RB + wv + NW * k; };
    // this lane's element of the first row of this wavefront in each LDS
    // array: the row part's accesses are fixed offsets from these
    float *const Pl = P(RB + wv, ln), *const Bl = B(RB + wv, ln);
    float *const Xl = X(RB + wv, ln), *const Yl = Y(RB + wv, ln);
    constexpr int P0 = (-2 * H - RB) / NW, P1 = cdiv(TY + 2 * H - RB, NW);    // old p
    constexpr int Q0 = (-H - RB) / NW, Q1 = cdiv(TY + H - RB, NW);            // p, kappa, vx
    constexpr int B0 = (-G - RB) / NW, B1 = cdiv(TY + G - RB, NW);            // buoyancy
    constexpr int V0 = (-G - RB) / NW, V1 = cdiv(TY + H + R - 1 - RB, NW);    // vy
    static_assert(P0 >= 0 && P0 <= Q0 && Q1 <= P1, "slot ranges");

    // Flattened lists of cells left and right of the tile columns (one
    // element per thread, the first three kept in registers):
    //   XH  vx^{n+1/2}: rows [-H, TY+H), columns [-G, 0) and [TX, TX+G-1)
    //   YH  vy^{n+1/2}: rows [-G, TY+H+R-1), columns [-H, 0) and [TX, TX+H)
    //   QH  p^{n+1} and kappa: rows [-H, TY+H), columns [-H, 0) and [TX, TX+H)
    //   PA  old p: rows [-H, TY+H), columns [-2H, -H) and [TX+H, TX+2H)
    //   PB  old p: rows [-2H, -H) and [TY+H, TY+2H), columns as QH
    //   BA  buoyancy: rows [-H, TY+H), columns [-G, 0) and [TX, TX+G)
    //   BB  buoyancy: rows [-G, -H) and [TY+H, TY+G), columns as QH
    constexpr int NXH = (2 * G - 1) * (TY + 2 * H);
    constexpr int NYH = 2 * H * (TY + H + G + R - 1);
    constexpr int NQH = 2 * H * (TY + 2 * H);
    constexpr int NPA = 2 * H * (TY + 2 * H), NPB = 2 * H * 2 * H;
    constexpr int NBA = 2 * G * (TY + 2 * H), NBB = 2 * H * 2 * R;
    static_assert(NXH <= NT && NYH <= NT && NQH <= NT,
                  "the lists of kept words must fit one pass of the workgroup");
    const tb::Side xh = tb::side<TX, -H, G, G - 1>(tid);
    const tb::Side yh = tb::side<TX, -G, H, H>(tid);
    const tb::Side qh = tb::side<TX, -H, H, H>(tid);
    const bool xh_on = tid < NXH, yh_on = tid < NYH, qh_on = tid < NQH;

    // ---- phase 1: every global load; old pressure and buoyancy to LDS
    W pw[P1 - P0], xw[Q1 - Q0], yw[V1 - V0];
    float km[Q1 - Q0], bm[B1 - B0];
    W xhw = W(), yhw = W(), qhw = W();
    float qhk = 0.0f;
    // 8-bit words of the kept cells (unused otherwise)
    int8_t qpw[Q1 - Q0], qxw[Q1 - Q0], qyw[V1 - V0], qxh = 0, qyh = 0, qqh = 0;
#pragma unroll
    for (int k = P0; k < P1; ++k) {
        const int r = row_of(k);
        if (r >= -2 * H && r < TY + 2 * H)
            pw[k - P0] = row_at(p_in, r);
    }
#pragma unroll
    for (int k = B0; k < B1; ++k) {
        const int r = row_of(k);
        if (r >= -G && r < TY + G)
            bm[k - B0] = row_at(b, r);
    }
#pragma unroll
    for (int k = Q0; k < Q1; ++k) {
        const int r = row_of(k);
        if (r >= -H && r < TY + H) {
            xw[k - Q0] = row_at(vx_in, r);
            km[k - Q0] = row_at(kap, r);
            if constexpr (C8) {
                qxw[k - Q0] = row_at(qx_in, r);
                qpw[k - Q0] = row_at(qp_in, r);
            }
        }
    }
#pragma unroll
    for (int k = V0; k < V1; ++k) {
        const int r = row_of(k);
        if (r >= -G && r < TY + H + R - 1) {
            yw[k - V0] = row_at(vy_in, r);
            if constexpr (C8)
                qyw[k - V0] = row_at(qy_in, r);
        }
    }
    if (xh_on) {
        const int q = grow(xh.r) * pitch + gcol(xh.c);
        xhw = vx_in[q];
        if constexpr (C8)
            qxh = qx_in[q];
    }
    if (yh_on) {
        const int q = grow(yh.r) * pitch + gcol(yh.c);
        yhw = vy_in[q];
        if constexpr (C8)
            qyh = qy_in[q];
    }
    if (qh_on) {
        const int q = grow(qh.r) * pitch + gcol(qh.c);
        qhw = p_in[q];
        qhk = kap[q];
        if constexpr (C8)
            qqh = qp_in[q];
    }
    // the old-pressure and buoyancy frames: element e of each goes to
    // thread e mod NT; loaded here with every other load (so the tile waits
    // for memory once), written to LDS after the row values
    constexpr int NPF = NPA + NPB, NBF = NBA + NBB;
    constexpr int KP = cdiv(NPF, NT), KB = cdiv(NBF, NT);
    W pfw[KP];
    float bfv[KB];
    int pfo[KP], bfo[KB];        // their LDS elements
#pragma unroll
    for (int i = 0; i < KP; ++i) {
        const int e = tid + i * NT;
        if (e < NPF) {
            int r, c;
            if (e < NPA) {
                const tb::Side s = tb::side<TX, -H, H, H>(e);
                r = s.r;
                c = s.c < 0 ? s.c - H : s.c + H;
            } else {
                const tb::Side s = tb::side<TX, 0, H, H>(e - NPA);
                r = s.r < H ? s.r - 2 * H : TY + s.r;
                c = s.c;
            }
            pfw[i] = p_in[grow(r) * pitch + gcol(c)];
            pfo[i] = (int)(P(r, c) - L.ps);
        }
    }
#pragma unroll
    for (int i = 0; i < KB; ++i) {
        const int e = tid + i * NT;
        if (e < NBF) {
            int r, c;
            if (e < NBA) {
                const tb::Side s = tb::side<TX, -H, G, G>(e);
                r = s.r;
                c = s.c;
            } else {
                const tb::Side s = tb::side<TX, 0, H, H>(e - NBA);
                r = s.r < R ? s.r - G : TY + H + (s.r - R);
                c = s.c;
            }
            bfv[i] = b[grow(r) * pitch + gcol(c)];
            bfo[i] = (int)(B(r, c) - L.bs);
        }
    }
#pragma unroll
    for (int k = P0; k < P1; ++k) {
        const int r = row_of(k);
        if (r >= -2 * H && r < TY + 2 * H)
            Pl[NW * k * PW] = S::load(WD::v(pw[k - P0]));
    }
#pragma unroll
    for (int k = B0; k < B1; ++k) {
        const int r = row_of(k);
        if (r >= -G && r < TY + G)
            Bl[NW * k * BW] = bm[k - B0];
    }
#pragma unroll
    for (int i = 0; i < KP; ++i)
        if (tid + i * NT < NPF)
            L.ps[pfo[i]] = S::load(WD::v(pfw[i]));
#pragma unroll
    for (int i = 0; i < KB; ++i)
        if (tid + i * NT < NBF)
            L.bs[bfo[i]] = bfv[i];
    if (qh_on)
        *P(qh.r, qh.c) = S::load(WD::v(qhw));
    __syncthreads();

    // increments of the three updates from the LDS values, in the op order
    // of the one-step kernels
    // (each stencil reads from a base at its lowest address: x offsets
    // -1 .. 2 (vx), rows -1 .. 2 (vy), -2 .. 1 (p); order 2 uses 0 .. 1)
    constexpr int LX = R - 1, LY = (R - 1) * PW;
    // (the staggered buoyancy of a velocity cell is the same in both steps:
    // the first step's value is kept in a register for the second)
    auto vx_g = [&](const float *pp) {
        const tb::lds_f *q = tb::lds_base(pp - LX);
        const float a0 = q[LX + 1] - q[LX];
        if constexpr (ORDER == 4) {
            const float a1 = q[LX + 2] - q[LX - 1];
            return w1 * a0 + w2 * a1;
        } else {
            return w1 * a0;
        }
    };
    auto bx_at = [&](const float *bb) {
        const tb::lds_f *c = tb::lds_base(bb);
        return 0.5f * (c[0] + c[1]);
    };
    auto vy_g = [&](const float *pc) {
        const tb::lds_f *q = tb::lds_base(pc - LY);
        const float a0 = q[LY + PW] - q[LY];
        if constexpr (ORDER == 4) {
            const float a1 = q[LY + 2 * PW] - q[LY - PW];
            return w1 * a0 + w2 * a1;
        } else {
            return w1 * a0;
        }
    };
    auto by_at = [&](const float *bb) {
        const tb::lds_f *c = tb::lds_base(bb);
        return 0.5f * (c[0] + c[BW]);
    };
    // the pressure increment; with `src` (the cell is the source cell of the
    // step) the sample s joins the right-hand side before the scaling
    auto p_at = [&](const float *vr0, const float *vc0, float kk, bool src, float s) {
        const tb::lds_f *vr = tb::lds_base(vr0 - R), *vc = tb::lds_base(vc0 - R * YW);
        const float ax0 = vr[R] - vr[R - 1];
        const float ay0 = vc[R * YW] - vc[(R - 1) * YW];
        float gxv, gyv;
        if constexpr (ORDER == 4) {
            const float ax1 = vr[R + 1] - vr[R - 2];
            const float ay1 = vc[(R + 1) * YW] - vc[(R - 2) * YW];
            gxv = w1 * ax0 + w2 * ax1;
            gyv = w1 * ay0 + w2 * ay1;
        } else {
            gxv = w1 * ax0;
            gyv = w1 * ay0;
        }
        float dv = gxv + gyv;
        if constexpr (FRC)
            if (src)
                dv = dv + s;
        return kk * dv;
    };
    auto p_inc = [&](int r, int c, float kk) {
        return p_at(X(r, c), Y(r, c), kk, src_at(f0, gcol(c), grow(r)), f0.s);
    };
    // the update of Alg. 1/2 on a kept word (and its 8-bit word)
    auto upd = [&](W &w, int8_t &q, float inc) {
        if constexpr (C8)
            update_store8<S>(w, q, inc);
        else
            update_one<S, COMP>(w, inc);
    };
    // Visits the register slots [K0, K1) whose rows pass on(k).  For fp16
    // words, where two neighbouring slots both do, their increments are
    // computed first and the two words updated together on packed
    // instructions (update_pair, update_pair8_f16: the same bits as two
    // single updates); otherwise slot by slot.  fin(k) follows each slot's
    // update.
    constexpr bool PAIR = S::id == F16::id;
    auto walk = [&](auto k0c, auto k1c, auto on, auto inc, auto wd, auto qb, auto fin) {
        constexpr int K0 = decltype(k0c)::value, K1 = decltype(k1c)::value;
        if constexpr (PAIR) {
#pragma unroll
            for (int k = K0; k < K1; k += 2) {
                const int k1 = k + 1 < K1 ? k + 1 : k;
                const bool a = on(k), b = k + 1 < K1 && on(k1);
                if (a && b) {
                    const float i0 = inc(k), i1 = inc(k1);
                    if constexpr (C8)
                        update_pair8_f16(wd(k), qb(k), wd(k1), qb(k1), i0, i1);
                    else
                        update_pair<S, COMP>(wd(k), wd(k1), i0, i1);
                    fin(k);
                    fin(k1);
                } else {
                    if (a) {
                        upd(wd(k), qb(k), inc(k));
                        fin(k);
                    }
                    if (b) {
                        upd(wd(k1), qb(k1), inc(k1));
                        fin(k1);
                    }
                }
            }
        } else {
#pragma unroll
            for (int k = K0; k < K1; ++k)
                if (on(k)) {
                    upd(wd(k), qb(k), inc(k));
                    fin(k);
                }
        }
    };
    using IQ0 = tb::IC<Q0>;
    using IQ1 = tb::IC<Q1>;
    using IV0 = tb::IC<V0>;
    using IV1 = tb::IC<V1>;
    auto store8 = [&](QO base, int r, int8_t q) {
        if constexpr (C8)
            if (!EDGE || (y0 + r < ny && x0 + ln < nx))
                __builtin_nontemporal_store(q, (base + (y0 + r) * pitch + x0) + (unsigned)ln);
    };
    auto store = [&](W HW_GLOBAL *base, int r, const W &w) {
        if (!EDGE || (y0 + r < ny && x0 + ln < nx))
            __builtin_nontemporal_store(w, (base + (y0 + r) * pitch + x0) + (unsigned)ln);
    };

    // ---- phase 2: v^{n+1/2} on the grown regions
    float bxk[Q1 - Q0], byk[V1 - V0], bxh = 0.0f;
    auto xwd = [&](int k) -> W & { return xw[k - Q0]; };
    auto xqb = [&](int k) -> int8_t & { return qxw[k - Q0]; };
    auto ywd = [&](int k) -> W & { return yw[k - V0]; };
    auto yqb = [&](int k) -> int8_t & { return qyw[k - V0]; };
    auto pwd = [&](int k) -> W & { return pw[k - P0]; };
    auto pqb = [&](int k) -> int8_t & { return qpw[k - Q0]; };
    auto xlds = [&](int k) { Xl[NW * k * XW] = S::load(WD::v(xw[k - Q0])); };
    auto ylds = [&](int k) { Yl[NW * k * YW] = S::load(WD::v(yw[k - V0])); };
    // the same, and a receiver's record of the step (rows of the tile only)
    auto xlds_rec = [&](const Forcing &f, int k) {
        xlds(k);
        rec(f, 1, row_of(k), S::load(WD::v(xw[k - Q0])));
    };
    auto ylds_rec = [&](const Forcing &f, int k) {
        ylds(k);
        rec(f, 2, row_of(k), S::load(WD::v(yw[k - V0])));
    };
    auto vx_slot = [&](int k) { return bxk[k - Q0] * vx_g(Pl + NW * k * PW); };
    auto vy_slot = [&](int k) { return byk[k - V0] * vy_g(Pl + NW * k * PW); };
    // the pressure increment of slot k in the step of forcing f
    auto p_slot = [&](const Forcing &f, int k) {
        return p_at(Xl + NW * k * XW, Yl + NW * k * YW, km[k - Q0],
                    src_at(f, (int)col, grow(row_of(k))), f.s);
    };
    walk(IQ0(), IQ1(), [&](int k) { const int r = row_of(k); return r >= -H && r < TY + H; },
         [&](int k) {
             bxk[k - Q0] = bx_at(Bl + NW * k * BW);
             return vx_slot(k);
         },
         xwd, xqb, [&](int k) { xlds_rec(f0, k); });
    walk(IV0(), IV1(),
         [&](int k) { const int r = row_of(k); return r >= -G && r < TY + H + R - 1; },
         [&](int k) {
             byk[k - V0] = by_at(Bl + NW * k * BW);
             return vy_slot(k);
         },
         ywd, yqb, [&](int k) { ylds_rec(f0, k); });
    if (xh_on) {
        bxh = bx_at(B(xh.r, xh.c));
        upd(xhw, qxh, bxh * vx_g(P(xh.r, xh.c)));
        *X(xh.r, xh.c) = S::load(WD::v(xhw));
    }
    if (yh_on) {
        upd(yhw, qyh, by_at(B(yh.r, yh.c)) * vy_g(P(yh.r, yh.c)));
        *Y(yh.r, yh.c) = S::load(WD::v(yhw));
    }
    __syncthreads();

    // ---- phase 3: p^{n+1} on the tile grown by H; its values replace the
    // old pressure values in LDS (phase 2 has finished reading them)
    walk(IQ0(), IQ1(), [&](int k) { const int r = row_of(k); return r >= -H && r < TY + H; },
         [&](int k) { return p_slot(f0, k); }, pwd, pqb,
         [&](int k) {
             Pl[NW * k * PW] = S::load(WD::v(pw[k - P0]));
             rec(f0, 0, row_of(k), S::load(WD::v(pw[k - P0])));
         });
    if (qh_on) {
        upd(qhw, qqh, p_inc(qh.r, qh.c, qhk));
        *P(qh.r, qh.c) = S::load(WD::v(qhw));
    }
    __syncthreads();

    // ---- phase 4: v^{n+3/2} on the cells the tile's new pressure needs --
    // vx on rows [0, TY), columns [-R, TX+R-1); vy on rows [-R, TY+R-1),
    // columns [0, TX) -- and the tile's own cells stored
    walk(IQ0(), IQ1(), [&](int k) { const int r = row_of(k); return r >= 0 && r < TY; },
         vx_slot, xwd, xqb, [&](int k) {
             xlds_rec(f1, k);
             store(vx_out, row_of(k), xw[k - Q0]);
             store8(qx_out, row_of(k), qxw[k - Q0]);
         });
    walk(IV0(), IV1(), [&](int k) { const int r = row_of(k); return r >= -R && r < TY + R - 1; },
         vy_slot, ywd, yqb, [&](int k) {
             ylds_rec(f1, k);
             const int r = row_of(k);
             if (r >= 0 && r < TY) {
                 store(vy_out, r, yw[k - V0]);
                 store8(qy_out, r, qyw[k - V0]);
             }
         });
    if (xh_on && xh.r >= 0 && xh.r < TY && xh.c >= -R && xh.c < TX + R - 1) {
        upd(xhw, qxh, bxh * vx_g(P(xh.r, xh.c)));
        *X(xh.r, xh.c) = S::load(WD::v(xhw));
    }
    __syncthreads();

    // ---- phase 5: p^{n+2} on the tile
    walk(IQ0(), IQ1(), [&](int k) { const int r = row_of(k); return r >= 0 && r < TY; },
         [&](int k) { return p_slot(f1, k); }, pwd, pqb, [&](int k) {
             rec(f1, 0, row_of(k), S::load(WD::v(pw[k - P0])));
             store(p_out, row_of(k), pw[k - P0]);
             store8(qp_out, row_of(k), qpw[k - Q0]);
         });
}

template <class S, int COMP, int ORDER, int TY, int NW, bool FRC>
__device__ __forceinline__ void ac2d_tile2_entry(const Ac2dDesc &d, int par, int tile,
                                                 int ntx, Tb2Lds<ORDER, TY> &L)
{
    constexpr int TX = 64, H = ORDER - 1;
    const int nx = (int)d.nx, ny = (int)d.ny;
    const int x0 = (tile % ntx) * TX;
    const int y0 = (tile / ntx) * TY;
    // every cell the tile touches lies within 2H cells of it
    const bool xin = x0 >= 2 * H && x0 + TX + 2 * H <= nx;
    const bool yin = y0 >= 2 * H && y0 + TY + 2 * H <= ny;
    if (xin && yin)
        ac2d_tile2<S, COMP, ORDER, TY, NW, false, FRC>(d, par, x0, y0, L);
    else
        ac2d_tile2<S, COMP, ORDER, TY, NW, true, FRC>(d, par, x0, y0, L);
}

template <class S, int COMP, int ORDER, int TY, int NW, bool FRC = false>
__global__ __launch_bounds__(64 * NW) void ac2d_step2_kernel(const Ac2dBatch a)
{
    __shared__ Tb2Lds<ORDER, TY> L;
    int32_t tile = xcd_tile(blockIdx.x, a.total_tiles);
    const int shot = find_shot(a, tile);
    ac2d_tile2_entry<S, COMP, ORDER, TY, NW, FRC>(*a.desc[shot], a.parity[shot],
                                                  tile - a.tile_start[shot], a.tiles_x[shot],
                                                  L);
}

template <class S, int COMP, int ORDER, int TY, int NW, bool FRC = false>
__global__ __launch_bounds__(64 * NW) void ac2d_step2_1_kernel(const Ac2dOne o)
{
    __shared__ Tb2Lds<ORDER, TY> L;
    ac2d_tile2_entry<S, COMP, ORDER, TY, NW, FRC>(o.d, o.parity,
                                                  xcd_tile(blockIdx.x, o.total_tiles),
                                                  o.tiles_x, L);
}

// ------------------------------------------------------------- dispatch --

template <bool FRC, class S, int COMP, int ORDER>
static hipError_t step2_tile(const Ac2dBatch &a, const Ac2dDesc *one, int tile,
                             hipStream_t s)
{
    Ac2dOne o;
    if (one) {
        o.d = *one;
        o.parity = a.parity[0];
        o.tiles_x = a.tiles_x[0];
        o.total_tiles = a.total_tiles;
    }
    const dim3 grid(a.total_tiles);
    switch (tile) {
#define HW_TILE2(n)                                                               \
    case n: {                                                                     \
        constexpr int TY = kTiles2D[n].ty;                                        \
        constexpr int NW = kTiles2D[n].kind == 5 ? 8 : 4;                         \
        if constexpr (kTiles2D[n].kind == 4 || kTiles2D[n].kind == 5) {           \
            if (one)                                                              \
                hipLaunchKernelGGL((ac2d_step2_1_kernel<S, COMP, ORDER, TY, NW, FRC>), \
                                   grid, dim3(64 * NW), 0, s, o);                 \
            else                                                                  \
                hipLaunchKernelGGL((ac2d_step2_kernel<S, COMP, ORDER, TY, NW, FRC>),   \
                                   grid, dim3(64 * NW), 0, s, a);                 \
            break;                                                                \
        } else {                                                                  \
            return hipErrorInvalidValue;                                          \
        }                                                                         \
    }
        HW_TILE2(9) HW_TILE2(10) HW_TILE2(11)
#undef HW_TILE2
    default:
        return hipErrorInvalidValue;
    }
    static_assert(kNumTiles2D == 12, "update the two-step tile dispatch");
    return hipGetLastError();
}

template <bool FRC, class S, int COMP>
static hipError_t step2_order(const Ac2dBatch &a, const Ac2dDesc *one, int order,
                              int tile, hipStream_t s)
{
    return order == 4 ? step2_tile<FRC, S, COMP, 4>(a, one, tile, s)
                      : step2_tile<FRC, S, COMP, 2>(a, one, tile, s);
}

template <bool FRC, class S>
static hipError_t step2_comp(const Ac2dBatch &a, const Ac2dDesc *one, int comp,
                             int order, int tile, hipStream_t s)
{
    switch (comp) {
    case COMP_NONE: return step2_order<FRC, S, COMP_NONE>(a, one, order, tile, s);
    case COMP_FAST2SUM: return step2_order<FRC, S, COMP_FAST2SUM>(a, one, order, tile, s);
    case COMP_TWOSUM: return step2_order<FRC, S, COMP_TWOSUM>(a, one, order, tile, s);
    case COMP_TWOSUM8:
        if constexpr (S::id != F32::id)
            return step2_order<FRC, S, COMP_TWOSUM8>(a, one, order, tile, s);
        break;
    }
    return hipErrorInvalidValue;
}

// Launch of every shot of `a` on two-step tile shape `tile`, with the
// forcing code compiled in or not.
template <bool FRC>
static hipError_t step2_launch(const Ac2dBatch &a, const Ac2dDesc *one, int storage,
                               int comp, int order, int tile, hipStream_t s)
{
    if (a.total_tiles <= 0)
        return hipSuccess;
    if (one && a.nshots != 1)
        return hipErrorInvalidValue;
    switch (storage) {
    case HW_F32: return step2_comp<FRC, F32>(a, one, comp, order, tile, s);
    case HW_F16: return step2_comp<FRC, F16>(a, one, comp, order, tile, s);
    case HW_BF16: return step2_comp<FRC, BF16>(a, one, comp, order, tile, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace hw
