// Stable recompaction by cell (Sec. III-A: particles must stay cell-ordered
// for the position codec to locate their cell).  The new order is the stable
// counting sort of the old order by new canonical cell.
//
// Fast path (every particle moved at most one coarse cell per axis): one
// workgroup owns a brick of destination cells made of BY x BZ segments of BX
// cells along x inside one tile, so every segment's output is one contiguous
// run of the new arrays.  Its particles can only come from the source window
// (BX+2) x (BY+2) x (BZ+2).  Per source cell, one thread walks the cell's
// particles in order twice: first to count, per destination cell of the brick
// and move code, the arrivals (each such pair has exactly one source cell, so
// its counter has one writer), then -- once each destination has ordered its
// 27 source cells by canonical index and formed prefix counts -- to give
// every incoming particle its slot
//   new_offset[dest] + (arrivals from earlier source cells)
//                    + (earlier same-code particles of its own source cell).
// Slots are mapped in LDS and the planes copied run by run (coalesced); a
// brick with more arrivals than the map holds scatters directly instead.
// Per-code counts and prefixes are 16-bit: the caller takes this path only
// when no cell of the old or the new counts holds more than 65535 particles.  Deterministic, no global atomics.
//
// General path: the new keys are sorted stably with the LSD radix sort and the
// planes are permuted.
#include <algorithm>

#include "common.h"

namespace cube {

namespace {

constexpr int kCThreads = 256;
constexpr int kMaxBX = 16;
constexpr int kSlots = 1024;
constexpr int kDirCap = 3072;                      // staged move codes of the source window
constexpr int kMovCap = 768;                       // movers of the window handled one thread per particle

struct CompactShape {
    int BX, BY, BZ;
};

// Brick of BX x BYZ x BYZ destination cells (BX a power of two <= 16,
// BYZ 1 or 2), fixed at compile time so that all window index arithmetic is
// by constants.
template <int BX, int BYZ>
__global__ __launch_bounds__(kCThreads) void k_compact_fast(Geom g, const int32_t* __restrict__ off_old,
                                                            const int32_t* __restrict__ off_new,
                                                            const uint8_t* __restrict__ dir, Planes src, Planes dst,
                                                            const StepScalars* sc) {
    if (*(volatile const int32_t*)&sc->halt) return;
    constexpr int BY = BYZ, BZ = BYZ;
    constexpr int SX = BX + 2, SY = BY + 2, SZ = BZ + 2;
    constexpr int nsrc = SX * SY * SZ, ndst = BX * BY * BZ, nrow = BY * BZ;
    static_assert(nsrc <= 512, "a window particle's source cell takes 9 bits");
    static_assert(ndst <= kWave, "one lane per destination cell");
    __shared__ int s_start[nsrc];              // first old index of each source cell
    __shared__ int s_pref[nsrc + 1];           // window position of each source cell's first particle
    __shared__ uint16_t s_arr[ndst][27];       // arrivals per (destination, code), then running ranks
    __shared__ uint16_t s_pre[ndst][27];       // arrivals from earlier source cells (< the new count <= 65535)
    __shared__ int s_doff[ndst + 1];
    __shared__ int s_run[nrow + 1];            // per destination row segment: slot base
    __shared__ uint8_t s_face[ndst];           // destination cells on a tile face
    __shared__ int s_nface;
    __shared__ uint16_t s_slot[kSlots];        // window index of the particle for each output slot
    __shared__ int s_scan[kCThreads / kWave + 1];
    // one word per window particle: source cell (bits 0-8), move code (9-13,
    // 31 = farther than one cell), movers before it in window order (14-31)
    __shared__ uint32_t s_e[kDirCap];
    __shared__ uint16_t s_mov[kMovCap];        // window index of each mover
    __shared__ uint16_t s_mrank[kMovCap];      // mover's rank among its cell's same-code particles

    const int nbx = g.Nc / BX, nby = g.Nc / BY;
    const int b = (int)xcd_logical_block();
    const int B0[3] = {(b % nbx) * BX, ((b / nbx) % nby) * BY, (b / (nbx * nby)) * BZ};
    const int Nc = g.Nc;
    auto wrap1 = [Nc](int x) { return x < 0 ? x + Nc : (x >= Nc ? x - Nc : x); };   // x in [-1, Nc]
    // window coordinates of source cell h
    auto win = [](int h, int& hx, int& hy, int& hz) {
        hx = h % SX;
        hy = (h / SX) % SY;
        hz = h / (SX * SY);
    };

    for (int i = threadIdx.x; i < ndst * 27; i += kCThreads) (&s_arr[0][0])[i] = 0;
    for (int e = threadIdx.x; e < ndst; e += kCThreads) {
        const int ex = e % BX, ey = (e / BX) % BY, ez = e / (BX * BY);
        s_doff[e] = off_new[canon(g, B0[0] + ex, B0[1] + ey, B0[2] + ez)];
    }
    if ((int)threadIdx.x < nrow) {
        // arrivals of each of the BY*BZ row segments (each contiguous in the new order)
        const int r = threadIdx.x, ey = r % BY, ez = r / BY;
        const int64_t first = canon(g, B0[0], B0[1] + ey, B0[2] + ez);
        s_run[r + 1] = off_new[first + BX] - off_new[first];
    }
    // source cells (two per thread at most): start, window coordinates and
    // count, then the prefix of the counts over the window
    {
        constexpr int kPer = (nsrc + kCThreads - 1) / kCThreads;
        int c[kPer], run = 0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int h = threadIdx.x * kPer + q;
            c[q] = 0;
            if (h < nsrc) {
                const int hx = h % SX, hy = (h / SX) % SY, hz = h / (SX * SY);
                const int64_t cc = canon(g, wrap1(B0[0] + hx - 1), wrap1(B0[1] + hy - 1), wrap1(B0[2] + hz - 1));
                const int st = off_old[cc];
                c[q] = off_old[cc + 1] - st;
                s_start[h] = st;
            }
            run += c[q];
        }
        int tot;
        int base = block_exclusive_scan(run, s_scan, &tot);
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int h = threadIdx.x * kPer + q;
            if (h < nsrc) s_pref[h] = base;
            base += c[q];
        }
        if (threadIdx.x == 0) s_pref[nsrc] = tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s_run[0] = 0;
        for (int r = 1; r <= nrow; ++r) s_run[r] += s_run[r - 1];
    }
    // destination cell (in the brick) of a code-d particle of the source cell
    // at window coordinates (hx, hy, hz), or -1
    auto dest_of = [&](int hx, int hy, int hz, int d) -> int {
        const int ex = hx + (d % 3 - 1) - 1, ey = hy + ((d / 3) % 3 - 1) - 1, ez = hz + (d / 9 - 1) - 1;
        if (ex < 0 || ex >= BX || ey < 0 || ey >= BY || ez < 0 || ez >= BZ) return -1;
        return ex + BX * (ey + BY * ez);
    };
    // Walk 1.  Most particles keep their cell (code 13).  When the window fits
    // in LDS every particle gets one word: its source cell (each cell's thread
    // fills its range), its code (staged one lane per particle, all loads in
    // flight) and the number of movers before it (a block scan).  A stayer's
    // rank in its cell is then its in-cell index minus the movers before it;
    // the movers (listed by the scan) are ranked by their cell's thread, so
    // per-thread work follows the few movers, not the crowded cells.  Blocks
    // with too many movers, or windows too large to stage, walk each source
    // cell serially.
    const int nwin = s_pref[nsrc];
    const bool staged = nwin <= kDirCap;
    constexpr int kStay = 13;
    constexpr int kFar = 31;
    bool bal = false;
    int nmov = 0;
    if (staged) {
        for (int h = threadIdx.x; h < nsrc; h += kCThreads) {
            const int e0 = s_pref[h], e1 = s_pref[h + 1];
            for (int e = e0; e < e1; ++e) s_e[e] = (uint32_t)h;
        }
        __syncthreads();
        constexpr int K = kDirCap / kCThreads;
        {
            int hv[K], cv[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int e = threadIdx.x + j * kCThreads;
                hv[j] = 0;
                cv[j] = 0;
                if (e < nwin) {
                    const int h = (int)s_e[e];
                    hv[j] = h;
                    cv[j] = dir[(int64_t)s_start[h] + (e - s_pref[h])];
                }
            }
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int e = threadIdx.x + j * kCThreads;
                if (e < nwin) s_e[e] = (uint32_t)hv[j] | ((uint32_t)(cv[j] < 27 ? cv[j] : kFar) << 9);
            }
        }
        __syncthreads();
        // movers before every window particle: K consecutive particles per thread
        uint32_t ev[K];
        int nm = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int e = threadIdx.x * K + j;
            ev[j] = e < nwin ? s_e[e] : (uint32_t)(kStay << 9);
            nm += ((ev[j] >> 9) & 31) != kStay ? 1 : 0;
        }
        int mb = block_exclusive_scan(nm, s_scan, &nmov);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int e = threadIdx.x * K + j;
            if (e < nwin) {
                s_e[e] = ev[j] | ((uint32_t)mb << 14);
                if (((ev[j] >> 9) & 31) != kStay) {
                    if (mb < kMovCap) s_mov[mb] = (uint16_t)e;
                    ++mb;
                }
            }
        }
        bal = nmov <= kMovCap;
        __syncthreads();
    }
    if (bal) {
        for (int h = threadIdx.x; h < nsrc; h += kCThreads) {
            const int start = s_pref[h], end = s_pref[h + 1];
            int hx, hy, hz;
            win(h, hx, hy, hz);
            const int m0 = start < nwin ? (int)(s_e[start] >> 14) : nmov;
            const int m1 = end < nwin ? (int)(s_e[end] >> 14) : nmov;
            const int dstay = dest_of(hx, hy, hz, kStay);
            if (dstay >= 0) s_arr[dstay][kStay] = (uint16_t)((end - start) - (m1 - m0));
            for (int m = m0; m < m1; ++m) {
                const int d = (int)((s_e[s_mov[m]] >> 9) & 31);
                const int dc = d < 27 ? dest_of(hx, hy, hz, d) : -1;
                if (dc >= 0) {
                    const int r = s_arr[dc][d];
                    s_arr[dc][d] = (uint16_t)(r + 1);
                    s_mrank[m] = (uint16_t)r;
                }
            }
        }
    } else {
        for (int h = threadIdx.x; h < nsrc; h += kCThreads) {
            const int st = s_start[h], base = s_pref[h], n = s_pref[h + 1] - base;
            int hx, hy, hz;
            win(h, hx, hy, hz);
            int stay = 0;
            for (int q0 = 0; q0 < n; q0 += 8) {
                int cq[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    cq[u] = (q0 + u < n) ? (staged ? (int)((s_e[base + q0 + u] >> 9) & 31) : (int)dir[st + q0 + u])
                                         : 255;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (q0 + u >= n) break;
                    const int d = cq[u];
                    if (d == kStay) {
                        ++stay;
                    } else {
                        const int dc = d < 27 ? dest_of(hx, hy, hz, d) : -1;
                        if (dc >= 0) s_arr[dc][d] = (uint16_t)(s_arr[dc][d] + 1);
                    }
                }
            }
            const int dstay = dest_of(hx, hy, hz, kStay);
            if (dstay >= 0) s_arr[dstay][kStay] = (uint16_t)stay;       // the only writer of this entry
        }
    }
    __syncthreads();
    auto code = [&](int h, int q) -> int {
        return staged ? (int)((s_e[s_pref[h] + q] >> 9) & 31) : (int)dir[s_start[h] + q];
    };

    // Arrivals from earlier source cells, per destination and code: the 27
    // source cells of a destination are ranked by canonical index.  When they
    // lie in one tile (the destination is not on a tile face) the order is the
    // reversed code order, and wave 0 forms suffix sums, one lane per
    // destination.  Tile-face destinations (a few per brick) are listed and
    // ranked by the whole block, one thread per (destination, code).
    if (threadIdx.x < kWave) {
        const int dcell = threadIdx.x;
        bool face = false;
        if (dcell < ndst) {
            const int gx = B0[0] + dcell % BX, gy = B0[1] + (dcell / BX) % BY, gz = B0[2] + dcell / (BX * BY);
            const int lx = g.tc_shift >= 0 ? (gx & (g.Tc - 1)) : gx % g.Tc;
            const int ly = g.tc_shift >= 0 ? (gy & (g.Tc - 1)) : gy % g.Tc;
            const int lz = g.tc_shift >= 0 ? (gz & (g.Tc - 1)) : gz % g.Tc;
            face = !(lx >= 1 && lx <= g.Tc - 2 && ly >= 1 && ly <= g.Tc - 2 && lz >= 1 && lz <= g.Tc - 2);
            if (!face) {
                int acc = 0;
#pragma unroll
                for (int d = 26; d >= 0; --d) {
                    const int c = s_arr[dcell][d];
                    s_pre[dcell][d] = (uint16_t)acc;
                    acc += c;
                }
            }
        }
        const uint64_t fm = __ballot(face);
        if (face) s_face[__popcll(fm & ((1ull << dcell) - 1ull))] = (uint8_t)dcell;
        if (dcell == 0) s_nface = __popcll(fm);
    }
    __syncthreads();
    {
        const int nface = s_nface;
        const int T3 = g.Tc * g.Tc * g.Tc;
        for (int t = threadIdx.x; t < nface * 27; t += kCThreads) {
            const int f = t / 27, d = t - 27 * f;
            const int dcell = s_face[f];
            const int gx = B0[0] + dcell % BX, gy = B0[1] + (dcell / BX) % BY, gz = B0[2] + dcell / (BX * BY);
            // canonical index of the source cell at offset (ox, oy, oz) is
            // Ax[ox+1] + Ay[oy+1] + Az[oz+1]; code d has offsets -carry
            int Ax[3], Ay[3], Az[3];
#pragma unroll
            for (int o = 0; o < 3; ++o) {
                const int x = wrap1(gx + o - 1), y = wrap1(gy + o - 1), z = wrap1(gz + o - 1);
                int tx, ty, tz, lx, ly, lz;
                if (g.tc_shift >= 0) {
                    const int sft = g.tc_shift, msk = g.Tc - 1;
                    tx = x >> sft; ty = y >> sft; tz = z >> sft;
                    lx = x & msk; ly = y & msk; lz = z & msk;
                } else {
                    tx = x / g.Tc; ty = y / g.Tc; tz = z / g.Tc;
                    lx = x - tx * g.Tc; ly = y - ty * g.Tc; lz = z - tz * g.Tc;
                }
                Ax[o] = tx * T3 + lx;
                Ay[o] = ty * g.nt * T3 + ly * g.Tc;
                Az[o] = tz * g.nt * g.nt * T3 + lz * g.Tc * g.Tc;
            }
            auto sel = [](const int* a, int i) { return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]); };
            const int kd = sel(Ax, 2 - d % 3) + sel(Ay, 2 - (d / 3) % 3) + sel(Az, 2 - d / 9);
            int acc = 0;
#pragma unroll
            for (int d2 = 0; d2 < 27; ++d2) {
                const int k2 = Ax[2 - d2 % 3] + Ay[2 - (d2 / 3) % 3] + Az[2 - d2 / 9];
                acc += (k2 < kd) ? (int)s_arr[dcell][d2] : 0;
            }
            s_pre[dcell][d] = (uint16_t)acc;
        }
    }
    __syncthreads();
    const bool use_slots = s_run[nrow] <= kSlots && nwin <= 65536;
    // particle p (window index e) goes to output o: through the slot map, or
    // copied directly when the brick's arrivals exceed the map
    auto place = [&](int dcell, int d, int rank, int e, int p) {
        const int o = s_doff[dcell] + s_pre[dcell][d] + rank;
        if (use_slots) {
            const int row = dcell / BX;
            const int slot = s_run[row] + (o - s_doff[BX * row]);
            if (slot >= 0 && slot < kSlots) s_slot[slot] = (uint16_t)e;
        } else if (o >= 0 && o < g.n) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                dst.m[a][o] = src.m[a][p];
                if (src.u[0]) dst.u[a][o] = src.u[a][p];
                if (src.v[0]) dst.v[a][o] = src.v[a][p];
            }
            if (dst.ids) dst.ids[o] = src.ids[p];
        }
    };
    if (bal) {
        // walk 2 visits only particles that can land in the brick: the
        // stayers of its own cells (nrow contiguous window ranges) and the
        // movers of the whole window
        int rs[nrow], rp[nrow + 1];
        rp[0] = 0;
#pragma unroll
        for (int r = 0; r < nrow; ++r) {
            const int h0 = 1 + SX * ((1 + r % BY) + SY * (1 + r / BY));
            rs[r] = s_pref[h0];
            rp[r + 1] = rp[r] + (s_pref[h0 + BX] - rs[r]);
        }
        const int ni = rp[nrow];
        for (int i = threadIdx.x; i < ni; i += kCThreads) {
            int e = rs[0] + i;
#pragma unroll
            for (int r = 1; r < nrow; ++r)
                if (i >= rp[r]) e = rs[r] + (i - rp[r]);
            const uint32_t v = s_e[e];
            if (((v >> 9) & 31) != kStay) continue;
            const int h = (int)(v & 511);
            int hx, hy, hz;
            win(h, hx, hy, hz);
            const int dc = (hx - 1) + BX * ((hy - 1) + BY * (hz - 1));
            const int start = s_pref[h];
            // a stayer's rank: its in-cell index minus the movers before it in its cell
            const int rank = (e - start) - ((int)(v >> 14) - (int)(s_e[start] >> 14));
            place(dc, kStay, rank, e, s_start[h] + (e - start));
        }
        for (int m = threadIdx.x; m < nmov; m += kCThreads) {
            const int e = s_mov[m];
            const uint32_t v = s_e[e];
            const int d = (int)((v >> 9) & 31);
            if (d >= 27) continue;
            const int h = (int)(v & 511);
            int hx, hy, hz;
            win(h, hx, hy, hz);
            const int dc = dest_of(hx, hy, hz, d);
            if (dc < 0) continue;
            place(dc, d, (int)s_mrank[m], e, s_start[h] + (e - s_pref[h]));
        }
    } else {
        // reuse the arrival counts as running ranks
        for (int i = threadIdx.x; i < ndst * 27; i += kCThreads) (&s_arr[0][0])[i] = 0;
        __syncthreads();
        // walk 2: slot of every particle that lands in this brick (four
        // particles per iteration so that their LDS reads overlap; stayers are
        // ranked by a register counter, movers by the LDS counters)
        for (int h = threadIdx.x; h < nsrc; h += kCThreads) {
            const int st = s_start[h], base = s_pref[h], n = s_pref[h + 1] - base;
            int hx, hy, hz;
            win(h, hx, hy, hz);
            const int dstay = dest_of(hx, hy, hz, kStay);
            int stay = 0;
            for (int q0 = 0; q0 < n; q0 += 4) {
                int dq[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) dq[u] = (q0 + u < n) ? code(h, q0 + u) : 255;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int d = dq[u];
                    const int dcell = d == kStay ? dstay : (d < 27 ? dest_of(hx, hy, hz, d) : -1);
                    if (dcell < 0) continue;
                    int rank;
                    if (d == kStay) {
                        rank = stay++;
                    } else {
                        rank = s_arr[dcell][d];
                        s_arr[dcell][d] = (uint16_t)(rank + 1);
                    }
                    place(dcell, d, rank, base + q0 + u, st + q0 + u);
                }
            }
        }
    }
    if (!use_slots) return;
    __syncthreads();
    // copy run by run: consecutive slots are consecutive outputs
    const int total = s_run[nrow];
    constexpr int U = 4;
    const bool cp_u = src.u[0] != nullptr, cp_v = src.v[0] != nullptr;
    for (int base = 0; base < total; base += kCThreads * U) {
        uint8_t mv[U][3];
        int8_t uv[U][3];
        float vv[U][3];
        uint32_t idv[U];
        int ov[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * kCThreads + threadIdx.x;
            ov[u] = -1;
            if (i < total) {
                int row = 0;
#pragma unroll
                for (int r = 1; r < nrow; ++r) row += i >= s_run[r] ? 1 : 0;
                const int o = s_doff[BX * row] + (i - s_run[row]);
                const int e = s_slot[i];
                int p = -1;
                if (e < nwin) {
                    const int h = staged ? (int)(s_e[e] & 511) : find_cell_fixed<9>(s_pref, nsrc, e);
                    p = s_start[h] + (e - s_pref[h]);
                }
                if (o >= 0 && o < g.n && p >= 0 && p < g.n) {
                    ov[u] = o;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        mv[u][a] = src.m[a][p];
                        if (cp_u) uv[u][a] = src.u[a][p];
                        if (cp_v) vv[u][a] = src.v[a][p];
                    }
                    if (dst.ids) idv[u] = src.ids[p];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int o = ov[u];
            if (o < 0) continue;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                dst.m[a][o] = mv[u][a];
                if (cp_u) dst.u[a][o] = uv[u][a];
                if (cp_v) dst.v[a][o] = vv[u][a];
            }
            if (dst.ids) dst.ids[o] = idv[u];
        }
    }
}

// Brick compaction from the gather's mover records.  One wave per gather
// brick D (tile-major numbering, XCD-aware).  The old storage order is the
// canonical cell order, so for a destination cell c the stable counting sort
// puts, in order of old index p: the particles arriving from cells stored
// before c, then c's own stayers, then the arrivals from cells stored after
// c.  Hence, with every arrival's old index p known,
//   stayer of c, k-th among them:  new_offset[c] + #(arrivals with p < off_old[c]) + k
//   arrival into c:                new_offset[c] + #(arrivals into c with smaller p)
//                                  + (p >= off_old[c] ? stayers of c : 0)
// with no distinction between tile faces, periodic wraps and interior cells.
// The arrivals are the records of class "towards D" of D and its 26
// neighbours (the gather groups each brick's records by class); stayers are
// D's own particles with move code 13, ranked by a wave scan per 64.
// The work per brick is a handful of short dependent phases, so every load
// of a phase is issued before the first is used, and a small LDS footprint
// keeps many bricks in flight per CU.  Bricks with more arrivals than the
// LDS list holds rank them from the records in memory (slower, same result).
constexpr int kKThreads = kWave;
constexpr int kInCap = 192;

template <int R>
__global__ __launch_bounds__(kKThreads) void k_compact_brick(Geom g, const int32_t* __restrict__ off_old,
                                                             const int32_t* __restrict__ off_new,
                                                             const uint8_t* __restrict__ dir,
                                                             const uint4* __restrict__ ment,
                                                             const int32_t* __restrict__ mhdr, Planes src,
                                                             Planes dst, const StepScalars* sc) {
    if (*(volatile const int32_t*)&sc->halt) return;
    constexpr int BXc = kGBX / R, BYc = kGBY / R, BZc = kGBZ / R;
    constexpr int NROW = BYc * BZc, NCELL = BXc * NROW;
    static_assert(NCELL <= kWave && NROW <= 8 && BXc <= 8, "brick shape");
    __shared__ int s_oo[NROW][BXc + 1], s_on[NROW][BXc + 1];
    __shared__ int s_rowpref[NROW + 1];
    __shared__ int s_abefore[NCELL], s_stay[NCELL];
    __shared__ int s_lbase[27], s_lpref[28];
    __shared__ uint4 s_in[kInCap];

    const int lane = (int)threadIdx.x;
    const int64_t lin = xcd_logical_block();
    const int nbx = g.T / kGBX, nby = g.T / kGBY, nbz = g.T / kGBZ, bpt = nbx * nby * nbz;
    const int tile = (int)(lin / bpt), b = (int)(lin - (int64_t)tile * bpt);
    const int tx = tile % g.nt, ty = (tile / g.nt) % g.nt, tz = tile / (g.nt * g.nt);
    // global brick coordinates and the brick's first coarse cell
    const int gb[3] = {tx * nbx + b % nbx, ty * nby + (b / nbx) % nby, tz * nbz + b / (nbx * nby)};
    const int c0[3] = {gb[0] * BXc, gb[1] * BYc, gb[2] * BZc};
    const int NB[3] = {g.nt * nbx, g.nt * nby, g.nt * nbz};

    for (int t = lane; t < NROW * (BXc + 1); t += kKThreads) {
        const int r = t / (BXc + 1), j = t - r * (BXc + 1);
        const int64_t c = canon(g, c0[0], c0[1] + r % BYc, c0[2] + r / BYc) + j;
        s_oo[r][j] = off_old[c];
        s_on[r][j] = off_new[c];
    }
    // the brick at offset o sends the records of class 26 - o here
    int cnt = 0;
    if (lane < 27) {
        const int o = lane;
        int sb[3] = {gb[0] + o % 3 - 1, gb[1] + (o / 3) % 3 - 1, gb[2] + o / 9 - 1};
#pragma unroll
        for (int k = 0; k < 3; ++k) sb[k] = sb[k] < 0 ? sb[k] + NB[k] : (sb[k] >= NB[k] ? sb[k] - NB[k] : sb[k]);
        const int stile = sb[0] / nbx + g.nt * (sb[1] / nby + g.nt * (sb[2] / nbz));
        const int sbl = sb[0] % nbx + nbx * (sb[1] % nby + nby * (sb[2] % nbz));
        const int32_t* h = mhdr + ((int64_t)stile * bpt + sbl) * kHdrInts;
        const int c = 26 - o;
        const int lo = h[1 + c], hi = h[2 + c];
        s_lbase[o] = h[0] + lo;
        cnt = hi - lo;
    }
    {
        const int incl = wave_inclusive_scan(cnt);
        if (lane < 27) s_lpref[lane] = incl - cnt;
        if (lane == 26) s_lpref[27] = incl;
    }
    if (lane < NCELL) {
        s_abefore[lane] = 0;
        s_stay[lane] = 0;
    }
    __syncthreads();
    if (lane == 0) {
        s_rowpref[0] = 0;
        for (int r = 0; r < NROW; ++r) s_rowpref[r + 1] = s_rowpref[r] + (s_oo[r][BXc] - s_oo[r][0]);
    }
    const int nin = s_lpref[27];
    const bool listed = nin <= kInCap;
    auto arrival = [&](int i) -> uint4 {
        const int l = find_cell_fixed<5>(s_lpref, 27, i);
        return ment[s_lbase[l] + (i - s_lpref[l])];
    };
    if (listed) {
        constexpr int UC = 3;                      // record loads in flight per lane
        for (int i0 = 0; i0 < nin; i0 += UC * kKThreads) {
            uint4 rec[UC];
#pragma unroll
            for (int u = 0; u < UC; ++u) {
                const int i = i0 + u * kKThreads + lane;
                if (i < nin) rec[u] = arrival(i);
            }
#pragma unroll
            for (int u = 0; u < UC; ++u) {
                const int i = i0 + u * kKThreads + lane;
                if (i < nin) s_in[i] = rec[u];
            }
        }
    }
    __syncthreads();
    auto oo_of = [&](int d) { return s_oo[d / BXc][d % BXc]; };
    // arrivals from cells stored before each destination cell
    for (int i = lane; i < nin; i += kKThreads) {
        const uint4 rec = listed ? s_in[i] : arrival(i);
        const int d = (int)(rec.y & 255);
        if ((int)rec.x < oo_of(d)) atomicAdd(&s_abefore[d], 1);
    }
    __syncthreads();

    // own particles in storage order, U chunks of 64 per round with every
    // load of the round in flight before the first is used: stayers keep
    // their order within their cell and are written straight to their slot
    const int nown = s_rowpref[NROW];
    const bool cp_u = src.u[0] != nullptr, cp_v = src.v[0] != nullptr, cp_id = dst.ids != nullptr;
    constexpr int U = 4;
    for (int base0 = 0; base0 < nown; base0 += U * kKThreads) {
        int pv[U], rowv[U], xv[U], code[U];
        uint32_t mb[U], ub[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base0 + u * kKThreads + lane;
            pv[u] = -1;
            rowv[u] = 0;
            xv[u] = 0;
            code[u] = 0;
            mb[u] = 0;
            ub[u] = 0;
            if (e < nown) {
                const int row = find_cell_fixed<3>(s_rowpref, NROW, e);
                const int p = s_oo[row][0] + (e - s_rowpref[row]);
                pv[u] = p;
                rowv[u] = row;
                xv[u] = find_cell_fixed<3>(s_oo[row], BXc, p);
                code[u] = dir[p];
                // the planes are read for every particle: waiting for the code
                // first would cost a round trip, and movers are few
                mb[u] = (uint32_t)src.m[0][p] | ((uint32_t)src.m[1][p] << 8) | ((uint32_t)src.m[2][p] << 16);
                if (cp_u)
                    ub[u] = (uint32_t)(uint8_t)src.u[0][p] | ((uint32_t)(uint8_t)src.u[1][p] << 8) |
                            ((uint32_t)(uint8_t)src.u[2][p] << 16);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int base = base0 + u * kKThreads;
            if (base >= nown) break;
            const int e = base + lane;
            const int row = rowv[u], x = xv[u], p = pv[u];
            const int cl = x + BXc * row;
            int stay = 0, first = 0, cell_end = 0;
            if (e < nown) {
                stay = code[u] == 13 ? 1 : 0;
                // chunk positions of this particle's cell
                const int cell_e = s_rowpref[row] + (s_oo[row][x] - s_oo[row][0]);
                cell_end = s_rowpref[row] + (s_oo[row][x + 1] - s_oo[row][0]);
                first = max(cell_e, base) - base;
            }
            const int incl = wave_inclusive_scan(stay);
            const int before_first = __shfl(incl, max(first - 1, 0), kWave);
            const int before = first > 0 ? before_first : 0;
            const int k = s_stay[cl] + (incl - stay - before);
            if (e < nown && stay) {
                const int o = s_on[row][x] + s_abefore[cl] + k;
                if (o >= 0 && o < g.n) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        dst.m[a][o] = (uint8_t)(mb[u] >> (8 * a));
                        if (cp_u) dst.u[a][o] = (int8_t)(ub[u] >> (8 * a));
                        if (cp_v) dst.v[a][o] = src.v[a][p];
                    }
                    if (cp_id) dst.ids[o] = src.ids[p];
                }
            }
            __syncthreads();
            // the last particle of each cell's run in this chunk carries the count on
            if (e < nown && (e == nown - 1 || lane == kKThreads - 1 || e + 1 == cell_end))
                s_stay[cl] += incl - before;
            __syncthreads();
        }
    }

    // arrivals: rank among the arrivals into the same cell by old index
    for (int i = lane; i < nin; i += kKThreads) {
        const uint4 rec = listed ? s_in[i] : arrival(i);
        const int d = (int)(rec.y & 255), p = (int)rec.x;
        int rank = 0;
        for (int j = 0; j < nin; ++j) {
            const uint4 q = listed ? s_in[j] : arrival(j);
            rank += ((int)(q.y & 255) == d && q.x < rec.x) ? 1 : 0;
        }
        const int row = d / BXc, x = d - row * BXc;
        const int o = s_on[row][x] + rank + (p >= s_oo[row][x] ? s_stay[d] : 0);
        if (o < 0 || o >= g.n || p < 0 || p >= g.n) continue;
        dst.m[0][o] = (uint8_t)(rec.z & 255);
        dst.m[1][o] = (uint8_t)((rec.z >> 8) & 255);
        dst.m[2][o] = (uint8_t)((rec.z >> 16) & 255);
        if (cp_u) {
            dst.u[0][o] = (int8_t)(rec.w & 255);
            dst.u[1][o] = (int8_t)((rec.w >> 8) & 255);
            dst.u[2][o] = (int8_t)((rec.w >> 16) & 255);
        }
        if (cp_v)
#pragma unroll
            for (int a = 0; a < 3; ++a) dst.v[a][o] = src.v[a][p];
        if (cp_id) dst.ids[o] = src.ids[p];
    }
}

// keys of the general path: new canonical cell of every particle, old order
__global__ __launch_bounds__(256) void k_general_keys(Geom g, const int32_t* __restrict__ offsets,
                                                       const uint8_t* __restrict__ dir,
                                                       const uint32_t* __restrict__ far_key, uint32_t* __restrict__ key,
                                                       uint32_t* __restrict__ idx) {
    extern __shared__ int offs[];
    const Chunk ch = chunk_of(g, blockIdx.x);
    for (int j = threadIdx.x; j <= g.Tc; j += blockDim.x) offs[j] = offsets[ch.c0 + j];
    __syncthreads();
    for (int p = offs[0] + threadIdx.x; p < offs[g.Tc]; p += blockDim.x) {
        const int d = dir[p];
        uint32_t k;
        if (d < 27) {
            const int j = find_cell(offs, g.Tc, p);
            k = (uint32_t)canon(g, wrapi(ch.cx0 + j + d % 3 - 1, g.Nc), wrapi(ch.cy + (d / 3) % 3 - 1, g.Nc),
                                wrapi(ch.cz + d / 9 - 1, g.Nc));
        } else {
            k = far_key[p];
        }
        key[p] = k;
        idx[p] = (uint32_t)p;
    }
}

__global__ void k_permute(const uint32_t* __restrict__ perm, Planes src, Planes dst, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t p = perm[j];
    if (p >= n) return;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dst.m[a][j] = src.m[a][p];
        if (src.u[0]) dst.u[a][j] = src.u[a][p];
        if (src.v[0]) dst.v[a][j] = src.v[a][p];
    }
    if (dst.ids) dst.ids[j] = src.ids[p];
}

CompactShape compact_shape(const Geom& g) {
    CompactShape sh;
    const int H = g.r / g.f;                       // particles per coarse cell ~ H^3
    sh.BY = sh.BZ = (H <= 2) ? 2 : 1;
    int bx = kMaxBX;
    // a power of two dividing the tile side; the window must not wrap onto itself
    while (bx > 1 && (bx > g.Tc || bx + 2 > g.Nc || g.Tc % bx)) bx /= 2;
    sh.BX = bx;
    return sh;
}

template <int BYZ>
void launch_compact_yz(int bx, dim3 grid, const Geom& g, const int32_t* off_old, const int32_t* off_new,
                       const uint8_t* dir, Planes src, Planes dst, const StepScalars* sc, hipStream_t s) {
    switch (bx) {
        case 16: hipLaunchKernelGGL((k_compact_fast<16, BYZ>), grid, dim3(kCThreads), 0, s, g, off_old, off_new, dir, src, dst, sc); break;
        case 8: hipLaunchKernelGGL((k_compact_fast<8, BYZ>), grid, dim3(kCThreads), 0, s, g, off_old, off_new, dir, src, dst, sc); break;
        case 4: hipLaunchKernelGGL((k_compact_fast<4, BYZ>), grid, dim3(kCThreads), 0, s, g, off_old, off_new, dir, src, dst, sc); break;
        case 2: hipLaunchKernelGGL((k_compact_fast<2, BYZ>), grid, dim3(kCThreads), 0, s, g, off_old, off_new, dir, src, dst, sc); break;
        default: hipLaunchKernelGGL((k_compact_fast<1, BYZ>), grid, dim3(kCThreads), 0, s, g, off_old, off_new, dir, src, dst, sc); break;
    }
}

}  // namespace

bool compact_supported(const Geom& g) {
    const CompactShape sh = compact_shape(g);
    return sh.BX >= 1 && g.Nc % sh.BX == 0 && g.Nc % sh.BY == 0 && sh.BY + 2 <= g.Nc;
}

void launch_compact_fast(const Geom& g, const int32_t* offsets_old, const int32_t* offsets_new, const uint8_t* dir,
                         Planes src, Planes dst, const StepScalars* sc, hipStream_t s) {
    const CompactShape sh = compact_shape(g);
    const int64_t nb = (int64_t)(g.Nc / sh.BX) * (g.Nc / sh.BY) * (g.Nc / sh.BZ);
    const dim3 grid((unsigned)nb);
    if (sh.BY == 2) launch_compact_yz<2>(sh.BX, grid, g, offsets_old, offsets_new, dir, src, dst, sc, s);
    else launch_compact_yz<1>(sh.BX, grid, g, offsets_old, offsets_new, dir, src, dst, sc, s);
}

int64_t compact_bricks(const Geom& g) {
    return (int64_t)g.ntiles * (g.T / kGBX) * (g.T / kGBY) * (g.T / kGBZ);
}

void launch_compact_bricks(const Geom& g, const int32_t* offsets_old, const int32_t* offsets_new,
                           const uint8_t* dir, const uint4* ment, const int32_t* mhdr, Planes src, Planes dst,
                           const StepScalars* sc, hipStream_t s) {
    const dim3 grid((unsigned)compact_bricks(g));
    if (g.r == 4)
        hipLaunchKernelGGL(k_compact_brick<4>, grid, dim3(kKThreads), 0, s, g, offsets_old, offsets_new, dir, ment,
                           mhdr, src, dst, sc);
    else
        hipLaunchKernelGGL(k_compact_brick<8>, grid, dim3(kKThreads), 0, s, g, offsets_old, offsets_new, dir, ment,
                           mhdr, src, dst, sc);
}

void launch_general_keys(const Geom& g, const int32_t* offsets_old, const uint8_t* dir, const uint32_t* far_key,
                         uint32_t* key, uint32_t* idx, hipStream_t s) {
    const int64_t chunks = g.ncells / g.Tc;
    hipLaunchKernelGGL(k_general_keys, dim3((unsigned)chunks), dim3(256), (g.Tc + 1) * sizeof(int), s, g,
                       offsets_old, dir, far_key, key, idx);
}

void launch_permute_planes(const uint32_t* perm, Planes src, Planes dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_permute, dim3(grid1d(n, 256)), dim3(256), 0, s, perm, src, dst, n);
}

}  // namespace cube
