// grid.cpp -- host-side grid builder: validates a block list and builds the device tables.
//
// The paper keeps its block tree and neighbour information on the CPU and rebuilds the ghost-cell
// "memory maps" only when the grid changes (Sec. 3.1, Sec. 4.4). Here the same split holds: this file
// runs once per grid on the host and produces flat integer tables that kernels only read:
//   * per block: the relation of each of its 6 faces (equal-level neighbour id, outflow, inflow, or a
//     level change whose ghost layers come from the halo buffer), flux-correction records, flags;
//   * the 26-direction neighbour table reported through the ABI;
//   * per simulation: block lookup tables per level (used by the inter-level ghost rules);
//   * a Morton-ordered block schedule so that neighbouring blocks run close together in time.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>

#include "bmhd_internal.h"

namespace bmhd {

namespace {

int64_t blocks_along(const bmhd_sim_desc &s, int lvl, int axis) { return int64_t(s.nroot[axis]) << lvl; }

struct Lookup {
    const HostGrid *g;
    int32_t at(int sim, int lvl, int64_t x, int64_t y, int64_t z) const {
        const bmhd_sim_desc &s = g->sdesc[sim];
        int64_t nx = blocks_along(s, lvl, 0), ny = blocks_along(s, lvl, 1), nz = blocks_along(s, lvl, 2);
        if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) return -1;
        return g->lut[size_t(g->sims[sim].lut_off[lvl] + (z * ny + y) * nx + x)];
    }
};

// Wrap a block coordinate along one axis at one level. Returns false when it leaves through a
// non-periodic face (then *bc_code is that face's boundary type).
bool wrap_block(const bmhd_sim_desc &s, int lvl, int axis, int64_t &c, int *bc_code) {
    int64_t n = blocks_along(s, lvl, axis);
    if (c >= 0 && c < n) return true;
    int t = s.bc[2 * axis + (c < 0 ? 0 : 1)];
    if (t == BMHD_BC_PERIODIC) {
        c = ((c % n) + n) % n;
        return true;
    }
    *bc_code = t;
    return false;
}

uint64_t spread3(uint64_t v) {
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

void prim_to_cons_host(const double *w, double *u) {
    const double rho = w[0];
    const double u2 = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
    const double b2 = w[4] * w[4] + w[5] * w[5] + w[6] * w[6];
    u[0] = rho;
    for (int a = 0; a < 3; ++a) u[1 + a] = rho * w[1 + a];
    for (int a = 0; a < 3; ++a) u[4 + a] = w[4 + a];
    u[7] = w[7] / (5.0 / 3.0 - 1.0) + 0.5 * rho * u2 + 0.5 * b2;
}

int32_t build_grid(const bmhd_grid_desc *d, HostGrid &g, std::string &err) {
    if (!d || d->n_blocks < 0 || d->n_sims <= 0 || !d->sims || (d->n_blocks > 0 && (!d->level || !d->ijk || !d->sim))) {
        err = "grid descriptor: null pointer or bad counts";
        return BMHD_EINVAL;
    }
    g.nb = d->n_blocks;
    g.ns = d->n_sims;
    g.level.assign(d->level, d->level + g.nb);
    g.ijk.assign(d->ijk, d->ijk + 3 * size_t(g.nb));
    g.sim.assign(d->sim, d->sim + g.nb);
    g.sdesc.assign(d->sims, d->sims + g.ns);

    // simulations and lookup tables
    g.sims.assign(size_t(g.ns), DevSim{});
    size_t lut_total = 0;
    for (int s = 0; s < g.ns; ++s) {
        const bmhd_sim_desc &sd = g.sdesc[s];
        for (int a = 0; a < 3; ++a)
            if (sd.nroot[a] <= 0 || sd.nroot[a] > (1 << 20)) {
                err = "simulation " + std::to_string(s) + ": nroot must be positive";
                return BMHD_EINVAL;
            }
        if (!(sd.dx0 > 0.0) || !std::isfinite(sd.dx0)) {
            err = "simulation " + std::to_string(s) + ": dx0 must be positive";
            return BMHD_EINVAL;
        }
        for (int a = 0; a < 3; ++a) {
            int lo = sd.bc[2 * a], hi = sd.bc[2 * a + 1];
            if (lo < 0 || lo > 2 || hi < 0 || hi > 2 || ((lo == BMHD_BC_PERIODIC) != (hi == BMHD_BC_PERIODIC))) {
                err = "simulation " + std::to_string(s) + ": bad or unpaired boundary codes";
                return BMHD_EINVAL;
            }
        }
        DevSim &ds = g.sims[s];
        for (int a = 0; a < 3; ++a) {
            ds.origin[a] = sd.origin[a];
            ds.body_c[a] = sd.body_c[a];
            ds.nroot[a] = sd.nroot[a];
        }
        ds.dx0 = sd.dx0;
        ds.body_r = sd.body_r;
        for (int f = 0; f < 6; ++f) ds.bc[f] = sd.bc[f];
        prim_to_cons_host(sd.inflow_W, ds.inflow_U);
        for (int l = 0; l < 2; ++l) {
            ds.lut_off[l] = int32_t(lut_total);
            lut_total += size_t(blocks_along(sd, l, 0) * blocks_along(sd, l, 1) * blocks_along(sd, l, 2));
        }
    }
    if (lut_total > (size_t(1) << 31)) {
        err = "lookup tables too large";
        return BMHD_EINVAL;
    }
    g.lut.assign(lut_total, -1);
    for (int b = 0; b < g.nb; ++b) {
        int s = g.sim[b], l = g.level[b];
        if (s < 0 || s >= g.ns || (l != 0 && l != 1)) {
            err = "block " + std::to_string(b) + ": bad simulation id or level";
            return BMHD_EINVAL;
        }
        const bmhd_sim_desc &sd = g.sdesc[s];
        int64_t c[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = g.ijk[3 * size_t(b) + a];
            if (c[a] < 0 || c[a] >= blocks_along(sd, l, a)) {
                err = "block " + std::to_string(b) + ": index outside the root box";
                return BMHD_EINVAL;
            }
        }
        int64_t nx = blocks_along(sd, l, 0), ny = blocks_along(sd, l, 1);
        int32_t &slot = g.lut[size_t(g.sims[s].lut_off[l] + (c[2] * ny + c[1]) * nx + c[0])];
        if (slot != -1) {
            err = "block " + std::to_string(b) + ": overlaps block " + std::to_string(slot);
            return BMHD_EINVAL;
        }
        slot = b;
    }
    Lookup L{&g};
    for (int s = 0; s < g.ns; ++s) {
        const bmhd_sim_desc &sd = g.sdesc[s];
        for (int64_t z = 0; z < sd.nroot[2]; ++z)
            for (int64_t y = 0; y < sd.nroot[1]; ++y)
                for (int64_t x = 0; x < sd.nroot[0]; ++x) {
                    bool leaf = L.at(s, 0, x, y, z) >= 0;
                    int kids = 0;
                    for (int q = 0; q < 8; ++q)
                        kids += L.at(s, 1, 2 * x + (q & 1), 2 * y + ((q >> 1) & 1), 2 * z + (q >> 2)) >= 0;
                    if (leaf ? kids != 0 : kids != 8) {
                        err = "simulation " + std::to_string(s) + ": root block (" + std::to_string(x) + "," +
                              std::to_string(y) + "," + std::to_string(z) + ") is not exactly covered";
                        return BMHD_EINVAL;
                    }
                }
    }

    // 26-direction neighbour table
    g.nbr.assign(size_t(g.nb) * NDIR * 5, -1);
    for (int b = 0; b < g.nb; ++b) {
        const int s = g.sim[b], l = g.level[b];
        const bmhd_sim_desc &sd = g.sdesc[s];
        int n = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!dx && !dy && !dz) continue;
                    int32_t *e = &g.nbr[(size_t(b) * NDIR + n++) * 5];
                    const int dd[3] = {dx, dy, dz};
                    int64_t c[3];
                    int code = -1;
                    bool inside = true;
                    for (int a = 0; a < 3 && inside; ++a) {
                        c[a] = int64_t(g.ijk[3 * size_t(b) + a]) + dd[a];
                        inside = wrap_block(sd, l, a, c[a], &code);
                    }
                    if (!inside) {
                        e[0] = code == BMHD_BC_OUTFLOW ? BMHD_REL_OUTFLOW : BMHD_REL_INFLOW;
                        continue;
                    }
                    int32_t id = L.at(s, l, c[0], c[1], c[2]);
                    if (id >= 0) {
                        e[0] = BMHD_REL_SAME;
                        e[1] = id;
                    } else if (l == 1) {
                        e[0] = BMHD_REL_COARSER;
                        e[1] = L.at(s, 0, c[0] >> 1, c[1] >> 1, c[2] >> 1);
                    } else {
                        e[0] = BMHD_REL_FINER;
                        int m = 1;
                        for (int q = 0; q < 8; ++q) {
                            const int sub[3] = {q & 1, (q >> 1) & 1, q >> 2};
                            bool touches = true;
                            for (int a = 0; a < 3; ++a)
                                if (dd[a] != 0 && sub[a] != (dd[a] > 0 ? 0 : 1)) touches = false;
                            if (touches) e[m++] = L.at(s, 1, 2 * c[0] + sub[0], 2 * c[1] + sub[1], 2 * c[2] + sub[2]);
                        }
                    }
                }
    }

    // per-block face relations, halo slots and flux-correction records
    g.blocks.assign(size_t(g.nb), DevBlock{});
    g.halo_items.clear();
    g.n_halo_slots = 0;
    g.n_fc_rec = 0;
    for (int b = 0; b < g.nb; ++b) {
        DevBlock &B = g.blocks[b];
        std::memset(&B, 0, sizeof B);
        B.sim = g.sim[b];
        B.level = g.level[b];
        for (int a = 0; a < 3; ++a) B.ijk[a] = g.ijk[3 * size_t(b) + a];
        B.halo_slot = -1;
        for (int f = 0; f < 6; ++f) {
            B.fc_rec[f] = -1;
            B.fc_quad[f] = 0;
        }
    }
    for (int b = 0; b < g.nb; ++b) {
        DevBlock &B = g.blocks[b];
        const bmhd_sim_desc &sd = g.sdesc[B.sim];
        for (int f = 0; f < 6; ++f) {
            const int a = f >> 1, side = f & 1;
            int64_t c[3] = {B.ijk[0], B.ijk[1], B.ijk[2]};
            c[a] += side ? 1 : -1;
            int code = -1;
            if (!wrap_block(sd, B.level, a, c[a], &code)) {
                B.face[f] = code == BMHD_BC_OUTFLOW ? FACE_OUTFLOW : FACE_INFLOW;
                continue;
            }
            int32_t id = L.at(B.sim, B.level, c[0], c[1], c[2]);
            if (id >= 0) {
                B.face[f] = id;
                continue;
            }
            B.face[f] = FACE_LEVEL;
            B.flags |= BF_LEVEL;
            g.halo_items.push_back((b << 3) | f);
            if (B.level == 0) {
                // coarse side: one flux-correction record per face, shared with the 4 fine blocks
                const int r = g.n_fc_rec++;
                B.fc_rec[f] = r;
                B.fc_role |= 1 << f;
                B.fc_skip |= 1 << f;
                B.flags |= BF_FC;
                const int a1 = a == 0 ? 1 : 0, a2 = a == 2 ? 1 : 2;
                for (int q2 = 0; q2 < 2; ++q2)
                    for (int q1 = 0; q1 < 2; ++q1) {
                        int64_t fc[3];
                        fc[a] = 2 * c[a] + (side ? 0 : 1);
                        fc[a1] = 2 * c[a1] + q1;
                        fc[a2] = 2 * c[a2] + q2;
                        int32_t fb = L.at(B.sim, 1, fc[0], fc[1], fc[2]);
                        if (fb < 0) {
                            err = "internal: missing fine block across a level face";
                            return BMHD_EINVAL;
                        }
                        DevBlock &F = g.blocks[fb];
                        F.fc_rec[f ^ 1] = r;
                        F.fc_quad[f ^ 1] = q1 + 2 * q2;
                        F.flags |= BF_FC;
                    }
            }
        }
        if (B.flags & BF_LEVEL) B.halo_slot = g.n_halo_slots++;
    }

    // coarse cells that take flux corrections (faces in ascending order per cell)
    g.fc_cells.clear();
    for (int b = 0; b < g.nb; ++b) {
        const DevBlock &B = g.blocks[b];
        if (!B.fc_role) continue;
        std::map<int, DevFcCell> cells;
        for (int f = 0; f < 6; ++f) {
            if (!((B.fc_role >> f) & 1)) continue;
            const int a = f >> 1, side = f & 1;
            const int a1 = a == 0 ? 1 : 0, a2 = a == 2 ? 1 : 2;
            for (int t2 = 0; t2 < 8; ++t2)
                for (int t1 = 0; t1 < 8; ++t1) {
                    int ii[3];
                    ii[a] = side ? 7 : 0;
                    ii[a1] = t1;
                    ii[a2] = t2;
                    const int cell = (ii[2] * 8 + ii[1]) * 8 + ii[0];
                    auto it = cells.find(cell);
                    if (it == cells.end()) {
                        DevFcCell e;
                        std::memset(&e, 0, sizeof e);
                        e.block = b;
                        e.cell = cell;
                        it = cells.emplace(cell, e).first;
                    }
                    DevFcCell &e = it->second;
                    e.rec[e.n] = B.fc_rec[f];
                    e.face[e.n] = f;
                    e.t[e.n] = t1 + 8 * t2;
                    e.n++;
                }
        }
        for (auto &kv : cells) g.fc_cells.push_back(kv.second);
    }

    // blocks whose cells or face ghosts can meet the body sphere
    for (int b = 0; b < g.nb; ++b) {
        DevBlock &B = g.blocks[b];
        const bmhd_sim_desc &sd = g.sdesc[B.sim];
        if (!(sd.body_r > 0.0)) continue;
        const double dx = sd.dx0 / double(1 << B.level);
        double dist2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double lo = sd.origin[a] + (double(B.ijk[a]) * 8 - 2) * dx;
            const double hi = sd.origin[a] + (double(B.ijk[a]) * 8 + 10) * dx;
            const double c = sd.body_c[a];
            const double t = c < lo ? lo - c : (c > hi ? c - hi : 0.0);
            dist2 += t * t;
        }
        if (dist2 <= sd.body_r * sd.body_r * (1.0 + 1e-12) + 1e-300) B.flags |= BF_NEAR_BODY;
    }

    // Morton schedule (per simulation, positions at level-1 resolution)
    g.order.resize(size_t(g.nb));
    std::iota(g.order.begin(), g.order.end(), 0);
    std::vector<uint64_t> key(size_t(g.nb));
    for (int b = 0; b < g.nb; ++b) {
        const DevBlock &B = g.blocks[b];
        const int sh = 1 - B.level;
        key[b] = spread3(uint64_t(B.ijk[0]) << sh) | (spread3(uint64_t(B.ijk[1]) << sh) << 1) |
                 (spread3(uint64_t(B.ijk[2]) << sh) << 2);
    }
    std::stable_sort(g.order.begin(), g.order.end(), [&](int32_t x, int32_t y) {
        if (g.sim[x] != g.sim[y]) return g.sim[x] < g.sim[y];
        return key[x] < key[y];
    });

    // the same schedule split for the stage kernel: the blocks clear of any body (block form), then the
    // blocks near a body (plane form). Where the clear blocks with a face on another level are at most a
    // fifth of the clear blocks, they go after the others (n_clear_plain of them), so that the others can
    // run while the level-change halo fill, which only the former read, is under way; with a larger share
    // (the paper's fast-wave grid: a third) the two partial launches lose more than that saves, and the
    // clear blocks keep their order.
    std::vector<int32_t> plain, level;
    for (int32_t b : g.order)
        if (!(g.blocks[b].flags & BF_NEAR_BODY)) ((g.blocks[b].flags & BF_LEVEL) ? level : plain).push_back(b);
    g.split_level = !level.empty() && plain.size() >= 4 * level.size();
    g.order_split.clear();
    if (g.split_level) {
        g.order_split = plain;
        g.order_split.insert(g.order_split.end(), level.begin(), level.end());
        g.n_clear_plain = int32_t(plain.size());
    } else {
        for (int32_t b : g.order)
            if (!(g.blocks[b].flags & BF_NEAR_BODY)) g.order_split.push_back(b);
        g.n_clear_plain = int32_t(g.order_split.size());
    }
    g.n_clear = int32_t(g.order_split.size());
    for (int32_t b : g.order)
        if (g.blocks[b].flags & BF_NEAR_BODY) g.order_split.push_back(b);

    // high face planes with no neighbour across them, numbered block by block (x, y, z)
    g.n_hb = 0;
    for (int b = 0; b < g.nb; ++b)
        for (int d = 0; d < 3; ++d)
            g.blocks[b].hb_pos[d] = g.blocks[b].face[2 * d + 1] < 0 ? g.n_hb++ : -1;

    // workspace layout
    size_t off = 0;
    g.off_blocks = off; off = align256(off + sizeof(DevBlock) * g.blocks.size());
    g.off_sims = off; off = align256(off + sizeof(DevSim) * g.sims.size());
    g.off_lut = off; off = align256(off + sizeof(int32_t) * g.lut.size());
    g.off_order = off; off = align256(off + sizeof(int32_t) * g.order.size());
    g.off_order_split = off; off = align256(off + sizeof(int32_t) * g.order_split.size());
    g.off_halo_items = off; off = align256(off + sizeof(int32_t) * std::max<size_t>(1, g.halo_items.size()));
    g.off_fc_cells = off; off = align256(off + sizeof(DevFcCell) * std::max<size_t>(1, g.fc_cells.size()));
    g.off_lam = off; off = align256(off + sizeof(unsigned long long) * size_t(g.ns));
    g.table_bytes = off;
    g.off_halo = off; off = align256(off + sizeof(double) * size_t(HALO_SLOT) * size_t(std::max(1, g.n_halo_slots)));
    g.off_fcbuf = off; off = align256(off + sizeof(double) * size_t(FC_REC) * size_t(std::max(1, g.n_fc_rec)));
    g.work_bytes = off;
    g.blob.assign(g.table_bytes, 0);
    auto put = [&](size_t at, const void *src, size_t n) { if (n) std::memcpy(g.blob.data() + at, src, n); };
    put(g.off_blocks, g.blocks.data(), sizeof(DevBlock) * g.blocks.size());
    put(g.off_sims, g.sims.data(), sizeof(DevSim) * g.sims.size());
    put(g.off_lut, g.lut.data(), sizeof(int32_t) * g.lut.size());
    put(g.off_order, g.order.data(), sizeof(int32_t) * g.order.size());
    put(g.off_order_split, g.order_split.data(), sizeof(int32_t) * g.order_split.size());
    put(g.off_halo_items, g.halo_items.data(), sizeof(int32_t) * g.halo_items.size());
    put(g.off_fc_cells, g.fc_cells.data(), sizeof(DevFcCell) * g.fc_cells.size());
    return BMHD_OK;
}

}  // namespace bmhd
