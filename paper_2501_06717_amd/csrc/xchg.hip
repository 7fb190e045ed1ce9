// xchg.hip -- ghost-cell exchange between processes (the paper's message passing, Sec. 4.2-4.4,
// Algorithms 3 and 4) at one GPU's shapes.
//
// Blocks are assigned to processes; a process keeps its blocks, in ascending global id (the local index),
// in a padded view [8][n_local][12][12][12] (two ghost layers). Ghost cells arrive as messages from the
// neighbouring blocks: a copy from an equal-level neighbour, a restriction computed by a finer sender, a
// prolongation computed by a coarser sender from its own ghost cells. Copies and restrictions travel in
// pass 1, prolongations in pass 2 (after the senders' ghost cells are complete). Messages between blocks
// of one process are written straight into its view; the others go into one buffer per (sender,
// receiver) pair: every message is a header of n_C = 1 + 2 n_D = 7 values (the receiving block's local
// index, the receive box's low and high corners, inclusive) and then 8 values per cell of the box, in the
// order (v, i, j, k) with v fastest. The message maps (which messages, their start offsets) are counted on
// the host once per grid and assignment (the paper's IsCounted) and uploaded; the pack kernel writes the
// headers and values, the unpack kernel finds each message by its counted start and places its values by
// the header it reads. After the passes that feed them, ghost cells outside the domain are filled by the
// receiver from its own view (outflow: the nearest cell inside along the outflow axes; inflow: the
// inflow state).
//
// On one GPU the processes are virtual: every view lives in the same device memory and the buffers move
// with device copies standing in for the point-to-point transfers. Copy, restriction and prolongation
// use the arithmetic of bmhd_fill_ghosts (no contraction), so the views equal its padded view bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "bmhd_internal.h"

namespace bmhd {

constexpr int XCHG_NC = 7;  // header values per message
constexpr int MSG_COPY = 0, MSG_RESTRICT = 1, MSG_PROLONG = 2;

// One message as the kernels see it.
struct DevMsg {
    int32_t sender;       // global id of the sending block
    int32_t s_local;      // its local index on the sending process
    int32_t r_local;      // local index of the receiving block on the receiving process
    int32_t type;         // MSG_*
    int32_t lo[3], hi[3]; // receive box, receiver's padded coordinates in [-2, 10), inclusive
    int32_t ru[3];        // the receiver's block position at its level as seen from the sender (unwrapped)
    int32_t ncell;        // cells of the box
    int64_t off;          // start of the message in the sender's send buffer (pack) or the receiver's
                          // receive buffer (unpack); for local messages unused
    int32_t cfirst;       // cells of the messages before this one in its group (one workgroup's work)
    int32_t pad;
};
static_assert(sizeof(DevMsg) == 72, "DevMsg layout");

}  // namespace bmhd

struct bmhd_xchg {
    const bmhd_grid *grid = nullptr;
    int32_t nr = 0;
    std::vector<int32_t> rank, local, nloc;
    // per pass p (0, 1) and process: the messages it packs (to other processes), the ones it unpacks, the
    // local ones; host copies and their offsets in the device workspace
    std::vector<bmhd::DevMsg> send[2], recv[2], loc[2];
    std::vector<int64_t> send_first[2], recv_first[2], loc_first[2];  // [nr + 1] prefix per process
    // messages grouped per block (the sending block for send, the receiving block otherwise), one
    // workgroup per group: first message of each group, and per process the range of its groups
    std::vector<int32_t> grp[2][3];
    std::vector<int64_t> grp_first[2][3];
    std::vector<int64_t> len[2];                                     // [nr][nr] doubles, sender-major
    std::vector<int32_t> bnd_blocks[2];                              // per pass: blocks whose boundary ghosts
    std::vector<int64_t> bnd_first[2];                               // are filled after it, per process
    std::vector<int32_t> blocks_local;                               // global ids in local order per process
    std::vector<int64_t> blocks_first;                               // [nr + 1]
    // for the stage from a process's view: its blocks clear of any body first (n_clear of them), then the
    // blocks near a body (ranges as blocks_first); its coarse cells taking flux corrections
    std::vector<int32_t> split, n_clear;
    std::vector<bmhd::DevFcCell> fc;
    std::vector<int64_t> fc_first;                                   // [nr + 1]
    // stage mode (bmhd_xchg_create_for_stage): the views hold only what the stage reads from them and
    // what the packs of those messages read; the interior copies cover only the blocks that send
    bool stage_mode = false;
    std::vector<int32_t> view_faces;                                 // [nb]: bit f, face f's ghosts from the view
    std::vector<int32_t> int_blocks;                                 // blocks whose interior is copied, per process
    std::vector<int64_t> int_first;                                  // [nr + 1]
    std::vector<std::vector<int64_t>> table;                         // or_xchg_messages-style rows
    size_t work_bytes = 0;
    size_t off_msgs[2][3] = {}, off_grp[2][3] = {}, off_bnd[2] = {}, off_blocks = 0;
    size_t off_split = 0, off_local = 0, off_fc = 0, off_vfaces = 0, off_int = 0;
    void *d_work = nullptr;
};

namespace bmhd {
namespace {

int64_t floordiv(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

int32_t lut_host(const HostGrid &g, int s, int l, const int64_t p[3]) {
    const DevSim &S = g.sims[s];
    const int64_t nx = int64_t(S.nroot[0]) << l, ny = int64_t(S.nroot[1]) << l, nz = int64_t(S.nroot[2]) << l;
    if (p[0] < 0 || p[1] < 0 || p[2] < 0 || p[0] >= nx || p[1] >= ny || p[2] >= nz) return -1;
    return g.lut[size_t(S.lut_off[l] + (p[2] * ny + p[1]) * nx + p[0])];
}

struct Msg {
    int32_t receiver, type, slot;
    int32_t lo[3], hi[3];
    int64_t ru[3];
};

// Messages sent by block b, in slot order: for each of the 26 directions (x fastest), the equal-level
// neighbour (copy), else the coarser block there (restriction, from a level-1 sender), else each finer
// block touching b (prolongation, from a level-0 sender); the receive box is the part of the receiver's
// padded box covered by b; directions leaving through a non-periodic face send nothing, and a receiver
// placement already served by b is not served again.
std::vector<Msg> block_messages(const HostGrid &g, int b) {
    std::vector<Msg> out;
    const int s = g.sim[b], l = g.level[b];
    const bmhd_sim_desc &sd = g.sdesc[s];
    int dir = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy && !dz) continue;
                const int d[3] = {dx, dy, dz};
                int64_t p[3], pw[3];
                bool inside = true;
                for (int a = 0; a < 3; ++a) {
                    const int64_t n = int64_t(sd.nroot[a]) << l;
                    p[a] = g.ijk[3 * b + a] + d[a];
                    pw[a] = p[a];
                    if (p[a] < 0 || p[a] >= n) {
                        if (sd.bc[2 * a + (p[a] < 0 ? 0 : 1)] != BMHD_BC_PERIODIC) inside = false;
                        pw[a] = ((p[a] % n) + n) % n;
                    }
                }
                const int this_dir = dir++;
                if (!inside) continue;
                std::vector<Msg> cand;
                const int32_t same = lut_host(g, s, l, pw);
                if (same >= 0) {
                    Msg m{};
                    m.receiver = same;
                    m.type = MSG_COPY;
                    for (int a = 0; a < 3; ++a) m.ru[a] = p[a];
                    cand.push_back(m);
                } else if (l == 1) {
                    Msg m{};
                    int64_t cw[3];
                    for (int a = 0; a < 3; ++a) {
                        m.ru[a] = floordiv(p[a], 2);
                        const int64_t n = int64_t(sd.nroot[a]);
                        cw[a] = ((m.ru[a] % n) + n) % n;
                    }
                    m.receiver = lut_host(g, s, 0, cw);
                    m.type = MSG_RESTRICT;
                    cand.push_back(m);
                } else {
                    for (int q = 0; q < 8; ++q) {
                        const int sub[3] = {q & 1, (q >> 1) & 1, q >> 2};
                        bool ok = true;
                        for (int a = 0; a < 3; ++a)
                            if ((d[a] == 1 && sub[a] != 0) || (d[a] == -1 && sub[a] != 1)) ok = false;
                        if (!ok) continue;
                        Msg m{};
                        int64_t fw[3];
                        for (int a = 0; a < 3; ++a) {
                            fw[a] = 2 * pw[a] + sub[a];
                            m.ru[a] = 2 * p[a] + sub[a];
                        }
                        m.receiver = lut_host(g, s, 1, fw);
                        m.type = MSG_PROLONG;
                        m.slot = int32_t(cand.size());
                        cand.push_back(m);
                    }
                }
                for (Msg &m : cand) {
                    if (m.receiver < 0) continue;
                    const int rl = g.level[m.receiver];
                    bool empty = false;
                    for (int a = 0; a < 3; ++a) {
                        // b's cells at the receiver's level, relative to the receiver's origin
                        const int64_t base = rl > l ? int64_t(g.ijk[3 * b + a]) * 16
                                                    : (rl < l ? int64_t(g.ijk[3 * b + a]) * 4 : int64_t(g.ijk[3 * b + a]) * 8);
                        const int64_t width = rl > l ? 16 : (rl < l ? 4 : 8);
                        int64_t lo = base - 8 * m.ru[a], hi = lo + width;
                        lo = std::max<int64_t>(lo, -2);
                        hi = std::min<int64_t>(hi, 10);
                        if (lo >= hi) empty = true;
                        m.lo[a] = int32_t(lo);
                        m.hi[a] = int32_t(hi - 1);
                    }
                    if (empty) continue;
                    bool dup = false;
                    for (const Msg &o : out)
                        if (o.receiver == m.receiver && o.ru[0] == m.ru[0] && o.ru[1] == m.ru[1] && o.ru[2] == m.ru[2])
                            dup = true;
                    if (dup) continue;
                    m.slot = this_dir * 4 + (m.type == MSG_PROLONG ? m.slot : 0);
                    out.push_back(m);
                }
            }
    return out;
}

__host__ __device__ inline int64_t box_cells(const int32_t lo[3], const int32_t hi[3]) {
    return int64_t(hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ------------------------------------------------------------------------------------------------
// device side

struct XView {
    const double *v;  // [8][n][12][12][12]
    size_t vs;        // variable stride = n * 1728
    __device__ __forceinline__ double at(int var, int lb, int i, int j, int k) const {
        return v[var * vs + size_t(lb) * 1728 + ((k + 2) * 12 + (j + 2)) * 12 + (i + 2)];
    }
};

__device__ __forceinline__ double minmod_pair(double a, double b) {
    return (a > 0.0 && b > 0.0) ? fmin(a, b) : ((a < 0.0 && b < 0.0) ? fmax(a, b) : 0.0);
}

// The value of cell (i, j, k) of message m's receive box (receiver's padded coordinates) from the sending
// block's padded cells, by the ghost rules of bmhd_fill_ghosts.
__device__ __forceinline__ void message_value(const Tables &T, const DevMsg &m, const XView &S, int i, int j, int k,
                                           double out[8]) {
#pragma clang fp contract(off)
    const DevBlock &B = T.blocks[m.sender];
    const long long gr[3] = {8LL * m.ru[0] + i, 8LL * m.ru[1] + j, 8LL * m.ru[2] + k};
    if (m.type == MSG_COPY) {
        const int c[3] = {int(gr[0] - 8LL * B.ijk[0]), int(gr[1] - 8LL * B.ijk[1]), int(gr[2] - 8LL * B.ijk[2])};
#pragma unroll
        for (int v = 0; v < 8; ++v) out[v] = S.at(v, m.s_local, c[0], c[1], c[2]);
    } else if (m.type == MSG_RESTRICT) {
        int f[8][3];
        for (int q = 0; q < 8; ++q) {
            f[q][0] = int(2 * gr[0] + (q & 1) - 8LL * B.ijk[0]);
            f[q][1] = int(2 * gr[1] + ((q >> 1) & 1) - 8LL * B.ijk[1]);
            f[q][2] = int(2 * gr[2] + (q >> 2) - 8LL * B.ijk[2]);
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            double c[8];
            for (int q = 0; q < 8; ++q) c[q] = S.at(v, m.s_local, f[q][0], f[q][1], f[q][2]);
            const double s = ((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]));
            out[v] = s * 0.125;
        }
    } else {
        int C[3];
        double sg[3];
        for (int a = 0; a < 3; ++a) {
            const long long h = gr[a] >= 0 ? gr[a] / 2 : -((-gr[a] + 1) / 2);
            C[a] = int(h - 8LL * B.ijk[a]);
            sg[a] = (gr[a] & 1) ? 0.25 : -0.25;
        }
        double acc[8], uc[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            uc[v] = S.at(v, m.s_local, C[0], C[1], C[2]);
            acc[v] = uc[v];
        }
        for (int d = 0; d < 3; ++d) {
            int cm[3] = {C[0], C[1], C[2]}, cp[3] = {C[0], C[1], C[2]};
            cm[d] -= 1;
            cp[d] += 1;
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const double um = S.at(v, m.s_local, cm[0], cm[1], cm[2]);
                const double up = S.at(v, m.s_local, cp[0], cp[1], cp[2]);
                acc[v] = acc[v] + sg[d] * minmod_pair(uc[v] - um, up - uc[v]);
            }
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) out[v] = acc[v];
    }
}

__device__ __forceinline__ void box_cell(const DevMsg &m, int q, int &i, int &j, int &k) {
    const int nx = m.hi[0] - m.lo[0] + 1, ny = m.hi[1] - m.lo[1] + 1;
    i = m.lo[0] + q % nx;
    j = m.lo[1] + (q / nx) % ny;
    k = m.lo[2] + q / (nx * ny);
}

// Messages are grouped per block (one workgroup per group) and a group's cells are spread over the
// workgroup's threads: q runs over the concatenated boxes of the group's messages, the message of cell q is
// the one whose [cfirst, cfirst + ncell) holds it.
__device__ __forceinline__ int group_msg(const DevMsg *__restrict__ msgs, int mi, int q) {
    while (q >= msgs[mi].cfirst + msgs[mi].ncell) ++mi;
    return mi;
}

// Pack: the headers and values of every message of the group's sending block into the send buffer.
__global__ void __launch_bounds__(256) k_xchg_pack(Tables T, const DevMsg *__restrict__ msgs,
                                                   const int32_t *__restrict__ grp, XView S, double *__restrict__ buf) {
    const int m0 = grp[blockIdx.x], m1 = grp[blockIdx.x + 1];
    for (int mi = m0 + threadIdx.x; mi < m1; mi += blockDim.x) {
        const DevMsg &m = msgs[mi];
        double *h = buf + m.off;
        h[0] = double(m.r_local);
        for (int a = 0; a < 3; ++a) {
            h[1 + a] = double(m.lo[a]);
            h[4 + a] = double(m.hi[a]);
        }
    }
    const int total = msgs[m1 - 1].cfirst + msgs[m1 - 1].ncell;
    int mi = m0;
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
        mi = group_msg(msgs, mi, q);
        const DevMsg &m = msgs[mi];
        int i, j, k;
        box_cell(m, q - m.cfirst, i, j, k);
        double u[8];
        message_value(T, m, S, i, j, k, u);
        double *d = buf + m.off + XCHG_NC + size_t(q - m.cfirst) * 8;
#pragma unroll
        for (int v = 0; v < 8; ++v) d[v] = u[v];
    }
}

// Unpack: the messages for the group's receiving block, each found at its counted start; its header names
// the receiving block and the box, the values follow in box order. A header that disagrees with the
// counted map (a damaged buffer) is not unpacked and is counted in *bad.
__global__ void __launch_bounds__(256) k_xchg_unpack(const DevMsg *__restrict__ msgs, const int32_t *__restrict__ grp,
                                                     const double *__restrict__ buf, double *__restrict__ view,
                                                     size_t vs, int32_t *bad) {
    const int m0 = grp[blockIdx.x], m1 = grp[blockIdx.x + 1];
    const int total = msgs[m1 - 1].cfirst + msgs[m1 - 1].ncell;
    int mi = m0;
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
        mi = group_msg(msgs, mi, q);
        const DevMsg &mm = msgs[mi];
        const double *h = buf + mm.off;
        const int lb = int(h[0]);
        DevMsg m;
        bool ok = lb == mm.r_local;
        for (int a = 0; a < 3; ++a) {
            m.lo[a] = int(h[1 + a]);
            m.hi[a] = int(h[4 + a]);
            ok = ok && m.lo[a] == mm.lo[a] && m.hi[a] == mm.hi[a];
        }
        const int qq = q - mm.cfirst;
        if (!ok) {
            if (qq == 0 && bad) atomicAdd(bad, 1);
            continue;
        }
        int i, j, k;
        box_cell(m, qq, i, j, k);
        const double *d = h + XCHG_NC + size_t(qq) * 8;
        const size_t c = size_t(lb) * 1728 + ((k + 2) * 12 + (j + 2)) * 12 + (i + 2);
#pragma unroll
        for (int v = 0; v < 8; ++v) view[v * vs + c] = d[v];
    }
}

// Messages between blocks of one process, grouped per receiving block: values straight from the
// sender's cells into the receiver's ghost cells of the same view (pass 1 reads interiors and writes
// ghosts; pass 2 reads level-0 blocks and writes level-1 ghosts: no cell is both read and written).
__global__ void __launch_bounds__(256) k_xchg_local(Tables T, const DevMsg *__restrict__ msgs,
                                                    const int32_t *__restrict__ grp, double *__restrict__ view,
                                                    size_t vs) {
    const XView S{view, vs};
    const int m0 = grp[blockIdx.x], m1 = grp[blockIdx.x + 1];
    const int total = msgs[m1 - 1].cfirst + msgs[m1 - 1].ncell;
    int mi = m0;
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
        mi = group_msg(msgs, mi, q);
        const DevMsg &m = msgs[mi];
        int i, j, k;
        box_cell(m, q - m.cfirst, i, j, k);
        double u[8];
        message_value(T, m, S, i, j, k, u);
        const size_t c = size_t(m.r_local) * 1728 + ((k + 2) * 12 + (j + 2)) * 12 + (i + 2);
#pragma unroll
        for (int v = 0; v < 8; ++v) view[v * vs + c] = u[v];
    }
}

// Ghost cells of one block outside its simulation's domain, from the block's own padded cells: the inflow
// state where an out-of-domain axis is an inflow face, else the cell with every out-of-domain outflow axis
// clamped to the block's boundary layer (periodic axes keep the index: those cells came by message).
__global__ void __launch_bounds__(256) k_xchg_bounds(Tables T, const int32_t *__restrict__ blocks,
                                                     const int32_t *__restrict__ local_of, double *__restrict__ view,
                                                     size_t vs) {
    const int b = blocks[blockIdx.x];
    const int lb = local_of[blockIdx.x];
    const DevBlock &B = T.blocks[b];
    const DevSim &S = T.sims[B.sim];
    for (int c = threadIdx.x; c < 1728; c += blockDim.x) {
        const int ii[3] = {c % 12 - 2, (c / 12) % 12 - 2, c / 144 - 2};
        int src[3] = {ii[0], ii[1], ii[2]};
        bool out = false, inflow = false;
        for (int a = 0; a < 3; ++a) {
            const long long G = (long long)B.ijk[a] * 8 + ii[a];
            const long long n = ((long long)S.nroot[a] * 8) << B.level;
            if (G >= 0 && G < n) continue;
            const int t = S.bc[2 * a + (G < 0 ? 0 : 1)];
            if (t == BMHD_BC_PERIODIC) continue;
            out = true;
            if (t == BMHD_BC_INFLOW) inflow = true;
            src[a] = G < 0 ? 0 : 7;
        }
        if (!out) continue;
        const size_t dst = size_t(lb) * 1728 + c;
        const size_t from = size_t(lb) * 1728 + ((src[2] + 2) * 12 + (src[1] + 2)) * 12 + (src[0] + 2);
#pragma unroll
        for (int v = 0; v < 8; ++v) view[v * vs + dst] = inflow ? S.inflow_U[v] : view[v * vs + from];
    }
}

// A process's view with its blocks' interior cells from the global state.
__global__ void __launch_bounds__(512) k_xchg_interior(const int32_t *__restrict__ blocks,
                                                       const int32_t *__restrict__ local, const double *__restrict__ U,
                                                       size_t us, double *__restrict__ view, size_t vs) {
    const int b = blocks[blockIdx.x], lb = local[b], c = threadIdx.x;
    const int i = c & 7, j = (c >> 3) & 7, k = c >> 6;
    const size_t dst = size_t(lb) * 1728 + ((k + 2) * 12 + (j + 2)) * 12 + (i + 2);
#pragma unroll
    for (int v = 0; v < 8; ++v) view[v * vs + dst] = U[v * us + size_t(b) * 512 + c];
}

int32_t hip_ok(hipError_t e, const char *what) {
    if (e == hipSuccess) return BMHD_OK;
    return set_last_error(BMHD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace
}  // namespace bmhd

using namespace bmhd;

namespace {

int32_t need_xchg(const bmhd_xchg *x, int32_t pass, int32_t r) {
    if (!x) return set_last_error(BMHD_EINVAL, "null exchange");
    if (!x->d_work) return set_last_error(BMHD_EINVAL, "exchange maps not uploaded (call bmhd_xchg_upload first)");
    if (!x->grid->h.d_work) return set_last_error(BMHD_EINVAL, "grid not uploaded");
    if (pass != 1 && pass != 2) return set_last_error(BMHD_EINVAL, "pass must be 1 or 2");
    if (r < 0 || r >= x->nr) return set_last_error(BMHD_EINVAL, "process index out of range");
    return BMHD_OK;
}

bool aligned8(const void *p) { return p && (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

// Process r's blocks and coarse flux-correction cells in the uploaded workspace, ghost cells from d_view.
ViewStage view_stage(const bmhd_xchg *x, int r, const double *d_view) {
    const unsigned char *base = static_cast<const unsigned char *>(x->d_work);
    ViewStage v{};
    v.view = d_view;
    v.view_local = reinterpret_cast<const int32_t *>(base + x->off_local);
    v.view_faces = reinterpret_cast<const int32_t *>(base + x->off_vfaces);
    v.view_vs = int64_t(x->nloc[r]) * 1728;
    v.split = reinterpret_cast<const int32_t *>(base + x->off_split) + x->blocks_first[r];
    v.n_clear = x->n_clear[r];
    v.n_total = x->nloc[r];
    v.fc_cells = reinterpret_cast<const DevFcCell *>(base + x->off_fc) + x->fc_first[r];
    v.n_fc = int32_t(x->fc_first[r + 1] - x->fc_first[r]);
    return v;
}

}  // namespace

namespace bmhd {
namespace {
int32_t xchg_create(const bmhd_grid *g, const int32_t *rank, int32_t n_ranks, bool stage_mode, bmhd_xchg **out);
}  // namespace
}  // namespace bmhd

extern "C" {

int32_t bmhd_xchg_create(const bmhd_grid *g, const int32_t *rank, int32_t n_ranks, bmhd_xchg **out) {
    return xchg_create(g, rank, n_ranks, false, out);
}

int32_t bmhd_xchg_create_for_stage(const bmhd_grid *g, const int32_t *rank, int32_t n_ranks, bmhd_xchg **out) {
    return xchg_create(g, rank, n_ranks, true, out);
}

}  // extern "C"

namespace bmhd {
namespace {
int32_t xchg_create(const bmhd_grid *g, const int32_t *rank, int32_t n_ranks, bool stage_mode, bmhd_xchg **out) {
    if (!g || !rank || !out || n_ranks < 1) return set_last_error(BMHD_EINVAL, "xchg_create: bad arguments");
    const HostGrid &h = g->h;
    for (int b = 0; b < h.nb; ++b)
        if (rank[b] < 0 || rank[b] >= n_ranks) return set_last_error(BMHD_EINVAL, "xchg_create: rank out of range");
    bmhd_xchg *x = new bmhd_xchg;
    x->grid = g;
    x->stage_mode = stage_mode;
    x->nr = n_ranks;
    x->rank.assign(rank, rank + h.nb);
    x->local.assign(size_t(h.nb), 0);
    x->nloc.assign(size_t(n_ranks), 0);
    for (int b = 0; b < h.nb; ++b) x->local[b] = x->nloc[rank[b]]++;
    x->blocks_first.assign(size_t(n_ranks) + 1, 0);
    for (int r = 0; r < n_ranks; ++r) x->blocks_first[r + 1] = x->blocks_first[r] + x->nloc[r];
    x->blocks_local.assign(size_t(h.nb), 0);
    for (int b = 0; b < h.nb; ++b) x->blocks_local[size_t(x->blocks_first[rank[b]] + x->local[b])] = b;
    x->split.reserve(size_t(h.nb));
    x->n_clear.assign(size_t(n_ranks), 0);
    for (int r = 0; r < n_ranks; ++r) {
        for (int near = 0; near < 2; ++near)
            for (int64_t q = x->blocks_first[r]; q < x->blocks_first[r + 1]; ++q) {
                const int b = x->blocks_local[size_t(q)];
                if (((h.blocks[b].flags & BF_NEAR_BODY) != 0) != (near != 0)) continue;
                x->split.push_back(b);
                if (!near) x->n_clear[r]++;
            }
    }
    x->fc_first.assign(size_t(n_ranks) + 1, 0);
    for (int r = 0; r < n_ranks; ++r) {
        for (const DevFcCell &c : h.fc_cells)
            if (rank[c.block] == r) x->fc.push_back(c);
        x->fc_first[r + 1] = int64_t(x->fc.size());
    }

    std::vector<std::vector<Msg>> per_block(size_t(h.nb));
    for (int b = 0; b < h.nb; ++b) per_block[b] = block_messages(h, b);
    const int nr = n_ranks;
    // faces whose ghost cells the stage reads from the view: a neighbour on another process or on another
    // level (same-process neighbours and domain boundaries are read in place)
    x->view_faces.assign(size_t(h.nb), 0);
    for (int b = 0; b < h.nb; ++b)
        for (int f = 0; f < 6; ++f) {
            const int32_t rel = h.blocks[b].face[f];
            if (rel == FACE_LEVEL || (rel >= 0 && rank[rel] != rank[b])) x->view_faces[b] |= 1 << f;
        }
    // in stage mode a message between blocks of one process is needed only where the stage or a
    // prolongation reads it: restrictions and prolongations, and every pass-1 ghost cell of a block that
    // sends prolongations (its slopes reach into them)
    std::vector<char> psend(size_t(h.nb), 0), sends(size_t(h.nb), 0);
    for (int b = 0; b < h.nb; ++b)
        for (const Msg &m : per_block[b])
            if (m.type == MSG_PROLONG) psend[b] = 1;
    auto kept_local = [&](const Msg &m) { return !stage_mode || m.type != MSG_COPY || psend[m.receiver]; };
    for (int p = 0; p < 2; ++p) {
        const int pass = p + 1;
        x->len[p].assign(size_t(nr) * nr, 0);
        // counting loop: sender process, receiving process, then the sender's blocks in local order and
        // their messages in slot order
        std::vector<std::vector<DevMsg>> locv(static_cast<size_t>(nr));
        std::vector<std::vector<std::vector<DevMsg>>> incoming(static_cast<size_t>(nr),
                                                               std::vector<std::vector<DevMsg>>(static_cast<size_t>(nr)));
        for (int sp = 0; sp < nr; ++sp)
            for (int rp = 0; rp < nr; ++rp) {
                int64_t im = 0, start = 0;
                for (int64_t q = x->blocks_first[sp]; q < x->blocks_first[sp + 1]; ++q) {
                    const int b = x->blocks_local[size_t(q)];
                    for (const Msg &m : per_block[b]) {
                        const int mpass = m.type == MSG_PROLONG ? 2 : 1;
                        if (mpass != pass || rank[m.receiver] != rp) continue;
                        DevMsg d{};
                        d.sender = b;
                        d.s_local = x->local[b];
                        d.r_local = x->local[m.receiver];
                        d.type = m.type;
                        for (int a = 0; a < 3; ++a) {
                            d.lo[a] = m.lo[a];
                            d.hi[a] = m.hi[a];
                            d.ru[a] = int32_t(m.ru[a]);
                        }
                        d.ncell = int32_t(box_cells(m.lo, m.hi));
                        d.off = start;
                        std::vector<int64_t> row = {sp, rp, pass, im, start, b, m.slot, m.receiver, x->local[m.receiver],
                                                    m.type, m.lo[0], m.lo[1], m.lo[2], m.hi[0], m.hi[1], m.hi[2]};
                        x->table.push_back(row);
                        if (rp != sp) {
                            incoming[rp][sp].push_back(d);
                            sends[b] = 1;
                        } else if (kept_local(m)) {
                            locv[sp].push_back(d);
                            sends[b] = 1;
                        }
                        start += XCHG_NC + 8 * int64_t(d.ncell);
                        ++im;
                    }
                }
                if (rp != sp) x->len[p][size_t(sp) * nr + rp] = start;
            }
        // absolute offsets: a sender's buffer holds its segments to the receivers in receiver order, a
        // receiver's buffer its segments from the senders in sender order
        x->send_first[p].assign(size_t(nr) + 1, 0);
        x->recv_first[p].assign(size_t(nr) + 1, 0);
        x->loc_first[p].assign(size_t(nr) + 1, 0);
        for (int sp = 0; sp < nr; ++sp) {
            // segment of receiver rp inside sp's send buffer
            std::vector<int64_t> seg(size_t(nr), 0);
            int64_t acc = 0;
            for (int rp = 0; rp < nr; ++rp) {
                seg[rp] = acc;
                acc += x->len[p][size_t(sp) * nr + rp];
            }
            for (int rp = 0; rp < nr; ++rp)
                for (DevMsg d : incoming[rp][sp]) {
                    d.off += seg[rp];
                    x->send[p].push_back(d);
                }
            x->send_first[p][sp + 1] = int64_t(x->send[p].size());
        }
        for (int rp = 0; rp < nr; ++rp) {
            int64_t acc = 0;
            for (int sp = 0; sp < nr; ++sp) {
                for (DevMsg d : incoming[rp][sp]) {
                    d.off += acc;
                    x->recv[p].push_back(d);
                }
                acc += x->len[p][size_t(sp) * nr + rp];
            }
            x->recv_first[p][rp + 1] = int64_t(x->recv[p].size());
            for (const DevMsg &d : locv[rp]) x->loc[p].push_back(d);
            x->loc_first[p][rp + 1] = int64_t(x->loc[p].size());
        }
        // groups: within each process's range, messages ordered by their block (the sending block for
        // send, the receiving block otherwise) and cut into one group per block
        for (int kind = 0; kind < 3; ++kind) {
            std::vector<DevMsg> &v = kind == 0 ? x->send[p] : (kind == 1 ? x->recv[p] : x->loc[p]);
            const std::vector<int64_t> &first = kind == 0 ? x->send_first[p] : (kind == 1 ? x->recv_first[p] : x->loc_first[p]);
            auto key = [kind](const DevMsg &m) { return kind == 0 ? m.sender : m.r_local; };
            x->grp[p][kind].clear();
            x->grp_first[p][kind].assign(size_t(nr) + 1, 0);
            for (int r = 0; r < nr; ++r) {
                std::stable_sort(v.begin() + first[r], v.begin() + first[r + 1],
                                 [&](const DevMsg &a, const DevMsg &b) { return key(a) < key(b); });
                int32_t cells = 0;
                for (int64_t q = first[r]; q < first[r + 1]; ++q) {
                    if (q == first[r] || key(v[size_t(q)]) != key(v[size_t(q - 1)])) {
                        x->grp[p][kind].push_back(int32_t(q));
                        cells = 0;
                    }
                    v[size_t(q)].cfirst = cells;
                    cells += v[size_t(q)].ncell;
                }
                x->grp_first[p][kind][r + 1] = int64_t(x->grp[p][kind].size());
            }
            x->grp[p][kind].push_back(int32_t(v.size()));  // the end of the last group
        }
        // boundary ghosts after this pass: the process's blocks of level pass - 1 that touch a non-periodic
        // domain face, in local order
        x->bnd_first[p].assign(size_t(nr) + 1, 0);
        for (int rp = 0; rp < nr; ++rp) {
            for (int64_t q = x->blocks_first[rp]; q < x->blocks_first[rp + 1]; ++q) {
                const int b = x->blocks_local[size_t(q)];
                if (h.level[b] != p) continue;
                if (stage_mode && !psend[b]) continue;
                const bmhd_sim_desc &sd = h.sdesc[h.sim[b]];
                bool edge = false;
                for (int a = 0; a < 3; ++a) {
                    const int64_t n = int64_t(sd.nroot[a]) << h.level[b];
                    if (h.ijk[3 * b + a] == 0 && sd.bc[2 * a] != BMHD_BC_PERIODIC) edge = true;
                    if (h.ijk[3 * b + a] == n - 1 && sd.bc[2 * a + 1] != BMHD_BC_PERIODIC) edge = true;
                }
                if (edge) x->bnd_blocks[p].push_back(b);
            }
            x->bnd_first[p][rp + 1] = int64_t(x->bnd_blocks[p].size());
        }
    }
    // blocks whose interior the views need: all of them for complete views, else the senders
    x->int_first.assign(size_t(nr) + 1, 0);
    for (int r = 0; r < nr; ++r) {
        for (int64_t q = x->blocks_first[r]; q < x->blocks_first[r + 1]; ++q) {
            const int b = x->blocks_local[size_t(q)];
            if (!stage_mode || sends[b]) x->int_blocks.push_back(b);
        }
        x->int_first[r + 1] = int64_t(x->int_blocks.size());
    }
    // the message list in the counting order: sending process, pass, receiving process
    std::stable_sort(x->table.begin(), x->table.end(), [](const std::vector<int64_t> &a, const std::vector<int64_t> &b) {
        if (a[0] != b[0]) return a[0] < b[0];
        if (a[2] != b[2]) return a[2] < b[2];
        return a[1] < b[1];
    });
    // workspace layout: messages (send, recv, local per pass), boundary block lists with local indices,
    // the per-process block lists
    size_t off = 0;
    for (int p = 0; p < 2; ++p) {
        x->off_msgs[p][0] = off; off = align256(off + sizeof(DevMsg) * std::max<size_t>(1, x->send[p].size()));
        x->off_msgs[p][1] = off; off = align256(off + sizeof(DevMsg) * std::max<size_t>(1, x->recv[p].size()));
        x->off_msgs[p][2] = off; off = align256(off + sizeof(DevMsg) * std::max<size_t>(1, x->loc[p].size()));
        for (int kind = 0; kind < 3; ++kind) {
            x->off_grp[p][kind] = off;
            off = align256(off + sizeof(int32_t) * x->grp[p][kind].size());
        }
        x->off_bnd[p] = off; off = align256(off + 2 * sizeof(int32_t) * std::max<size_t>(1, x->bnd_blocks[p].size()));
    }
    x->off_blocks = off;
    off = align256(off + sizeof(int32_t) * std::max<size_t>(1, x->blocks_local.size()));
    x->off_split = off;
    off = align256(off + sizeof(int32_t) * std::max<size_t>(1, x->split.size()));
    x->off_local = off;
    off = align256(off + sizeof(int32_t) * std::max<size_t>(1, x->local.size()));
    x->off_fc = off;
    off = align256(off + sizeof(DevFcCell) * std::max<size_t>(1, x->fc.size()));
    x->off_vfaces = off;
    off = align256(off + sizeof(int32_t) * std::max<size_t>(1, x->view_faces.size()));
    x->off_int = off;
    off = align256(off + sizeof(int32_t) * std::max<size_t>(1, x->int_blocks.size()));
    x->work_bytes = off;
    *out = x;
    return BMHD_OK;
}
}  // namespace
}  // namespace bmhd

extern "C" {

void bmhd_xchg_destroy(bmhd_xchg *x) { delete x; }

int32_t bmhd_xchg_sizes(const bmhd_xchg *x, int32_t *h_nloc, int64_t *h_len, size_t *work_bytes) {
    if (!x) return set_last_error(BMHD_EINVAL, "null exchange");
    const int nr = x->nr;
    if (h_nloc)
        for (int r = 0; r < nr; ++r) h_nloc[r] = x->nloc[r];
    if (h_len)
        for (int p = 0; p < 2; ++p)
            for (size_t q = 0; q < size_t(nr) * nr; ++q) h_len[size_t(p) * nr * nr + q] = x->len[p][q];
    if (work_bytes) *work_bytes = x->work_bytes;
    return BMHD_OK;
}

int64_t bmhd_xchg_messages(const bmhd_xchg *x, int64_t *h_out, int64_t max_rows) {
    if (!x) return set_last_error(BMHD_EINVAL, "null exchange");
    const int64_t n = int64_t(x->table.size());
    if (!h_out) return n;
    if (max_rows < n) return set_last_error(BMHD_ENOMEM, "xchg_messages: output too small");
    for (int64_t q = 0; q < n; ++q) std::memcpy(h_out + q * 16, x->table[size_t(q)].data(), 16 * sizeof(int64_t));
    return n;
}

int32_t bmhd_xchg_upload(bmhd_xchg *x, void *d_work, size_t work_bytes, void *stream) {
    if (!x || !d_work || (reinterpret_cast<uintptr_t>(d_work) & 255u))
        return set_last_error(BMHD_EINVAL, "xchg_upload: null or misaligned workspace");
    if (work_bytes < x->work_bytes) return set_last_error(BMHD_ENOMEM, "xchg_upload: workspace too small");
    std::vector<unsigned char> blob(x->work_bytes, 0);
    auto put = [&](size_t at, const void *src, size_t n) { if (n) std::memcpy(blob.data() + at, src, n); };
    for (int p = 0; p < 2; ++p) {
        put(x->off_msgs[p][0], x->send[p].data(), sizeof(DevMsg) * x->send[p].size());
        put(x->off_msgs[p][1], x->recv[p].data(), sizeof(DevMsg) * x->recv[p].size());
        put(x->off_msgs[p][2], x->loc[p].data(), sizeof(DevMsg) * x->loc[p].size());
        for (int kind = 0; kind < 3; ++kind)
            put(x->off_grp[p][kind], x->grp[p][kind].data(), sizeof(int32_t) * x->grp[p][kind].size());
        std::vector<int32_t> bl(x->bnd_blocks[p].size() * 2);
        for (size_t q = 0; q < x->bnd_blocks[p].size(); ++q) {
            bl[q] = x->bnd_blocks[p][q];
            bl[x->bnd_blocks[p].size() + q] = x->local[x->bnd_blocks[p][q]];
        }
        put(x->off_bnd[p], bl.data(), sizeof(int32_t) * bl.size());
    }
    put(x->off_blocks, x->blocks_local.data(), sizeof(int32_t) * x->blocks_local.size());
    put(x->off_split, x->split.data(), sizeof(int32_t) * x->split.size());
    put(x->off_local, x->local.data(), sizeof(int32_t) * x->local.size());
    put(x->off_fc, x->fc.data(), sizeof(DevFcCell) * x->fc.size());
    put(x->off_vfaces, x->view_faces.data(), sizeof(int32_t) * x->view_faces.size());
    put(x->off_int, x->int_blocks.data(), sizeof(int32_t) * x->int_blocks.size());
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (int32_t rc = hip_ok(hipMemcpyAsync(d_work, blob.data(), x->work_bytes, hipMemcpyHostToDevice, s), "xchg upload"))
        return rc;
    if (int32_t rc = hip_ok(hipStreamSynchronize(s), "xchg upload sync")) return rc;
    x->d_work = d_work;
    return BMHD_OK;
}

int32_t bmhd_xchg_interior(const bmhd_xchg *x, int32_t r, const double *d_U, double *d_view, void *stream) {
    if (int32_t rc = need_xchg(x, 1, r)) return rc;
    const int n = x->nloc[r];
    if (n == 0) return BMHD_OK;  // a process without blocks has an empty view
    if (!aligned8(d_U) || !aligned8(d_view)) return set_last_error(BMHD_EINVAL, "xchg_interior: null or misaligned buffer");
    const int64_t ni = x->int_first[r + 1] - x->int_first[r];
    if (ni == 0) return BMHD_OK;
    const unsigned char *base = static_cast<const unsigned char *>(x->d_work);
    const auto *blocks = reinterpret_cast<const int32_t *>(base + x->off_int) + x->int_first[r];
    const auto *local = reinterpret_cast<const int32_t *>(base + x->off_local);
    k_xchg_interior<<<unsigned(ni), 512, 0, reinterpret_cast<hipStream_t>(stream)>>>(
        blocks, local, d_U, size_t(x->grid->h.nb) * 512, d_view, size_t(n) * 1728);
    return hip_ok(hipGetLastError(), "xchg interior");
}

int32_t bmhd_xchg_pack(const bmhd_xchg *x, int32_t pass, int32_t s, const double *d_view, double *d_send,
                       void *stream) {
    if (int32_t rc = need_xchg(x, pass, s)) return rc;
    const int p = pass - 1;
    const int64_t g0 = x->grp_first[p][0][s], ng = x->grp_first[p][0][s + 1] - g0;
    if (ng == 0) return BMHD_OK;
    if (!aligned8(d_view) || !aligned8(d_send)) return set_last_error(BMHD_EINVAL, "xchg_pack: null or misaligned buffer");
    const unsigned char *base = static_cast<const unsigned char *>(x->d_work);
    const auto *msgs = reinterpret_cast<const DevMsg *>(base + x->off_msgs[p][0]);
    const auto *grp = reinterpret_cast<const int32_t *>(base + x->off_grp[p][0]) + g0;
    const XView S{d_view, size_t(x->nloc[s]) * 1728};
    k_xchg_pack<<<unsigned(ng), 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(x->grid->h.dev, msgs, grp, S, d_send);
    return hip_ok(hipGetLastError(), "xchg pack");
}

int32_t bmhd_xchg_unpack(const bmhd_xchg *x, int32_t pass, int32_t r, const double *d_recv, double *d_view,
                         int32_t *d_bad, void *stream) {
    if (int32_t rc = need_xchg(x, pass, r)) return rc;
    if (x->nloc[r] == 0) return BMHD_OK;  // no blocks: nothing is sent to this process
    if (!aligned8(d_view)) return set_last_error(BMHD_EINVAL, "xchg_unpack: null or misaligned view");
    const int p = pass - 1;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const unsigned char *base = static_cast<const unsigned char *>(x->d_work);
    const size_t vs = size_t(x->nloc[r]) * 1728;
    const int64_t rg = x->grp_first[p][1][r], rn = x->grp_first[p][1][r + 1] - rg;
    if (rn) {
        if (!aligned8(d_recv)) return set_last_error(BMHD_EINVAL, "xchg_unpack: null or misaligned receive buffer");
        k_xchg_unpack<<<unsigned(rn), 256, 0, st>>>(reinterpret_cast<const DevMsg *>(base + x->off_msgs[p][1]),
                                                   reinterpret_cast<const int32_t *>(base + x->off_grp[p][1]) + rg,
                                                   d_recv, d_view, vs, d_bad);
    }
    const int64_t lg = x->grp_first[p][2][r], ln = x->grp_first[p][2][r + 1] - lg;
    if (ln)
        k_xchg_local<<<unsigned(ln), 256, 0, st>>>(x->grid->h.dev, reinterpret_cast<const DevMsg *>(base + x->off_msgs[p][2]),
                                                  reinterpret_cast<const int32_t *>(base + x->off_grp[p][2]) + lg,
                                                  d_view, vs);
    const int64_t bf = x->bnd_first[p][r], bn = x->bnd_first[p][r + 1] - bf;
    if (bn) {
        const auto *bl = reinterpret_cast<const int32_t *>(base + x->off_bnd[p]);
        const size_t nb_all = x->bnd_blocks[p].size();
        k_xchg_bounds<<<unsigned(bn), 256, 0, st>>>(x->grid->h.dev, bl + bf, bl + nb_all + bf, d_view, vs);
    }
    return hip_ok(hipGetLastError(), "xchg unpack");
}

int32_t bmhd_xchg_stage(const bmhd_xchg *x, int32_t r, int32_t stage, const double *d_view, const double *d_U0,
                        const double *d_Uin, double *d_Uout, const double *d_dt, const bmhd_opts *o,
                        int32_t *d_faults, void *stream) {
    if (int32_t rc = need_xchg(x, 1, r)) return rc;
    if (!o) return set_last_error(BMHD_EINVAL, "xchg_stage: null options");
    if (x->nloc[r] == 0) return BMHD_OK;  // no blocks, nothing to advance
    if (!aligned8(d_view) || !aligned8(d_U0) || !aligned8(d_Uin) || !aligned8(d_Uout) || !aligned8(d_dt))
        return set_last_error(BMHD_EINVAL, "xchg_stage: null or misaligned buffer");
    const ViewStage v = view_stage(x, r, d_view);
    return stage_from_view(x->grid->h, v, stage, d_U0, d_Uin, d_Uout, d_dt, *o, d_faults, stream);
}

int32_t bmhd_xchg_flux_correct(const bmhd_xchg *x, int32_t r, int32_t stage, double *d_Uout, const double *d_dt,
                               const bmhd_opts *o, int32_t *d_faults, void *stream) {
    if (int32_t rc = need_xchg(x, 1, r)) return rc;
    if (!o) return set_last_error(BMHD_EINVAL, "xchg_flux_correct: null options");
    if (x->fc_first[r + 1] == x->fc_first[r]) return BMHD_OK;
    if (!aligned8(d_Uout) || !aligned8(d_dt)) return set_last_error(BMHD_EINVAL, "xchg_flux_correct: null or misaligned buffer");
    const ViewStage v = view_stage(x, r, nullptr);
    return flux_correct_subset(x->grid->h, v, stage, d_Uout, d_dt, *o, d_faults, stream);
}

}  // extern "C"
