// bmhd_internal.h -- device-side table layout shared by the host grid builder (grid.cpp) and the
// HIP kernels (kernels.hip). Plain structs only; everything lives in one caller-owned workspace.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bmhd.h"

namespace bmhd {

constexpr int NB1 = 8;              // cells per block and axis
constexpr int NCELL = 512;          // cells per block
constexpr int NVAR = 8;
constexpr int NDIR = 26;

// Face relation codes in DevBlock::face (faces ordered x-lo, x-hi, y-lo, y-hi, z-lo, z-hi).
// >= 0: id of the equal-level neighbour (periodic wrap already applied).
constexpr int32_t FACE_OUTFLOW = -1;
constexpr int32_t FACE_INFLOW = -2;
constexpr int32_t FACE_LEVEL = -3;   // a different level: ghost layers come from the halo buffer

// DevBlock::flags
constexpr int32_t BF_NEAR_BODY = 1;  // the block or its face ghosts may contain body cells
constexpr int32_t BF_LEVEL = 2;      // at least one face borders a different level
constexpr int32_t BF_FC = 4;         // at least one face takes part in flux correction

struct DevBlock {
    int32_t sim, level;
    int32_t ijk[3];
    int32_t flags;
    int32_t face[6];       // relation per face (see above)
    int32_t halo_slot;     // slot in the halo buffer (BF_LEVEL), else -1
    int32_t fc_rec[6];     // flux-correction record per face, -1 if none
    int32_t fc_role;       // bit f: this block is the coarse side of face f's record
    int32_t fc_quad[6];    // fine side: quadrant (q1 + 2 q2) of the coarse face this block covers
    int32_t fc_skip;       // bit f: cells on face f are finished by the flux-correction kernel
    int32_t hb_pos[3];     // per direction d: index of the block's high face plane among those with no
                           // neighbour across them (learned correction's compact face layout), else -1
    int32_t pad[2];
};
static_assert(sizeof(DevBlock) == 128, "DevBlock layout");

struct DevSim {
    double origin[3];
    double dx0;
    double inflow_U[8];    // conserved inflow state
    double body_c[3];
    double body_r;         // <= 0: none
    int32_t nroot[3];
    int32_t bc[6];
    int32_t lut_off[2];    // offsets of the level-0 / level-1 block lookup tables in the lut array
    int32_t pad;
};
static_assert(sizeof(DevSim) == 176, "DevSim layout");

// One coarse cell that receives flux corrections from up to three coarse-fine faces.
struct DevFcCell {
    int32_t block, cell, n;
    int32_t rec[3];        // flux-correction record
    int32_t face[3];       // face number 0..5 of the coarse block
    int32_t t[3];          // t1 + 8 * t2 within the face
    int32_t pad[4];
};
static_assert(sizeof(DevFcCell) == 64, "DevFcCell layout");

// Flux record: coarse face fluxes [8 var][8 t2][8 t1] then fine fluxes [8 var][16 t2][16 t1].
constexpr int FC_COARSE = 8 * 64;
constexpr int FC_FINE = 8 * 256;
constexpr int FC_REC = FC_COARSE + FC_FINE;

// Halo buffer slot: [6 faces][8 var][2 layers][8 t2][8 t1] conserved values.
constexpr int HALO_FACE = 8 * 2 * 64;
constexpr int HALO_SLOT = 6 * HALO_FACE;

// Device view of the workspace (pointers into d_work), passed to kernels by value.
struct Tables {
    const DevBlock *blocks;
    const DevSim *sims;
    const int32_t *lut;
    const int32_t *order;       // Morton schedule of blocks
    const int32_t *order_split; // the same schedule, blocks clear of any body first (n_clear of them), then
                                // the blocks near a body
    const int32_t *halo_items;  // (block << 3) | face for every level face
    const DevFcCell *fc_cells;
    double *halo;               // [n_halo_slots][HALO_SLOT]
    double *fcbuf;              // [n_fc_rec][FC_REC]
    unsigned long long *lam;    // [n_sims] max of the dt bound (bit patterns of positive doubles)
    int32_t nb, ns, n_halo_items, n_fc_cells, n_clear;
};

// Host-side grid.
struct HostGrid {
    int32_t nb = 0, ns = 0;
    std::vector<int32_t> level, ijk, sim;
    std::vector<bmhd_sim_desc> sdesc;
    std::vector<DevBlock> blocks;
    std::vector<DevSim> sims;
    std::vector<int32_t> lut;
    std::vector<int32_t> order;
    std::vector<int32_t> order_split;
    int32_t n_clear = 0;        // blocks clear of any body (the first n_clear of order_split)
    int32_t n_clear_plain = 0;  // of those, the ones launched at once (with split_level: the ones with no
                                // face on another level, which come first; else all of them)
    bool split_level = false;   // the clear blocks at a level change are launched after the halo fill
    int32_t n_hb = 0;           // high face planes with no neighbour across them (see DevBlock::hb_pos)
    std::vector<int32_t> halo_items;
    std::vector<DevFcCell> fc_cells;
    int32_t n_halo_slots = 0, n_fc_rec = 0;
    std::vector<int32_t> nbr;   // [nb][26][5]
    // workspace layout (byte offsets)
    size_t off_blocks = 0, off_sims = 0, off_lut = 0, off_order = 0, off_order_split = 0, off_halo_items = 0,
           off_fc_cells = 0;
    size_t off_halo = 0, off_fcbuf = 0, off_lam = 0, work_bytes = 0, table_bytes = 0;
    std::vector<unsigned char> blob;  // packed tables (first table_bytes of the workspace)
    void *d_work = nullptr;
    Tables dev{};
    // cached HIP graph of one step (opaque hipGraph_t / hipGraphExec_t / hipStream_t) and its key
    void *graph = nullptr, *graph_exec = nullptr, *capture_stream = nullptr;
    std::vector<unsigned char> graph_key;
    // side stream (default priority) and fork / join events (hipStream_t / hipEvent_t) on which the
    // blocks near a body, and with split_level the halo fill and the blocks that read it, run beside the
    // block form's main launch; created on first use
    mutable void *side_stream = nullptr, *fork_event = nullptr, *join_event = nullptr;
};

int32_t build_grid(const bmhd_grid_desc *d, HostGrid &g, std::string &err);

// BF16 inference of the flux-correction MLP on inputs already rounded to BF16 ([n][32], 16-byte
// aligned), the same products as bmhd_mlp_forward in mode 0 on their FP32 originals; enqueued on stream.
int32_t mlp_infer_bf16_inputs(const float *d_params, const uint16_t *d_params_bf16, int32_t hidden, int32_t n,
                              const uint16_t *d_x, float *d_y, void *stream, std::string &err);
void prim_to_cons_host(const double *w, double *u);

// A subset of a grid's blocks (one process's) whose ghost cells come from a padded view filled by the
// ghost exchange between processes. All pointers are device pointers into the exchange's workspace or
// the caller's view.
struct ViewStage {
    const double *view;          // [8][n_local][12][12][12]
    const int32_t *view_local;   // [nb]: each block's index in its process's view
    const int32_t *view_faces;   // [nb]: bit f set where face f's ghost cells come from the view (a neighbour
                                 // on another process or level); the others are read in place
    int64_t view_vs;             // n_local * 1728
    const int32_t *split;        // the subset's blocks, those clear of any body first
    int32_t n_clear, n_total;
    const DevFcCell *fc_cells;   // the subset's coarse cells that take flux corrections
    int32_t n_fc;
};

// One stage of the two-stage scheme (stage e in {0, 1} of o's table) for the subset, and its flux
// corrections (to be enqueued after every process's stage kernels, which record the face fluxes).
int32_t stage_from_view(const HostGrid &h, const ViewStage &v, int e, const double *U0, const double *Uin,
                        double *Uout, const double *dt, const bmhd_opts &o, int32_t *faults, void *stream);
int32_t flux_correct_subset(const HostGrid &h, const ViewStage &v, int e, double *Uout, const double *dt,
                            const bmhd_opts &o, int32_t *faults, void *stream);

// Sets the message bmhd_last_error reports on this thread; returns code.
int32_t set_last_error(int32_t code, const std::string &msg);

}  // namespace bmhd

struct bmhd_grid {
    bmhd::HostGrid h;
    ~bmhd_grid();
};
