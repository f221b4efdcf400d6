// Host-side building blocks of the FWI library shared by the single-problem
// entry points (fwi_host.cpp) and the batched plans (fwi_batch.cpp):
// validation, workspace layout, pointers into the workspace, geometry
// upload and the argument blocks of the stencil kernels.  Internal; not
// part of the C ABI.
#pragma once

#include "fwi.h"
#include "fwi_internal.h"

namespace fwi {
namespace host {

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Validate the grid and geometry and derive the dimensions (FWI_* status).
int make_dims(const fwi_grid *grid, const fwi_geom *geom, Dims &d);
// Checkpoint interval minimising checkpoint plus segment-buffer memory.
int stream_depth(const Dims &d);
int choose_k(const Dims &d, int depth);
// Row bands of the streaming decomposition (stored in L); `groups` shot
// groups share the chip.
void make_tiling(const Dims &d, Layout &L, int groups = 1);
// Row bands of height `rows` for both kernels (batched plans).
void fixed_bands(Layout &L, int rows, int depth);
// Workspace layout for a save mode (-1: fwi_gradient); k > 0 forces the
// checkpoint interval (a multiple of the streaming depth).  With `shared`,
// one shot group's layout from byte `start` (see make_group_layout).
int make_layout(const Dims &d, int mode, Layout &L, int k = 0, int depth = 0, size_t start = 0,
                const Layout *shared = nullptr, int s0 = 0);

// A gradient's shots in G groups run concurrently (fwi_host.cpp).
constexpr int kMaxShotGroups = 4;
struct GroupLayout {
    int G;
    int s0[kMaxShotGroups + 1];   // first shot of each group, then S
    Layout shared;                // arrays shared by the groups (all S shots)
    Layout grp[kMaxShotGroups];
    size_t total;
};
int make_group_layout(const Dims &d, int G, GroupLayout &GL);
int auto_shot_groups(const Dims &d);
int gradient_workspace(const Dims &d, size_t &bytes);

// Pointers into the workspace.
struct Ptrs {
    char *base;
    const Layout *L;
    float *f(size_t off) const { return reinterpret_cast<float *>(base + off); }
    int *i(size_t off) const { return reinterpret_cast<int *>(base + off); }
    Profiles prof() const {
        const Dims &d = L->d;
        float *p = f(L->off_prof);
        Profiles q;
        q.bEx = p; q.aEx = p + d.NX; q.kEx = p + 2 * d.NX;
        q.bHx = p + 3 * d.NX; q.aHx = p + 4 * d.NX; q.kHx = p + 5 * d.NX;
        float *y = p + 6 * d.NX;
        q.bEy = y; q.aEy = y + d.NY; q.kEy = y + 2 * d.NY;
        q.bHy = y + 3 * d.NY; q.aHy = y + 4 * d.NY; q.kHy = y + 5 * d.NY;
        return q;
    }
    // A State laid out at `off`: [E][Hx][Hy][phx][phy][pex][pey] (E only when
    // with_e).
    State state(size_t off, bool with_e) const {
        const Dims &d = L->d;
        const size_t S = (size_t)d.S;
        const size_t field = align_up(S * d.plane * sizeof(float));
        const size_t xs = align_up(S * d.xs * sizeof(float));
        const size_t ys = align_up(S * d.ys * sizeof(float));
        State st;
        size_t o = off;
        st.E = nullptr;
        if (with_e) { st.E = f(o); o += field; }
        st.Hx = f(o); o += field;
        st.Hy = f(o); o += field;
        st.phx = f(o); o += ys;
        st.phy = f(o); o += xs;
        st.pex = f(o); o += xs;
        st.pey = f(o);
        return st;
    }
    float *slot(int k) const {
        const Dims &d = L->d;
        return f(L->off_slots) + (size_t)k * d.S * d.plane;
    }
};

#define FWI_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return FWI_EHIP;          \
    } while (0)

// Geometry tables, band table and cold arguments to the workspace (waits for
// the copies, so the host arrays may be released on return).
int upload_geometry(const Ptrs &P, const fwi_geom *g, const StreamCold &cold, hipStream_t st);
int zero_state(const State &s, const Dims &d, bool with_e, hipStream_t st);
int copy_state(const State &dst, const State &src, const Dims &d, hipStream_t st);
Tiling tiling(const Ptrs &P);       // forward kernel
Tiling tiling_adj(const Ptrs &P);   // adjoint kernel
StreamCold make_cold(const Ptrs &P, const fwi_geom *g, float *traces, const float *residual,
                     float *src_adjoint);
FwdStreamArgs fwd_args(const Ptrs &P);
AdjStreamArgs adj_args(const Ptrs &P);

}  // namespace host
}  // namespace fwi
