// Kernel bodies that run either as their own launch or inside the persistent executor.
//
// A body is a __device__ function of its kernel's parameters plus the coordinates of the workgroup
// in the body's grid (VBlk) and a pointer to the LDS it may use.  Its __global__ wrapper passes the
// hardware block coordinates and its own LDS; the persistent executor (solvers.hip) passes the
// coordinates of a virtual block of a recorded launch and a slice of its dynamic LDS.
//
// Recording: while a Recorder is installed on the calling host thread, the launch sites of the
// bodies listed in TaskKind append a TaskRec (which body, its grid, its dynamic LDS, its arguments)
// instead of launching.  The ground-state solver records one outer step this way and the persistent
// executor replays it.
#pragma once
#include <cstring>
#include <vector>

#include "nlf_internal.h"

namespace nlf {

struct VBlk {
    int x, y, z;
    int gx, gy, gz;
};

__device__ __forceinline__ VBlk hw_block() {
    return VBlk{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, (int)gridDim.x, (int)gridDim.y, (int)gridDim.z};
}

// Every body the persistent executor can run (its threads per workgroup are 256).
enum TaskKind : int {
    // FFT passes: potential (forward with the density load, inverse with the potential store) and
    // the solver's full transforms; _D / _F: FP64 / FP32 data
    TK_ROWS_RHO_D = 0, TK_ROWS_RHO_F,         // k_fft_rows, LOAD_RHO -> grid, forward
    TK_ROWS_U_D, TK_ROWS_U_DF,                // k_fft_rows, grid -> u (FP64 grid; u FP64 / FP32), inverse
    TK_ROWS_FWD_D, TK_ROWS_FWD_F, TK_ROWS_INV_D, TK_ROWS_INV_F,   // k_fft_rows, grid -> grid
    TK_COLS_PFWD_D, TK_COLS_PFWD_F,           // k_fft_cols, pruned load, forward
    TK_COLS_PINV_D,                           // k_fft_cols, pruned store, inverse (FP64 grid)
    TK_COLS_FWD_D, TK_COLS_FWD_F, TK_COLS_INV_D, TK_COLS_INV_F,   // k_fft_cols, full columns
    // NUFFT stencils at the default widths (msp 12 FP64, 7 FP32), gather lists, 128-candidate blocks
    TK_BINTERP_D, TK_BINTERP_F, TK_MSPREAD_D, TK_MSPREAD_F,
    // gradient-flow kernels
    TK_NORM2_D, TK_NORM2_F, TK_NORMALIZE_D, TK_NORMALIZE_F, TK_RESID_D, TK_RESID_F,
    TK_GFPREP_D, TK_GFPREP_F, TK_KIN_D, TK_KIN_F, TK_SHIFT, TK_PCGINIT_D, TK_PCGINIT_F, TK_BB,
    TK_RZ_D, TK_RZ_F, TK_DIR_D, TK_DIR_F, TK_APPLY_D, TK_APPLY_F, TK_UPDATE_D, TK_UPDATE_F, TK_CHECK,
    TK_TO_D,                                  // k_convert FP32 -> FP64 (mixed schedule switch)
    TK_COUNT
};

constexpr int kTaskArgBytes = 1024;
constexpr int kExecThreads = 256;
// Register budget of k_exec (launch bound: waves per SIMD) and resident executor workgroups per
// CU.  The executor holds the registers of its largest body (376 VGPRs at one wave per SIMD).
// Measured on 64 batched 2D ground states (ground states/s): 1/1 20.9, 2/1 20.7, 2/2 18.3,
// 4/2 14.0, 4/4 9.5: the grid barriers of more workgroups and the spills of a smaller budget cost
// more than the occupancy gains.
constexpr int kExecWavesPerEU = 1;
constexpr int kExecPerCU = 1;

struct TaskRec {
    int kind;
    int gx, gy, gz;
    int lds;                         // dynamic LDS bytes the body needs
    int pad[3];
    alignas(16) unsigned char args[kTaskArgBytes];
};

struct Recorder {
    std::vector<TaskRec> tasks;
    int failed = 0;                  // a launch without a body in TaskKind, or arguments too large
};

// the recorder installed on this host thread, or nullptr (launch directly)
Recorder*& recorder();

template <class A>
inline int record(Recorder* r, int kind, dim3 grid, size_t lds, const A& args) {
    static_assert(sizeof(A) <= kTaskArgBytes, "task arguments exceed the record size");
    TaskRec t{};
    t.kind = kind;
    t.gx = (int)grid.x;
    t.gy = (int)grid.y;
    t.gz = (int)grid.z;
    t.lds = (int)lds;
    std::memcpy(t.args, &args, sizeof(A));
    r->tasks.push_back(t);
    return NLF_OK;
}

}  // namespace nlf
