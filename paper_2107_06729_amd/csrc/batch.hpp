// Job-table launches of a batch of meshes: one kernel per pass of a step
// (per FFT length for the FFT passes) covers the mesh groups of a batch,
// one workgroup per entry of a job table of (mesh group, tile) entries.
// The arguments of each group are the ones the single-mesh launchers take
// (kernels.hpp); batch.hip turns them into job ranges.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "kernels.hpp"

namespace llgx {

constexpr int BMAX = 4;  // mesh groups per job-table launch

enum BatchKind { BK_XFWD, BK_COL, BK_ZMUL, BK_XINV, BK_EPOLY, BK_STAGE, BK_STAGE_FINAL, BK_COMBINE, BK_FINAL };

// Per-group arguments (spectra in the working precision; scales 1).  `jobs`
// and the tile counts are filled in by launch_batch.
template <typename T>
struct BXfwd {
    Combo<T> in;
    T* mk_out;
    int nin;
    long nrows;
    cx<T>* spec;
    int SX;
    const cx<T>* twL;
    const cx<T>* twP;
    int LX;
    int jobs;
};
template <typename T>
struct BCol {
    const cx<T>* src;
    long s_cs, s_os, s_is;
    int n_in;
    cx<T>* dst;
    long d_cs, d_os, d_is;
    int n_out, Kx;
    const cx<T>* tw;
    int L, nouter, ncomp;
    int ntx, jobs;
};
template <typename T>
struct BZmul {
    cx<T>* buf;
    int SX, Kx, nz, nyrows, Py, nb;
    const T* kfold;
    const cx<T>* tw;
    int LZ;
    int ntile, nq, jobs;
};
template <typename T>
struct BXinv {  // XINV_RHS
    const cx<T>* spec;
    int SX;
    const T* M;
    Phys<T> ph;
    XinvOut out;
    const cx<T>* twL;
    const cx<T>* twP;
    int LX;
    int gx, jobs;
};
template <typename T>
struct BEpoly {
    EPoly<T> ep;
    long n;
    int vec, nblk, jobs;
};
template <typename T>
struct BStage {
    Combo<T> mk;
    Extrap<T> ex;
    Phys<T> ph;
    T* F;
    NextStage<T> nx;
    int tx, ry, gx, gy, jobs;
};
template <typename T>
struct BStageFinal {
    Combo<T> mk;
    Extrap<T> ex;
    Phys<T> ph;
    const T* M0;
    Final<T> fs;
    double inv_ms;
    T* mnew;
    double* parts;
    int tx, ry, gx, gy, jobs;
};
template <typename T>
struct BCombine {
    Combo<T> c;
    T* out;
    long n;
    int vec, nblk, jobs;
};
template <typename T>
struct BFinal {
    long ncell;
    int nb;
    const T* base;
    Final<T> fs;
    double inv_ms;
    T* mnew;
    double* parts;
    int nblk, jobs;
};

// job table of one launch: jobs start[g] .. start[g] + g[g].jobs - 1
// belong to group g (start[g] is a multiple of 8, so a job's XCD is its
// index within the group modulo 8, as in the single-mesh kernels)
template <typename A>
struct BJobs {
    A g[BMAX];
    int start[BMAX + 1];
    int ng;
};

// A prepared job-table launch: its job table is copied into device memory
// (at `offset` of a buffer the caller owns) before enqueue_batch launches
// the kernel with a pointer to it, so the launch can be captured into a
// graph.
struct BatchLaunch {
    int kind, nf;
    unsigned grid;   // workgroups: one per job and padding slot
    size_t offset;   // of the job table in the table buffer
    const void* fn;  // the kernel (its one argument: the job table)
};

// launch b on stream s with its job table at table_dev (device memory that
// outlives the launch)
hipError_t enqueue_batch(const BatchLaunch& b, const void* table_dev, hipStream_t s);

// The FFT length a group's launch of kind `kind` is built for (its B*
// struct at arg): groups of one launch share it; -1 when the group has no
// jobs in that launch (a column pass of a one-row mesh); 0 for the per-cell
// kinds.
template <typename T>
int batch_instance(int kind, const void* arg);

// Build the launch of kind `kind` over the groups whose arguments args[g]
// point to (the B* struct of the kind, in the working precision T); nf is
// the template count of the kind (Eq. (4) terms, Eq. (6) nodes, Eq. (3)
// derivatives; for BK_COL 0 forward, 1 inverse).  At most BMAX groups, all
// of one batch_instance.  The job table is appended to `blob` (256-byte
// aligned).  hipErrorInvalidValue when a group is outside what the
// job-table kernels are built for.
template <typename T>
hipError_t prepare_batch(int kind, int nf, const std::vector<const void*>& args, std::vector<unsigned char>& blob,
                         BatchLaunch& out);

}  // namespace llgx
