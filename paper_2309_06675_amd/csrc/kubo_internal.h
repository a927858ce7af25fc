// kubo_internal.h -- types shared by the host planner and the device kernels.
#pragma once

#include <cstdint>

namespace kubo {

constexpr int kMaxOrb = 512;
constexpr int kMaxFermi = 4096;
constexpr int kMaxSweeps = 30;

// Status bits written by the kernels into the workspace status word.
constexpr unsigned kStatNoConv = 1u;
constexpr unsigned kStatNonFinite = 2u;

// Per-model description on the device.
struct ModelDev {
    int n;           // orbitals
    int nR;          // lattice vectors
    int nR0;         // distinct R_x values
    int N0, N1, N2;  // grid
    int r0_first;    // first entry of this model in r0val[] (nR0 entries)
    int gs_first;    // first entry in grp_start[] (nR0 + 1 entries, relative to grp_first)
    int grp_first;   // first entry in grp_r/grp_R1/grp_R2 (nR entries, grouped by R_x)
    int neg_first;   // first entry in negr[] (nR entries): index of -R
    int f_off;       // offset of this model in e_fermi / sigma (model * n_fermi)
    int slot_first;  // first partial-sum slot (k-block) of the model
    int slot_count;  // number of slots
    int orb_off;     // offset of this model's orbitals in a per-orbital array (spin)
    long long t_off; // offset (complex elements) of the model in t / t' / grad_t
    long long Nk;    // full grid size (normaliser)
};

// One kx pencil (fixed i1, i2) of one model inside a chunk.
struct PencilItem {
    int model, i1, i2, pad;
    long long tbuf_off;  // complex offset of its T matrices in the chunk's T region
};

// One k-block: count consecutive i0 of one pencil.
struct BlockItem {
    int model, i0, count, slot;
    int i1, i2;
    int xfull;  // adjoint: 1 if its per-k matrices are stored whole, 0 if upper triangles only
    int pad1;
    long long tbuf_off;  // its pencil's T matrices (chunk-relative)
    long long pbuf_off;  // adjoint: its pencil-sum matrices (chunk-relative)
    long long xbuf_off;  // adjoint: its k-points' Hbar, vbar_x, vbar_y (chunk-relative;
                         // -1 in the forward)
};

constexpr int kMaxR0 = 16;  // distinct R_x values per model

// Up to kPencilGroup consecutive pencils of one model whose partial Bloch sums one
// workgroup forms together (each hopping read once for the group).
constexpr int kPencilGroup = 8;
struct PencilGroup {
    int first, count;
};

// A run of consecutive k-blocks of one model (the adjoint's transposed Bloch sum).
struct GaccRange {
    int model, begin, count, pad;
};

// Device pointers of the tables uploaded into the workspace.
struct Tables {
    const ModelDev* models;
    const int* r0val;
    const int* grp_start;
    const int* grp_r;
    const int* grp_R1;
    const int* grp_R2;
    const int* grp_rho;   // index of the R_x group of each grouped entry
    const int* negr;
    const PencilItem* pencils;
    const PencilGroup* pgroups;
    const BlockItem* blocks;
    const GaccRange* granges;
};

}  // namespace kubo
