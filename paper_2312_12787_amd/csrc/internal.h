// internal.h -- data layout shared by the host runtime and the gfx950 kernels.
//
// Everything the kernels read lives in one caller-owned device buffer (the
// "geometry buffer"); GeomLayout holds the byte offset of each table.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace bemk {

constexpr int QMAX = 16;      // largest Gauss rule
constexpr int ROW_TILE = 256; // collocation rows per assembly workgroup
constexpr int COL_CHUNK = 32; // source elements per assembly workgroup
#ifndef ASM_NEAR_PART
#define ASM_NEAR_PART 4  // 2.24 ms against 2.36 ms at 8 and 2.51 ms at 16 (FP64 kite of 4096 elements)
#endif
constexpr int NEAR_PART = ASM_NEAR_PART;  // source elements per workgroup of the near-element launch
// |k r| below which the device Hankel evaluator uses the ascending series
// (FP64 and FP32 amplitude paths; the same values as in hankel_tables.h)
constexpr double XS_SERIES_F64 = 6.0, XS_SERIES_F32 = 4.0;
constexpr int MAX_DIRS = 4096;
// Largest Im k / Re k of a lossy medium: tan(10 degrees).
constexpr double MAX_TAN_ARG_K = 0.17632698070846498;

// One boundary element (128 bytes).  Normal = left normal of the travel
// direction a -> b.
struct ElemRec {
    double cx, cy;  // midpoint = collocation point
    double tx, ty;  // unit tangent (b - a) / h
    double nx, ny;  // unit normal (-ty, tx)
    double h;       // length |b - a|
    double ax, ay;  // first node
    double bx, by;  // second node
    double pad[5];
};

// Gauss points of one element and their weights (h/2) w_g.
struct GaussRec {
    double x[QMAX], y[QMAX], w[QMAX];
};

struct GaussRec32 {
    float x[QMAX], y[QMAX], w[QMAX];
};

// Inputs of a domain as given by the caller (complex numbers as re, im).
struct DomIn {
    double k[2];
    double bm[2];
    int has_bm;
    int pad;
};

struct GlobalIn {
    double alpha[2];
    double beta[2];
    int has_alpha, has_beta, form, n_dom;
};

// Derived per-domain constants (computed on the device).
struct DomConst {
    double k[2];     // wavenumber
    double eps[2];   // (k / k0)^2
    double c[2];     // Burton-Miller coefficient alpha / eps (or the caller's)
    double beta[2];  // scaling of the standard-type rows
    int cplx;        // Im k != 0
    int pad;
};

// Per-wavenumber constants of the device Hankel evaluator (hankel_dev.h): the
// polynomial coefficients are compile-time constants, the wavenumber enters
// through the arguments w = (XS/k)^2 / r^2 and t = (k/2)^2 r^2.
struct WaveConst {
    double kr, ki;
    double r2_small;            // (XS / |k|)^2: below it the ascending series
    double wr, wi;              // (XS / k)^2
    double ur, ui;              // XS / k
    double a0r, a0i, a1r, a1i;  // sqrt(2/(pi k)) e^{-i pi/4}, sqrt(2/(pi k)) e^{-3 i pi/4}
    double tr, ti;              // (k / 2)^2
    double hr, hi;              // k / 2
    double lkr, lki;            // ln(k / 2)
    double y1r, y1i;            // -2 / (pi k)
    double ampr, ampi;          // sqrt(2 / (pi k))
    double rs;                  // XS / |k|: the ascending series below this distance
    double rs32;                // the same for the FP32 amplitude evaluation (WaveConst32)
};

// FP32 amplitude evaluation (|k r| >= 4); the series below it runs in FP64.
struct WaveConst32 {
    float r2_small;
    float wr, wi, ur, ui;
    float a0r, a0i, a1r, a1i;
    float ampr, ampi;  // sqrt(2 / (pi k))
};

// Interface plan (host-computed integer bookkeeping).
struct IfacePlan {
    int off, count;   // element range
    int dl, dr;       // domain the normal enters / leaves
    int bm_r;         // the dom_right equation is of Burton-Miller type
    int row_l, row_r; // first row of the dom_left / dom_right equation block
    int pad;
};

// A tile of consecutive elements of one interface.
struct Tile {
    int iface, start, count, pad;
};

struct GeomLayout {
    size_t nodes, elnodes, elem, gauss, gauss32, gl, dom_in, glob_in, dom, wave, wave32, self,
        iface, rtiles, cchunks, sigma, elif, vtiles, npairs, total;
};

}  // namespace bemk
