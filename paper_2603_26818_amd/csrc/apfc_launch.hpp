// apfc_launch.hpp -- host-side view of the complex-amplitude kernels (apfc.hpp): their argument
// structures and launchers, one set per dtype.  Shapes are validated by the caller.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "types.hpp"

namespace pfc {

constexpr int kApfcMaxFields = 32;

// One product of the resonant nonlinearity of one field: coef * eta_a eta_b (* eta_c), with signed
// field indices s = +-(f + 1) (negative: the conjugate amplitude) and c = 0 for a pair.  The
// multiplicity of an unordered product among the ordered resonant tuples is folded into coef.
struct ApfcTerm {
    int16_t a, b, c, pad;
    float coef32;
    double coef;
};

// Arguments of the fused last-axis pass.  Pencil (field f, column col) has element e at
// f * fstride + e * ncols + col, col = k1 * nx + kx < ncols = n1 * nx.
template <typename T>
struct ApfcStepArgs {
    const cx<T> *src;  // FFT(N_f) along every other axis
    cx<T> *dst;        // inverse FFT along this axis of the new state (may be src)
    cx<T> *state;      // spectra of the amplitudes, updated in place
    int64_t ncols, nx, n1, fstride, tiles;  // tiles (column tiles per field) and W: set by the launcher
    int W;
    T fk[3];  // 2 pi / (n dx) per axis (axis 0, axis 1 (3D), x)
    T dt, dB, Bx;
    T kv[kApfcMaxFields][3];  // k_f along (axis 0, axis 1, x); axis 1 is 0 in 2D
    T kk[kApfcMaxFields];     // |k_f|^2
    const cx<T> *tw;
    int lt_shift;
};

// out_f = N_f at all P points of every field (nf fields of P points back to back): c3 (A^2 -
// |eta_f|^2) eta_f for the triples (f, i, -i), plus the products terms[off[f] .. off[f+1]) (device
// pointers).
template <typename T>
hipError_t launch_apfc_nonlin(const cx<T> *eta, cx<T> *out, int64_t P, int nf, const ApfcTerm *terms, const int *off,
                              double c3, hipStream_t s);

// FFT (dir -1 forward, +1 inverse) of nrows contiguous rows of length L, times scale.
template <typename T>
hipError_t launch_apfc_rows(int64_t L, const cx<T> *in, cx<T> *out, int64_t nrows, int dir, double scale, bool nt,
                            const cx<T> *tw, int lt_shift, hipStream_t s);

// Fused last-axis pass (length L) over nf fields.
template <typename T>
hipError_t launch_apfc_last_step(int64_t L, int nf, ApfcStepArgs<T> a, hipStream_t s);

}  // namespace pfc
