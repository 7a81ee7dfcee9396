// Pressure-equation assembly: the step before the solve in every SIMPLE
// iteration.  The paper ports it to the GPU with the rest of the application
// and profiles its pieces (Sec. 4.3: lduMatrix::negSumDiag, the face
// interpolation and divergence kernels; the pressure-assembly rows of the
// scaling tables, Sec. 4.4).  On the handle's mesh:
//   gamma_f = w_f gamma[own] + (1 - w_f) gamma[nb]   (linear interpolation)
//   upper_f = lower_f = gamma_f |S_f| delta_f         (Laplacian coefficients)
//   diag_i  = -(off-diagonal sum of column i) - diag_bc_i
//   b_i     = sum_{own(f)=i} phi_f - sum_{nb(f)=i} phi_f + b_bc_i
// Row i visits its faces in the face loop's order (those where it is the
// neighbour, by ascending owner, then those it owns, by ascending
// neighbour), so every sum is bitwise the serial face loop's.  No atomics.
#include "device.hpp"

namespace ldu {

__global__ void __launch_bounds__(kBlock)
k_asm_faces(int64_t nf, const int32_t *__restrict__ own, const int32_t *__restrict__ nb,
            const double *__restrict__ gamma, const double *__restrict__ w,
            const double *__restrict__ mag_sf, const double *__restrict__ delta,
            double *__restrict__ upper, double *__restrict__ lower) {
    for (int64_t f = blockIdx.x * (int64_t)kBlock + threadIdx.x; f < nf;
         f += (int64_t)gridDim.x * kBlock) {
        const double wf = w[f];
        const double gf = wf * gamma[own[f]] + (1.0 - wf) * gamma[nb[f]];
        const double c = gf * mag_sf[f] * delta[f];
        upper[f] = c;
        lower[f] = c;
    }
}

// per row: diag from the transposed values (column sums), and the divergence
// of phi (faces where the row is the neighbour are found in their owner's
// face range, which holds a handful of faces)
__global__ void __launch_bounds__(kBlock)
k_asm_rows(Sell A, const int64_t *__restrict__ own_start, const int32_t *__restrict__ fnb,
           const double *__restrict__ diag_bc, const double *__restrict__ phi,
           const double *__restrict__ b_bc, double *__restrict__ diag, double *__restrict__ b) {
    const int lane = threadIdx.x & 63;
    for_each_slice(A.nslices, [&](int64_t s) {
        const int64_t p = s * kWave + lane;
        if (p >= A.n) return;
        const int32_t i = A.perm ? A.perm[p] : (int32_t)p;
        const int w = row_len(A, p);
        double d = 0.0;
        for (int k = 0; k < w; ++k) d = d - A.valT[entry_at(A, p, k)];
        diag[i] = diag_bc ? d - diag_bc[i] : d;
        if (!b) return;  // phi is read only through faces, so it may be null without any
        double acc = 0.0;
        for (int k = 0; k < w; ++k) {
            const int32_t c = A.col[entry_at(A, p, k)];
            if (c >= i) continue;  // owners of the faces where i is the neighbour
            for (int64_t f = own_start[c]; f < own_start[c + 1]; ++f)
                if (fnb[f] == i) acc = acc - phi[f];
        }
        for (int64_t f = own_start[i]; f < own_start[i + 1]; ++f) acc = acc + phi[f];
        b[i] = b_bc ? acc + b_bc[i] : acc;
    });
}

void assemble_pressure(ldu_t *h, const double *gamma, const double *w, const double *mag_sf,
                       const double *delta, const double *diag_bc, const double *phi,
                       const double *b_bc, double *b, hipStream_t st) {
    Level &L = h->L0;
    const int G = stream_grid_slices(L.A.nslices);
    if (L.nf > 0) {
        int64_t g = (L.nf + kBlock - 1) / kBlock;
        g = g > 8192 ? 8192 : g;
        k_asm_faces<<<(unsigned)g, kBlock, 0, st>>>(L.nf, L.own, L.nb, gamma, w, mag_sf, delta,
                                                    L.upper, L.lower);
    }
    set_level_values(L, st);  // face values -> row values (val, valT)
    k_asm_rows<<<G, kBlock, 0, st>>>(L.A, L.ownStart, L.nb, diag_bc, phi, b_bc, L.diag, b);
    HIP_CHECK(hipGetLastError());
}

}  // namespace ldu
