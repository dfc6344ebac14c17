// dg_basis.hpp -- compile-time description of the modal basis and the layout of the
// quadrature tables shared by the host set-up code and the gfx950 kernels.
//
// Basis (Sec. 2.1; total-degree truncation per the footnote of Sec. 3.2 and Sec. 7):
// phi_(a,b,c)(xi) = Lt_a(xi_1) Lt_b(xi_2) Lt_c(xi_3), Lt_n = sqrt(2n+1) P_n, a+b+c <= K,
// modes ordered by total degree ascending, then a descending, then b descending.
// Quadrature (Sec. 2.2, Sec. 7): K+1 Gauss-Legendre points per dimension for the
// volume (NQ = (K+1)^3 points) and for each face (NF = (K+1)^2 points).
#pragma once

namespace dg {

template <int K>
struct Shape {
    static constexpr int N1 = K + 1;
    static constexpr int NQ = N1 * N1 * N1;
    static constexpr int NF = N1 * N1;
    static constexpr int NB = (K + 1) * (K + 2) * (K + 3) / 6;
    static constexpr int NB2 = (K + 1) * (K + 2) / 2;   // modes of the 2D face basis
    static constexpr int ND = NB - NB2;                  // modes with a positive exponent along an axis
};

// tangential axes of a face normal to d (increasing order)
constexpr int tan1(int d) { return d == 0 ? 1 : 0; }
constexpr int tan2(int d) { return d == 2 ? 1 : 2; }

// position of the 2D exponent pair (p, q) in the graded 2D order (p+q ascending, p descending)
constexpr int idx2(int p, int q) { return (p + q) * (p + q + 1) / 2 + q; }

template <int K>
struct Modes {
    int e[Shape<K>::NB][3];     // exponents (a, b, c) of every mode
    int d2[3][Shape<K>::NB];    // 2D index of the tangential exponents on a face normal to d
    int dj[3][Shape<K>::NB];    // index among the modes with e[d] >= 1, or -1
    int p2[Shape<K>::NB2][2];   // exponent pair of every 2D mode
};

template <int K>
constexpr Modes<K> make_modes()
{
    Modes<K> M{};
    int m = 0;
    for (int n = 0; n <= K; ++n)
        for (int a = n; a >= 0; --a)
            for (int b = n - a; b >= 0; --b) {
                M.e[m][0] = a;
                M.e[m][1] = b;
                M.e[m][2] = n - a - b;
                ++m;
            }
    for (int d = 0; d < 3; ++d) {
        int j = 0;
        for (int l = 0; l < Shape<K>::NB; ++l) {
            M.d2[d][l] = idx2(M.e[l][tan1(d)], M.e[l][tan2(d)]);
            M.dj[d][l] = M.e[l][d] >= 1 ? j++ : -1;
        }
    }
    for (int n = 0; n <= K; ++n)
        for (int p = n; p >= 0; --p) {
            M.p2[idx2(p, n - p)][0] = p;
            M.p2[idx2(p, n - p)][1] = n - p;
        }
    return M;
}

// position of the mode with exponents (a, b, c) in the graded order
constexpr int idx3(int a, int b, int c)
{
    const int n = a + b + c;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + c;
}

// Derivative of a basis function along one axis in the basis itself: from
// P_n' = sum over j = n-1, n-3, ... >= 0 of (2j+1) P_j it follows that
// d/dxi Lt_n = sum_j sqrt((2n+1)(2j+1)) Lt_j, so d/dxi_d phi_e is a combination of the
// modes with e_d replaced by j; all of them have total degree < K.  The divergence of a
// degree-K vector field is therefore a degree-(K-1) polynomial with NDIV coefficients,
// the first NDIV modes of the graded order.
template <int K>
struct DivMap {
    static constexpr int NDIV = K * (K + 1) * (K + 2) / 6;
    static constexpr int MAXT = (K + 1) / 2;    // terms per derivative (j of the right parity)
    int m[3][Shape<K>::NB][MAXT];               // target mode, or -1
    int f[3][Shape<K>::NB][MAXT];               // (2n+1)(2j+1): the factor is its square root
};

template <int K>
constexpr DivMap<K> make_divmap()
{
    DivMap<K> D{};
    const Modes<K> M = make_modes<K>();
    for (int d = 0; d < 3; ++d)
        for (int l = 0; l < Shape<K>::NB; ++l) {
            int t = 0;
            for (int i = 0; i < DivMap<K>::MAXT; ++i) { D.m[d][l][i] = -1; D.f[d][l][i] = 0; }
            const int n = M.e[l][d];
            for (int j = n - 1; j >= 0; j -= 2) {
                int e[3] = {M.e[l][0], M.e[l][1], M.e[l][2]};
                e[d] = j;
                D.m[d][l][t] = idx3(e[0], e[1], e[2]);
                D.f[d][l][t] = (2 * n + 1) * (2 * j + 1);
                ++t;
            }
        }
    return D;
}

// Offsets (in elements) of the quadrature tables inside one contiguous device array.
template <int K>
struct TabLayout {
    using S = Shape<K>;
    static constexpr int VPHI = 0;                          // [NQ][NB]   phi_l at volume points
    static constexpr int VDPHI = VPHI + S::NQ * S::NB;      // [NQ][3][ND] dphi_l/dxi_d, modes with e_d >= 1
    static constexpr int VW = VDPHI + S::NQ * 3 * S::ND;    // [NQ]       product Gauss weights
    static constexpr int F2 = VW + S::NQ;                   // [NF][NB2]  2D basis at face points
    static constexpr int FW = F2 + S::NF * S::NB2;          // [NF]       face weights
    static constexpr int LEND = FW + S::NF;                 // [K+1][2]   Lt_n(-1), Lt_n(+1)
    static constexpr int VXI = LEND + 2 * (K + 1);          // [NQ][3]    reference coordinates
    static constexpr int PLIFT = VXI + 3 * S::NQ;           // [3][2][NF][NB] phi_l at the face points of
                                                            //   face (normal d, side s: 0 low, 1 high)
    static constexpr int WLT = PLIFT + 3 * 2 * S::NF * S::NB;  // [K+1][K+1] w_t Lt_a(xi_t): 1D weight times
                                                            //   the 1D basis of degree a at 1D point t
    static constexpr int SIZE = WLT + (K + 1) * (K + 1);
};

}  // namespace dg
