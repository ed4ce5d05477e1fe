// Host-side FP64 generation of the per-material physics tables X(E) that the
// paper's VP engine reads from pre-computed databases (Methods A: energy
// loss, straggling, deflection and interaction probability; Methods B: the
// range-shifter and brass tables depend on energy only).  The tables are
// analytic: Bethe stopping power, CSDA range by Gauss-Legendre quadrature,
// Bohr straggling, a Gaussian scattering power and a nuclear removal
// coefficient.  They are rounded once to FP32 for the device.
#include <math.h>
#include <string.h>

#include <mutex>

#include "vpmc_internal.hpp"

namespace vpmc {

// Z/A, I (eV), X0 (g/cm^2), nuclear removal (cm^2/g, above 20 MeV), density.
// Brass: Cu/Zn 63/37 by mass; I by Bragg additivity of 322 and 330 eV; X0 from
// 1/X0 = sum w_i / X0_i with 12.86 and 12.43 g/cm^2.
const MaterialDef kMaterials[NMAT] = {
    {0.55508, 75.0, 36.08, 0.0115, 1.0},          // water
    {0.49919, 85.7, 36.62, 0.0110, 0.00120479},   // air
    {0.53937, 74.0, 40.55, 0.0112, 1.19},         // PMMA
    {0.457285, 324.947, 12.6975, 0.0075, 8.5},    // brass
    {0.52130, 106.4, 16.71, 0.0107, 1.85},        // cortical bone
};

namespace {

constexpr double kNA = 6.02214076e23;       // 1/mol
constexpr double kRe = 2.8179403262e-13;    // cm
constexpr double kMe = 0.51099895000;       // MeV
constexpr double kMp = 938.27208816;        // MeV
constexpr double kEs = 13.6;                // MeV, scattering-power constant
constexpr double kPi = 3.14159265358979323846;

double lorentz_beta2(double T) {
    const double gam = (T + kMp) / kMp;
    return (gam * gam - 1.0) / (gam * gam);
}

// electronic stopping power of a proton of kinetic energy T (MeV cm^2/g)
double bethe(const MaterialDef &m, double T) {
    const double K = 4.0 * kPi * kNA * kRe * kRe * kMe;
    const double gam = (T + kMp) / kMp;
    const double b2 = lorentz_beta2(T);
    const double bg2 = b2 * gam * gam;
    const double mr = kMe / kMp;
    const double wmax = 2.0 * kMe * bg2 / (1.0 + 2.0 * gam * mr + mr * mr);
    const double I = m.mean_exc_ev * 1.0e-6;
    const double logterm = 0.5 * log(2.0 * kMe * bg2 * wmax / (I * I));
    return K * m.z_over_a * (logterm - b2) / b2;
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n
void gauss_legendre(int n, double *x, double *w) {
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = cos(kPi * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

HostTables g_tables;
std::once_flag g_once;

void generate() {
    HostTables &t = g_tables;
    const double ratio = E_HI / E_LO;
    for (int i = 0; i < NE; ++i) t.E[i] = E_LO * exp(log(ratio) * i / (NE - 1.0));
    t.E[0] = E_LO;
    t.E[NE - 1] = E_HI;
    constexpr int NG = 24, NSUB = 4;
    double gx[NG], gw[NG];
    gauss_legendre(NG, gx, gw);
    for (int m = 0; m < NMAT; ++m) {
        const MaterialDef &mat = kMaterials[m];
        double acc = 0.0;
        t.R[m][0] = 0.0;
        for (int i = 1; i < NE; ++i) {
            const double a = t.E[i - 1], b = t.E[i], h = (b - a) / NSUB;
            double part = 0.0;
            for (int s = 0; s < NSUB; ++s) {
                const double lo = a + s * h, mid = lo + 0.5 * h;
                for (int g = 0; g < NG; ++g) part += gw[g] * 0.5 * h / bethe(mat, mid + 0.5 * h * gx[g]);
            }
            acc += part;
            t.R[m][i] = acc;
        }
        const double bohr = 4.0 * kPi * kNA * kRe * kRe * kMe * kMe;
        for (int i = 0; i < NE; ++i) {
            const double T = t.E[i];
            const double b2 = lorentz_beta2(T);
            t.W2[m][i] = bohr * mat.z_over_a * (1.0 - 0.5 * b2) / (1.0 - b2);
            const double pv = T * (T + 2.0 * kMp) / (T + kMp);
            t.T[m][i] = (kEs / pv) * (kEs / pv) / mat.rad_len_gcm2;
            double ramp = T <= 7.0 ? 0.0 : T >= 20.0 ? 1.0 : (T - 7.0) / 13.0;
            t.SN[m][i] = mat.nuc_coeff * ramp;
        }
    }
}

}  // namespace

const HostTables &host_tables() {
    std::call_once(g_once, generate);
    return g_tables;
}

// Device tables are per unit of (density x path length in mm), i.e. 10x the
// areal density in g/cm^2: a 1 mm step in water is then exactly 1.0 in FP32,
// whereas 0.1 g/cm^2 is not representable and would bias every step alike.
namespace {
// FP64 value as an unevaluated pair of FP32 (high part, rounded remainder)
void split_pair(double x, float *hi, float *lo) {
    *hi = (float)x;
    *lo = (float)(x - (double)*hi);
}
}  // namespace

void pack_device_tables(float *blob) {
    const HostTables &t = host_tables();
    memset(blob, 0, sizeof(float) * TAB_FLOATS);
    for (int i = 0; i < NE; ++i) {
        split_pair(t.E[i], blob + TAB_E + i, blob + TAB_EL + i);
        if (i + 1 < NE) split_pair(t.E[i + 1] - t.E[i], blob + TAB_DWH + i, blob + TAB_DWL + i);
    }
    for (int m = 0; m < NMAT; ++m) {
        float *b = blob + TAB_MAT0 + m * TAB_PER_MAT;
        float *bl = blob + TAB_LMAT0 + m * TAB_PER_LMAT;
        for (int i = 0; i < NE; ++i) {
            b[T_R * NE + i] = (float)(10.0 * t.R[m][i]);
            if (i + 1 < NE) {
                const double dR = 10.0 * (t.R[m][i + 1] - t.R[m][i]);
                split_pair((t.E[i + 1] - t.E[i]) / dR, b + T_SH * NE + i, bl + L_SL * NE + i);
                split_pair(dR, b + T_DH * NE + i, bl + L_DL * NE + i);
            }
            b[T_W2 * NE + i] = (float)(0.1 * t.W2[m][i]);
            b[T_T * NE + i] = (float)(0.1 * t.T[m][i]);
            b[T_SN * NE + i] = (float)(0.1 * t.SN[m][i]);
        }
    }
}

double range_host(int m, double E) {
    const HostTables &t = host_tables();
    if (E <= E_LO) return 0.0;
    int lo = 0, hi = NE - 1;
    if (E >= t.E[NE - 1]) lo = NE - 2;
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        (t.E[mid] <= E ? lo : hi) = mid;
    }
    return t.R[m][lo] + (E - t.E[lo]) * (t.R[m][lo + 1] - t.R[m][lo]) / (t.E[lo + 1] - t.E[lo]);
}

// Physical thickness of the PMMA range shifter: WET scaled by the ratio of
// areal CSDA ranges of PMMA and water at 150 MeV, divided by the density.
double rs_thickness_mm(double wet_mm) {
    const double rw = range_host(MAT_WATER, 150.0), rp = range_host(MAT_PMMA, 150.0);
    return wet_mm * (rp / kMaterials[MAT_PMMA].density) / (rw / kMaterials[MAT_WATER].density);
}

}  // namespace vpmc
