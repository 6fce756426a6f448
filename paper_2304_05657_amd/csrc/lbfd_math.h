#pragma once
// lbfd_math.h -- double-precision reciprocal, exponential and logarithm of
// the chemistry (gfx950 device code).  Self-contained (it includes only the
// HIP runtime header, which the run-time compiler does not need): the
// library's kernels include it, and the mechanism-specialised chemistry
// kernels compiled at run time are given its text.
#ifndef __HIPCC_RTC__  // (the run-time compiler provides the HIP device API itself)
#include <hip/hip_runtime.h>
#endif

namespace lbfd {

// ------------------------------------------------------------ reciprocal
// 1/x for a positive normal x (densities, temperatures, WENO denominators):
// the hardware estimate, refined in double precision by two Newton-Raphson
// steps r <- r + r (1 - x r), each of which doubles the correct bits (the
// step sequence of the compiler's own division, without the scaling and
// fix-up it needs near the ends of the exponent range); the single-precision
// estimate is already within 1 ulp.
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ------------------------------------------------------------ exponential
// 2^(j/256), j = 0..255, each the double nearest to the exact value
// (computed with 60-digit decimal arithmetic).
constexpr int kExpTabN = 256;
static __constant__ double kExp2Tab[kExpTabN] = {
    0x1.0000000000000p+0, 0x1.00b1afa5abcbfp+0, 0x1.0163da9fb3335p+0, 0x1.02168143b0281p+0,
    0x1.02c9a3e778061p+0, 0x1.037d42e11bbccp+0, 0x1.04315e86e7f85p+0, 0x1.04e5f72f654b1p+0,
    0x1.059b0d3158574p+0, 0x1.0650a0e3c1f89p+0, 0x1.0706b29ddf6dep+0, 0x1.07bd42b72a836p+0,
    0x1.0874518759bc8p+0, 0x1.092bdf66607e0p+0, 0x1.09e3ecac6f383p+0, 0x1.0a9c79b1f3919p+0,
    0x1.0b5586cf9890fp+0, 0x1.0c0f145e46c85p+0, 0x1.0cc922b7247f7p+0, 0x1.0d83b23395decp+0,
    0x1.0e3ec32d3d1a2p+0, 0x1.0efa55fdfa9c5p+0, 0x1.0fb66affed31bp+0, 0x1.1073028d7233ep+0,
    0x1.11301d0125b51p+0, 0x1.11edbab5e2ab6p+0, 0x1.12abdc06c31ccp+0, 0x1.136a814f204abp+0,
    0x1.1429aaea92de0p+0, 0x1.14e95934f312ep+0, 0x1.15a98c8a58e51p+0, 0x1.166a45471c3c2p+0,
    0x1.172b83c7d517bp+0, 0x1.17ed48695bbc0p+0, 0x1.18af9388c8deap+0, 0x1.1972658375d2fp+0,
    0x1.1a35beb6fcb75p+0, 0x1.1af99f8138a1cp+0, 0x1.1bbe084045cd4p+0, 0x1.1c82f95281c6bp+0,
    0x1.1d4873168b9aap+0, 0x1.1e0e75eb44027p+0, 0x1.1ed5022fcd91dp+0, 0x1.1f9c18438ce4dp+0,
    0x1.2063b88628cd6p+0, 0x1.212be3578a819p+0, 0x1.21f49917ddc96p+0, 0x1.22bdda27912d1p+0,
    0x1.2387a6e756238p+0, 0x1.2451ffb82140ap+0, 0x1.251ce4fb2a63fp+0, 0x1.25e85711ece75p+0,
    0x1.26b4565e27cddp+0, 0x1.2780e341ddf29p+0, 0x1.284dfe1f56381p+0, 0x1.291ba7591bb70p+0,
    0x1.29e9df51fdee1p+0, 0x1.2ab8a66d10f13p+0, 0x1.2b87fd0dad990p+0, 0x1.2c57e39771b2fp+0,
    0x1.2d285a6e4030bp+0, 0x1.2df961f641589p+0, 0x1.2ecafa93e2f56p+0, 0x1.2f9d24abd886bp+0,
    0x1.306fe0a31b715p+0, 0x1.31432edeeb2fdp+0, 0x1.32170fc4cd831p+0, 0x1.32eb83ba8ea32p+0,
    0x1.33c08b26416ffp+0, 0x1.3496266e3fa2dp+0, 0x1.356c55f929ff1p+0, 0x1.36431a2de883bp+0,
    0x1.371a7373aa9cbp+0, 0x1.37f26231e754ap+0, 0x1.38cae6d05d866p+0, 0x1.39a401b7140efp+0,
    0x1.3a7db34e59ff7p+0, 0x1.3b57fbfec6cf4p+0, 0x1.3c32dc313a8e5p+0, 0x1.3d0e544ede173p+0,
    0x1.3dea64c123422p+0, 0x1.3ec70df1c5175p+0, 0x1.3fa4504ac801cp+0, 0x1.40822c367a024p+0,
    0x1.4160a21f72e2ap+0, 0x1.423fb2709468ap+0, 0x1.431f5d950a897p+0, 0x1.43ffa3f84b9d4p+0,
    0x1.44e086061892dp+0, 0x1.45c2042a7d232p+0, 0x1.46a41ed1d0057p+0, 0x1.4786d668b3237p+0,
    0x1.486a2b5c13cd0p+0, 0x1.494e1e192aed2p+0, 0x1.4a32af0d7d3dep+0, 0x1.4b17dea6db7d7p+0,
    0x1.4bfdad5362a27p+0, 0x1.4ce41b817c114p+0, 0x1.4dcb299fddd0dp+0, 0x1.4eb2d81d8abffp+0,
    0x1.4f9b2769d2ca7p+0, 0x1.508417f4531eep+0, 0x1.516daa2cf6642p+0, 0x1.5257de83f4eefp+0,
    0x1.5342b569d4f82p+0, 0x1.542e2f4f6ad27p+0, 0x1.551a4ca5d920fp+0, 0x1.56070dde910d2p+0,
    0x1.56f4736b527dap+0, 0x1.57e27dbe2c4cfp+0, 0x1.58d12d497c7fdp+0, 0x1.59c0827ff07ccp+0,
    0x1.5ab07dd485429p+0, 0x1.5ba11fba87a03p+0, 0x1.5c9268a5946b7p+0, 0x1.5d84590998b93p+0,
    0x1.5e76f15ad2148p+0, 0x1.5f6a320dceb71p+0, 0x1.605e1b976dc09p+0, 0x1.6152ae6cdf6f4p+0,
    0x1.6247eb03a5585p+0, 0x1.633dd1d1929fdp+0, 0x1.6434634ccc320p+0, 0x1.652b9febc8fb7p+0,
    0x1.6623882552225p+0, 0x1.671c1c70833f6p+0, 0x1.68155d44ca973p+0, 0x1.690f4b19e9538p+0,
    0x1.6a09e667f3bcdp+0, 0x1.6b052fa75173ep+0, 0x1.6c012750bdabfp+0, 0x1.6cfdcddd47645p+0,
    0x1.6dfb23c651a2fp+0, 0x1.6ef9298593ae5p+0, 0x1.6ff7df9519484p+0, 0x1.70f7466f42e87p+0,
    0x1.71f75e8ec5f74p+0, 0x1.72f8286ead08ap+0, 0x1.73f9a48a58174p+0, 0x1.74fbd35d7cbfdp+0,
    0x1.75feb564267c9p+0, 0x1.77024b1ab6e09p+0, 0x1.780694fde5d3fp+0, 0x1.790b938ac1cf6p+0,
    0x1.7a11473eb0187p+0, 0x1.7b17b0976cfdbp+0, 0x1.7c1ed0130c132p+0, 0x1.7d26a62ff86f0p+0,
    0x1.7e2f336cf4e62p+0, 0x1.7f3878491c491p+0, 0x1.80427543e1a12p+0, 0x1.814d2add106d9p+0,
    0x1.82589994cce13p+0, 0x1.8364c1eb941f7p+0, 0x1.8471a4623c7adp+0, 0x1.857f4179f5b21p+0,
    0x1.868d99b4492edp+0, 0x1.879cad931a436p+0, 0x1.88ac7d98a6699p+0, 0x1.89bd0a478580fp+0,
    0x1.8ace5422aa0dbp+0, 0x1.8be05bad61778p+0, 0x1.8cf3216b5448cp+0, 0x1.8e06a5e0866d9p+0,
    0x1.8f1ae99157736p+0, 0x1.902fed0282c8ap+0, 0x1.9145b0b91ffc6p+0, 0x1.925c353aa2fe2p+0,
    0x1.93737b0cdc5e5p+0, 0x1.948b82b5f98e5p+0, 0x1.95a44cbc8520fp+0, 0x1.96bdd9a7670b3p+0,
    0x1.97d829fde4e50p+0, 0x1.98f33e47a22a2p+0, 0x1.9a0f170ca07bap+0, 0x1.9b2bb4d53fe0dp+0,
    0x1.9c49182a3f090p+0, 0x1.9d674194bb8d5p+0, 0x1.9e86319e32323p+0, 0x1.9fa5e8d07f29ep+0,
    0x1.a0c667b5de565p+0, 0x1.a1e7aed8eb8bbp+0, 0x1.a309bec4a2d33p+0, 0x1.a42c980460ad8p+0,
    0x1.a5503b23e255dp+0, 0x1.a674a8af46052p+0, 0x1.a799e1330b358p+0, 0x1.a8bfe53c12e59p+0,
    0x1.a9e6b5579fdbfp+0, 0x1.ab0e521356ebap+0, 0x1.ac36bbfd3f37ap+0, 0x1.ad5ff3a3c2774p+0,
    0x1.ae89f995ad3adp+0, 0x1.afb4ce622f2ffp+0, 0x1.b0e07298db666p+0, 0x1.b20ce6c9a8952p+0,
    0x1.b33a2b84f15fbp+0, 0x1.b468415b749b1p+0, 0x1.b59728de5593ap+0, 0x1.b6c6e29f1c52ap+0,
    0x1.b7f76f2fb5e47p+0, 0x1.b928cf22749e4p+0, 0x1.ba5b030a1064ap+0, 0x1.bb8e0b79a6f1fp+0,
    0x1.bcc1e904bc1d2p+0, 0x1.bdf69c3f3a207p+0, 0x1.bf2c25bd71e09p+0, 0x1.c06286141b33dp+0,
    0x1.c199bdd85529cp+0, 0x1.c2d1cd9fa652cp+0, 0x1.c40ab5fffd07ap+0, 0x1.c544778fafb22p+0,
    0x1.c67f12e57d14bp+0, 0x1.c7ba88988c933p+0, 0x1.c8f6d9406e7b5p+0, 0x1.ca3405751c4dbp+0,
    0x1.cb720dcef9069p+0, 0x1.ccb0f2e6d1675p+0, 0x1.cdf0b555dc3fap+0, 0x1.cf3155b5bab74p+0,
    0x1.d072d4a07897cp+0, 0x1.d1b532b08c968p+0, 0x1.d2f87080d89f2p+0, 0x1.d43c8eacaa1d6p+0,
    0x1.d5818dcfba487p+0, 0x1.d6c76e862e6d3p+0, 0x1.d80e316c98398p+0, 0x1.d955d71ff6075p+0,
    0x1.da9e603db3285p+0, 0x1.dbe7cd63a8315p+0, 0x1.dd321f301b460p+0, 0x1.de7d5641c0658p+0,
    0x1.dfc97337b9b5fp+0, 0x1.e11676b197d17p+0, 0x1.e264614f5a129p+0, 0x1.e3b333b16ee12p+0,
    0x1.e502ee78b3ff6p+0, 0x1.e653924676d76p+0, 0x1.e7a51fbc74c83p+0, 0x1.e8f7977cdb740p+0,
    0x1.ea4afa2a490dap+0, 0x1.eb9f4867cca6ep+0, 0x1.ecf482d8e67f1p+0, 0x1.ee4aaa2188510p+0,
    0x1.efa1bee615a27p+0, 0x1.f0f9c1cb6412ap+0, 0x1.f252b376bba97p+0, 0x1.f3ac948dd7274p+0,
    0x1.f50765b6e4540p+0, 0x1.f6632798844f8p+0, 0x1.f7bfdad9cbe14p+0, 0x1.f91d802243c89p+0,
    0x1.fa7c1819e90d8p+0, 0x1.fbdba3692d514p+0, 0x1.fd3c22b8f71f1p+0, 0x1.fe9d96b2a23d9p+0,
};

// exp(x) by table-driven argument reduction (P. T. P. Tang, Table-driven
// implementation of the exponential function in IEEE floating-point
// arithmetic, ACM TOMS 15, 1989): x = (256 m + j) ln2/256 + r,
// |r| <= ln2/512, with ln2/256 split into a 33-bit head (n times it is exact
// for |n| < 2^20) and a tail; exp(x) = 2^m 2^(j/256) (1 + p(r)), p the
// degree-4 Taylor polynomial of exp(r) - 1 (truncation below 4e-17
// relative).  About one ulp from the correctly rounded value; x is clamped
// to [-1000, 1000] (exp underflows to 0 and overflows to infinity well
// inside it).  `tab` holds kExp2Tab (in LDS in the chemistry launches, the
// constant table elsewhere).
__device__ __forceinline__ double exp_tab(double x, const double *tab)
{
    constexpr double kInvLn2_256 = 0x1.71547652b82fep+8;   // 256 / ln 2
    constexpr double kLn2_256_hi = 0x1.62e42fee00000p-9;   // ln 2 / 256, head
    constexpr double kLn2_256_lo = 0x1.a39ef35793c76p-41;  // and tail
    x = fmin(fmax(x, -1000.0), 1000.0);
    const double n = __builtin_rint(x * kInvLn2_256);
    const double r = fma(-n, kLn2_256_lo, fma(-n, kLn2_256_hi, x));
    const int ni = (int)n;
    double p = fma(r, 1.0 / 24.0, 1.0 / 6.0);
    p = fma(r, p, 0.5);
    p = fma(r, p, 1.0);
    p *= r;
    const double t = tab[ni & (kExpTabN - 1)];
    return __builtin_ldexp(fma(t, p, t), ni >> 8);
}

// ------------------------------------------------------------ logarithm
// 1/F_j and ln F_j for F_j = 1 + j/256, j = 0..255, interleaved (1/F_j at
// 2 j, ln F_j at 2 j + 1), each the double nearest to the exact value
// (computed with 60-digit decimal arithmetic).
constexpr int kLogTabN = 256;
static __constant__ double kLogTab[2 * kLogTabN] = {
    0x1.0000000000000p+0, 0.0, 0x1.fe01fe01fe020p-1, 0x1.ff00aa2b10bc0p-9,
    0x1.fc07f01fc07f0p-1, 0x1.fe02a6b106789p-8, 0x1.fa11caa01fa12p-1, 0x1.7dc475f810a77p-7,
    0x1.f81f81f81f820p-1, 0x1.fc0a8b0fc03e4p-7, 0x1.f6310aca0dbb5p-1, 0x1.3cea44346a575p-6,
    0x1.f44659e4a4271p-1, 0x1.7b91b07d5b11bp-6, 0x1.f25f644230ab5p-1, 0x1.b9fc027af9198p-6,
    0x1.f07c1f07c1f08p-1, 0x1.f829b0e783300p-6, 0x1.ee9c7f8458e02p-1, 0x1.1b0d98923d980p-5,
    0x1.ecc07b301ecc0p-1, 0x1.39e87b9febd60p-5, 0x1.eae807aba01ebp-1, 0x1.58a5bafc8e4d5p-5,
    0x1.e9131abf0b767p-1, 0x1.77458f632dcfcp-5, 0x1.e741aa59750e4p-1, 0x1.95c830ec8e3ebp-5,
    0x1.e573ac901e574p-1, 0x1.b42dd711971bfp-5, 0x1.e3a9179dc1a73p-1, 0x1.d276b8adb0b52p-5,
    0x1.e1e1e1e1e1e1ep-1, 0x1.f0a30c01162a6p-5, 0x1.e01e01e01e01ep-1, 0x1.075983598e471p-4,
    0x1.de5d6e3f8868ap-1, 0x1.16536eea37ae1p-4, 0x1.dca01dca01dcap-1, 0x1.253f62f0a1417p-4,
    0x1.dae6076b981dbp-1, 0x1.341d7961bd1d1p-4, 0x1.d92f2231e7f8ap-1, 0x1.42edcbea646f0p-4,
    0x1.d77b654b82c34p-1, 0x1.51b073f06183fp-4, 0x1.d5cac807572b2p-1, 0x1.60658a93750c4p-4,
    0x1.d41d41d41d41dp-1, 0x1.6f0d28ae56b4cp-4, 0x1.d272ca3fc5b1ap-1, 0x1.7da766d7b12cdp-4,
    0x1.d0cb58f6ec074p-1, 0x1.8c345d6319b21p-4, 0x1.cf26e5c44bfc6p-1, 0x1.9ab42462033adp-4,
    0x1.cd85689039b0bp-1, 0x1.a926d3a4ad563p-4, 0x1.cbe6d9601cbe7p-1, 0x1.b78c82bb0eda1p-4,
    0x1.ca4b3055ee191p-1, 0x1.c5e548f5bc743p-4, 0x1.c8b265afb8a42p-1, 0x1.d4313d66cb35dp-4,
    0x1.c71c71c71c71cp-1, 0x1.e27076e2af2e6p-4, 0x1.c5894d10d4986p-1, 0x1.f0a30c01162a6p-4,
    0x1.c3f8f01c3f8f0p-1, 0x1.fec9131dbeabbp-4, 0x1.c26b5392ea01cp-1, 0x1.0671512ca596ep-3,
    0x1.c0e070381c0e0p-1, 0x1.0d77e7cd08e59p-3, 0x1.bf583ee868d8bp-1, 0x1.14785846742acp-3,
    0x1.bdd2b899406f7p-1, 0x1.1b72ad52f67a0p-3, 0x1.bc4fd65883e7bp-1, 0x1.2266f190a5acbp-3,
    0x1.bacf914c1bad0p-1, 0x1.29552f81ff523p-3, 0x1.b951e2b18ff23p-1, 0x1.303d718e47fd3p-3,
    0x1.b7d6c3dda338bp-1, 0x1.371fc201e8f74p-3, 0x1.b65e2e3beee05p-1, 0x1.3dfc2b0ecc62ap-3,
    0x1.b4e81b4e81b4fp-1, 0x1.44d2b6ccb7d1ep-3, 0x1.b37484ad806cep-1, 0x1.4ba36f39a55e5p-3,
    0x1.b2036406c80d9p-1, 0x1.526e5e3a1b438p-3, 0x1.b094b31d922a4p-1, 0x1.59338d9982086p-3,
    0x1.af286bca1af28p-1, 0x1.5ff3070a793d4p-3, 0x1.adbe87f94905ep-1, 0x1.66acd4272ad51p-3,
    0x1.ac5701ac5701bp-1, 0x1.6d60fe719d21dp-3, 0x1.aaf1d2f87ebfdp-1, 0x1.740f8f54037a5p-3,
    0x1.a98ef606a63bep-1, 0x1.7ab890210d909p-3, 0x1.a82e65130e159p-1, 0x1.815c0a14357ebp-3,
    0x1.a6d01a6d01a6dp-1, 0x1.87fa06520c911p-3, 0x1.a574107688a4ap-1, 0x1.8e928de886d41p-3,
    0x1.a41a41a41a41ap-1, 0x1.9525a9cf456b4p-3, 0x1.a2c2a87c51ca0p-1, 0x1.9bb362e7dfb83p-3,
    0x1.a16d3f97a4b02p-1, 0x1.a23bc1fe2b563p-3, 0x1.a01a01a01a01ap-1, 0x1.a8becfc882f19p-3,
    0x1.9ec8e951033d9p-1, 0x1.af3c94e80bff3p-3, 0x1.9d79f176b682dp-1, 0x1.b5b519e8fb5a4p-3,
    0x1.9c2d14ee4a102p-1, 0x1.bc286742d8cd6p-3, 0x1.9ae24ea5510dap-1, 0x1.c2968558c18c1p-3,
    0x1.999999999999ap-1, 0x1.c8ff7c79a9a22p-3, 0x1.9852f0d8ec0ffp-1, 0x1.cf6354e09c5dcp-3,
    0x1.970e4f80cb872p-1, 0x1.d5c216b4fbb91p-3, 0x1.95cbb0be377aep-1, 0x1.dc1bca0abec7dp-3,
    0x1.948b0fcd6e9e0p-1, 0x1.e27076e2af2e6p-3, 0x1.934c67f9b2ce6p-1, 0x1.e8c0252aa5a60p-3,
    0x1.920fb49d0e229p-1, 0x1.ef0adcbdc5936p-3, 0x1.90d4f120190d5p-1, 0x1.f550a564b7b37p-3,
    0x1.8f9c18f9c18fap-1, 0x1.fb9186d5e3e2bp-3, 0x1.8e6527af1373fp-1, 0x1.00e6c45ad501dp-2,
    0x1.8d3018d3018d3p-1, 0x1.0402594b4d041p-2, 0x1.8bfce8062ff3ap-1, 0x1.071b85fcd590dp-2,
    0x1.8acb90f6bf3aap-1, 0x1.0a324e27390e3p-2, 0x1.899c0f601899cp-1, 0x1.0d46b579ab74bp-2,
    0x1.886e5f0abb04ap-1, 0x1.1058bf9ae4ad5p-2, 0x1.87427bcc092b9p-1, 0x1.136870293a8b0p-2,
    0x1.8618618618618p-1, 0x1.1675cababa60ep-2, 0x1.84f00c2780614p-1, 0x1.1980d2dd4236fp-2,
    0x1.83c977ab2beddp-1, 0x1.1c898c16999fbp-2, 0x1.82a4a0182a4a0p-1, 0x1.1f8ff9e48a2f3p-2,
    0x1.8181818181818p-1, 0x1.22941fbcf7966p-2, 0x1.8060180601806p-1, 0x1.2596010df763ap-2,
    0x1.7f405fd017f40p-1, 0x1.2895a13de86a3p-2, 0x1.7e225515a4f1dp-1, 0x1.2b9303ab89d25p-2,
    0x1.7d05f417d05f4p-1, 0x1.2e8e2bae11d31p-2, 0x1.7beb3922e017cp-1, 0x1.31871c9544185p-2,
    0x1.7ad2208e0ecc3p-1, 0x1.347dd9a987d55p-2, 0x1.79baa6bb6398bp-1, 0x1.3772662bfd85bp-2,
    0x1.78a4c8178a4c8p-1, 0x1.3a64c556945eap-2, 0x1.77908119ac60dp-1, 0x1.3d54fa5c1f710p-2,
    0x1.767dce434a9b1p-1, 0x1.404308686a7e4p-2, 0x1.756cac201756dp-1, 0x1.432ef2a04e814p-2,
    0x1.745d1745d1746p-1, 0x1.4618bc21c5ec2p-2, 0x1.734f0c541fe8dp-1, 0x1.49006804009d1p-2,
    0x1.724287f46debcp-1, 0x1.4be5f957778a1p-2, 0x1.713786d9c7c09p-1, 0x1.4ec973260026ap-2,
    0x1.702e05c0b8170p-1, 0x1.51aad872df82dp-2, 0x1.6f26016f26017p-1, 0x1.548a2c3add263p-2,
    0x1.6e1f76b4337c7p-1, 0x1.5767717455a6cp-2, 0x1.6d1a62681c861p-1, 0x1.5a42ab0f4cfe2p-2,
    0x1.6c16c16c16c17p-1, 0x1.5d1bdbf5809cap-2, 0x1.6b1490aa31a3dp-1, 0x1.5ff3070a793d4p-2,
    0x1.6a13cd1537290p-1, 0x1.62c82f2b9c795p-2, 0x1.691473a88d0c0p-1, 0x1.659b57303e1f3p-2,
    0x1.6816816816817p-1, 0x1.686c81e9b14afp-2, 0x1.6719f3601671ap-1, 0x1.6b3bb2235943ep-2,
    0x1.661ec6a5122f9p-1, 0x1.6e08eaa2ba1e4p-2, 0x1.6524f853b4aa3p-1, 0x1.70d42e2789236p-2,
    0x1.642c8590b2164p-1, 0x1.739d7f6bbd007p-2, 0x1.63356b88ac0dep-1, 0x1.7664e1239dbcfp-2,
    0x1.623fa77016240p-1, 0x1.792a55fdd47a2p-2, 0x1.614b36831ae94p-1, 0x1.7bede0a37afc0p-2,
    0x1.6058160581606p-1, 0x1.7eaf83b82afc3p-2, 0x1.5f66434292dfcp-1, 0x1.816f41da0d496p-2,
    0x1.5e75bb8d015e7p-1, 0x1.842d1da1e8b17p-2, 0x1.5d867c3ece2a5p-1, 0x1.86e919a330ba0p-2,
    0x1.5c9882b931057p-1, 0x1.89a3386c1425bp-2, 0x1.5babcc647fa91p-1, 0x1.8c5b7c858b48bp-2,
    0x1.5ac056b015ac0p-1, 0x1.8f11e873662c7p-2, 0x1.59d61f123ccaap-1, 0x1.91c67eb45a83ep-2,
    0x1.58ed2308158edp-1, 0x1.947941c2116fbp-2, 0x1.5805601580560p-1, 0x1.972a341135158p-2,
    0x1.571ed3c506b3ap-1, 0x1.99d958117e08bp-2, 0x1.56397ba7c52e2p-1, 0x1.9c86b02dc0863p-2,
    0x1.5555555555555p-1, 0x1.9f323ecbf984cp-2, 0x1.54725e6bb82fep-1, 0x1.a1dc064d5b995p-2,
    0x1.5390948f40febp-1, 0x1.a484090e5bb0ap-2, 0x1.52aff56a8054bp-1, 0x1.a72a4966bd9eap-2,
    0x1.51d07eae2f815p-1, 0x1.a9cec9a9a084ap-2, 0x1.50f22e111c4c5p-1, 0x1.ac718c258b0e4p-2,
    0x1.5015015015015p-1, 0x1.af1293247786bp-2, 0x1.4f38f62dd4c9bp-1, 0x1.b1b1e0ebdfc5bp-2,
    0x1.4e5e0a72f0539p-1, 0x1.b44f77bcc8f63p-2, 0x1.4d843bedc2c4cp-1, 0x1.b6eb59d3cf35ep-2,
    0x1.4cab88725af6ep-1, 0x1.b9858969310fbp-2, 0x1.4bd3edda68fe1p-1, 0x1.bc1e08b0dad0ap-2,
    0x1.4afd6a052bf5bp-1, 0x1.beb4d9da71b7cp-2, 0x1.4a27fad76014ap-1, 0x1.c149ff115f027p-2,
    0x1.49539e3b2d067p-1, 0x1.c3dd7a7cdad4dp-2, 0x1.4880522014880p-1, 0x1.c66f4e3ff6ff8p-2,
    0x1.47ae147ae147bp-1, 0x1.c8ff7c79a9a22p-2, 0x1.46dce34596066p-1, 0x1.cb8e0744d7acap-2,
    0x1.460cbc7f5cf9ap-1, 0x1.ce1af0b85f3ebp-2, 0x1.453d9e2c776cap-1, 0x1.d0a63ae721e64p-2,
    0x1.446f86562d9fbp-1, 0x1.d32fe7e00ebd5p-2, 0x1.43a2730abee4dp-1, 0x1.d5b7f9ae2c684p-2,
    0x1.42d6625d51f87p-1, 0x1.d83e7258a2f3ep-2, 0x1.420b5265e5951p-1, 0x1.dac353e2c5954p-2,
    0x1.4141414141414p-1, 0x1.dd46a04c1c4a1p-2, 0x1.40782d10e6566p-1, 0x1.dfc859906d5b5p-2,
    0x1.3fb013fb013fbp-1, 0x1.e24881a7c6c26p-2, 0x1.3ee8f42a5af07p-1, 0x1.e4c71a8687704p-2,
    0x1.3e22cbce4a902p-1, 0x1.e744261d68788p-2, 0x1.3d5d991aa75c6p-1, 0x1.e9bfa659861f5p-2,
    0x1.3c995a47babe7p-1, 0x1.ec399d2468cc0p-2, 0x1.3bd60d9232955p-1, 0x1.eeb20c640ddf4p-2,
    0x1.3b13b13b13b14p-1, 0x1.f128f5faf06edp-2, 0x1.3a524387ac822p-1, 0x1.f39e5bc811e5cp-2,
    0x1.3991c2c187f63p-1, 0x1.f6123fa7028acp-2, 0x1.38d22d366088ep-1, 0x1.f884a36fe9ec2p-2,
    0x1.3813813813814p-1, 0x1.faf588f78f31fp-2, 0x1.3755bd1c945eep-1, 0x1.fd64f20f61572p-2,
    0x1.3698df3de0748p-1, 0x1.ffd2e0857f498p-2, 0x1.35dce5f9f2af8p-1, 0x1.011fab125ff8ap-1,
    0x1.3521cfb2b78c1p-1, 0x1.02552a5a5d0ffp-1, 0x1.34679ace01346p-1, 0x1.0389eefce633bp-1,
    0x1.33ae45b57bcb2p-1, 0x1.04bdf9da926d2p-1, 0x1.32f5ced6a1dfap-1, 0x1.05f14bd26459cp-1,
    0x1.323e34a2b10bfp-1, 0x1.0723e5c1cdf40p-1, 0x1.3187758e9ebb6p-1, 0x1.0855c884b450ep-1,
    0x1.30d190130d190p-1, 0x1.0986f4f573521p-1, 0x1.301c82ac40260p-1, 0x1.0ab76bece14d2p-1,
    0x1.2f684bda12f68p-1, 0x1.0be72e4252a83p-1, 0x1.2eb4ea1fed14bp-1, 0x1.0d163ccb9d6b8p-1,
    0x1.2e025c04b8097p-1, 0x1.0e44985d1cc8cp-1, 0x1.2d50a012d50a0p-1, 0x1.0f7241c9b497dp-1,
    0x1.2c9fb4d812ca0p-1, 0x1.109f39e2d4c97p-1, 0x1.2bef98e5a3711p-1, 0x1.11cb81787ccf8p-1,
    0x1.2b404ad012b40p-1, 0x1.12f719593efbcp-1, 0x1.2a91c92f3c105p-1, 0x1.1422025243d45p-1,
    0x1.29e4129e4129ep-1, 0x1.154c3d2f4d5eap-1, 0x1.293725bb804a5p-1, 0x1.1675cababa60ep-1,
    0x1.288b01288b013p-1, 0x1.179eabbd899a1p-1, 0x1.27dfa38a1ce4dp-1, 0x1.18c6e0ff5cf06p-1,
    0x1.27350b8812735p-1, 0x1.19ee6b467c96fp-1, 0x1.268b37cd60127p-1, 0x1.1b154b57da29fp-1,
    0x1.25e22708092f1p-1, 0x1.1c3b81f713c25p-1, 0x1.2539d7e9177b2p-1, 0x1.1d610fe677003p-1,
    0x1.2492492492492p-1, 0x1.1e85f5e7040d0p-1, 0x1.23eb79717605bp-1, 0x1.1faa34b87094cp-1,
    0x1.23456789abcdfp-1, 0x1.20cdcd192ab6ep-1, 0x1.22a0122a0122ap-1, 0x1.21f0bfc65beecp-1,
    0x1.21fb78121fb78p-1, 0x1.23130d7bebf43p-1, 0x1.21579804855e6p-1, 0x1.2434b6f483934p-1,
    0x1.20b470c67c0d9p-1, 0x1.2555bce98f7cbp-1, 0x1.2012012012012p-1, 0x1.26762013430e0p-1,
    0x1.1f7047dc11f70p-1, 0x1.2795e1289b11bp-1, 0x1.1ecf43c7fb84cp-1, 0x1.28b500df60783p-1,
    0x1.1e2ef3b3fb874p-1, 0x1.29d37fec2b08bp-1, 0x1.1d8f5672e4abdp-1, 0x1.2af15f02640adp-1,
    0x1.1cf06ada2811dp-1, 0x1.2c0e9ed448e8cp-1, 0x1.1c522fc1ce059p-1, 0x1.2d2b4012edc9ep-1,
    0x1.1bb4a4046ed29p-1, 0x1.2e47436e40268p-1, 0x1.1b17c67f2bae3p-1, 0x1.2f62a99509546p-1,
    0x1.1a7b9611a7b96p-1, 0x1.307d7334f10bep-1, 0x1.19e0119e0119ep-1, 0x1.3197a0fa7fe6ap-1,
    0x1.19453808ca29cp-1, 0x1.32b1339121d71p-1, 0x1.18ab083902bdbp-1, 0x1.33ca2ba328995p-1,
    0x1.1811811811812p-1, 0x1.34e289d9ce1d3p-1, 0x1.1778a191bd684p-1, 0x1.35fa4edd36ea0p-1,
    0x1.16e0689427379p-1, 0x1.37117b54747b6p-1, 0x1.1648d50fc3201p-1, 0x1.38280fe58797fp-1,
    0x1.15b1e5f75270dp-1, 0x1.393e0d3562a1ap-1, 0x1.151b9a3fdd5c9p-1, 0x1.3a5373e7ebdfap-1,
    0x1.1485f0e0acd3bp-1, 0x1.3b68449fffc23p-1, 0x1.13f0e8d344724p-1, 0x1.3c7c7fff73206p-1,
    0x1.135c81135c811p-1, 0x1.3d9026a7156fbp-1, 0x1.12c8b89edc0acp-1, 0x1.3ea33936b2f5cp-1,
    0x1.12358e75d3033p-1, 0x1.3fb5b84d16f42p-1, 0x1.11a3019a74826p-1, 0x1.40c7a4880dce9p-1,
    0x1.1111111111111p-1, 0x1.41d8fe84672aep-1, 0x1.107fbbe011080p-1, 0x1.42e9c6ddf80bfp-1,
    0x1.0fef010fef011p-1, 0x1.43f9fe2f9ce67p-1, 0x1.0f5edfab325a2p-1, 0x1.4509a5133bb0ap-1,
    0x1.0ecf56be69c90p-1, 0x1.4618bc21c5ec2p-1, 0x1.0e40655826011p-1, 0x1.472743f33aaadp-1,
    0x1.0db20a88f4696p-1, 0x1.48353d1ea88dfp-1, 0x1.0d24456359e3ap-1, 0x1.4942a83a2fc07p-1,
    0x1.0c9714fbcda3bp-1, 0x1.4a4f85db03ebbp-1, 0x1.0c0a7868b4171p-1, 0x1.4b5bd6956e274p-1,
    0x1.0b7e6ec259dc8p-1, 0x1.4c679afccee3ap-1, 0x1.0af2f722eecb5p-1, 0x1.4d72d3a39fd00p-1,
    0x1.0a6810a6810a7p-1, 0x1.4e7d811b75bb1p-1, 0x1.09ddba6af8360p-1, 0x1.4f87a3f5026e9p-1,
    0x1.0953f39010954p-1, 0x1.50913cc01686bp-1, 0x1.08cabb37565e2p-1, 0x1.519a4c0ba3446p-1,
    0x1.0842108421084p-1, 0x1.52a2d265bc5abp-1, 0x1.07b9f29b8eae2p-1, 0x1.53aad05b99b7dp-1,
    0x1.073260a47f7c6p-1, 0x1.54b2467999498p-1, 0x1.06ab59c7912fbp-1, 0x1.55b9354b40bcdp-1,
    0x1.0624dd2f1a9fcp-1, 0x1.56bf9d5b3f399p-1, 0x1.059eea0727586p-1, 0x1.57c57f336f191p-1,
    0x1.05197f7d73404p-1, 0x1.58cadb5cd7989p-1, 0x1.04949cc1664c5p-1, 0x1.59cfb25fae87ep-1,
    0x1.0410410410410p-1, 0x1.5ad404c359f2dp-1, 0x1.038c6b78247fcp-1, 0x1.5bd7d30e71c73p-1,
    0x1.03091b51f5e1ap-1, 0x1.5cdb1dc6c1765p-1, 0x1.02864fc7729e9p-1, 0x1.5ddde57149923p-1,
    0x1.0204081020408p-1, 0x1.5ee02a9241675p-1, 0x1.0182436517a37p-1, 0x1.5fe1edad18919p-1,
    0x1.0101010101010p-1, 0x1.60e32f44788d9p-1, 0x1.0080402010080p-1, 0x1.61e3efda46467p-1,
};

// ln x by table-driven reduction (P. T. P. Tang, Table-driven
// implementation of the logarithm function in IEEE floating-point
// arithmetic, ACM TOMS 16, 1990): x = 2^e m, m in [1, 2), F = 1 + j/256 the
// mantissa cut to 8 bits, r = (m - F)/F in [0, 2^-8) (m - F exact),
// ln x = e ln 2 + ln F + ln(1 + r), ln(1 + r) by its degree-6 Taylor
// polynomial (truncation below r^7/7 < 2^-58), e ln 2 carried in two parts.
// Within about one ulp of the exact value for x >= 2 and within 1e-15
// absolute below; NaN for x <= 0 or NaN (subnormal and infinite x are not
// handled: the temperatures it serves are positive and normal).  `ltab` holds kLogTab
// (in LDS in the chemistry launch, the constant table elsewhere).
__device__ __forceinline__ double log_tab(double x, const double *ltab)
{
    constexpr double kLn2 = 0x1.62e42fefa39efp-1;     // ln 2, nearest double
    constexpr double kLn2_lo = 0x1.abc9e3b39803fp-56;  // ln 2 - kLn2
    const unsigned hi = (unsigned)__double2hiint(x);
    const int lo = __double2loint(x);
    const int j = (int)((hi >> 12) & 0xffu);
    const double m = __hiloint2double((int)((hi & 0x000fffffu) | 0x3ff00000u), lo);
    const double F = __hiloint2double((int)((hi & 0x000ff000u) | 0x3ff00000u), 0);
    const double r = (m - F) * ltab[2 * j];
    const double lnF = ltab[2 * j + 1];
    double p = fma(r, -1.0 / 6.0, 0.2);
    p = fma(r, p, -0.25);
    p = fma(r, p, 1.0 / 3.0);
    p = fma(r, p, -0.5);
    const double l1p = fma(r * r, p, r);
    const double e = (double)((int)(hi >> 20) - 1023);
    const double res = fma(e, kLn2, lnF) + fma(e, kLn2_lo, l1p);
    return x > 0.0 ? res : __builtin_nan("");
}

// exp(x) from xs = x 256/ln 2 (the caller folds the scale into the
// constants it forms xs from): n = rint(xs), s = xs - n (exact, |s| <= 1/2),
// exp(x) = 2^(n/256) exp(s ln2/256), exp(s ln2/256) - 1 by the degree-4
// Taylor polynomial in s with the coefficients (ln2/256)^i / i!.  The
// argument needs no two-part reduction (s is exact); its own rounding, one
// part in 2^53 of xs, is the same relative error the unscaled x carries.
// xs is clamped below (exp underflows to 0); the arguments it serves stay
// far below the overflow.  CLAMP = false leaves the clamp out for finite
// arguments: below it the result is 0 all the same (the exponent the table
// entry is scaled by is then below -1445; a saturated conversion keeps it
// there), but -inf and NaN give NaN.
template <bool CLAMP = true>
__device__ __forceinline__ double exp_scaled_tab(double xs, const double *tab)
{
    constexpr double k1 = 0x1.62e42fefa39efp-9;   // ln 2 / 256
    constexpr double k2 = 0x1.ebfbdff82c58fp-19;  // k1^2 / 2
    constexpr double k3 = 0x1.c6b08d704a0c0p-29;  // k1^3 / 6
    constexpr double k4 = 0x1.3b2ab6fba4e77p-39;  // k1^4 / 24
    if constexpr (CLAMP) xs = fmax(xs, -370000.0);  // x below -1000
    const double n = __builtin_rint(xs);
    const double sr = xs - n;
    double p = fma(sr, k4, k3);
    p = fma(sr, p, k2);
    p = fma(sr, p, k1);
    p *= sr;
    const int ni = (int)n;
    const double t = tab[ni & (kExpTabN - 1)];
    return __builtin_ldexp(fma(t, p, t), ni >> 8);
}

}  // namespace lbfd
